// Factor leverage scores, whitened factor rows and integer sampling tables.
//
// Alg. 3 first step: the statistical leverage score of row i of A(n) is
// l_i = a_i (A^T A)^+ a_i^T (Sec. 2, ridge score at lambda = 0).  With the
// FP64 Cholesky factor C_n = A^T A = L L^T this is l_i = ||L^{-1} a_i^T||^2,
// and q_i = L^{-1} a_i^T is row i of the whitened factor Q_n = A L^{-T},
// whose columns are orthonormal.  The per-mode CDF of the proof of Thm 4.2
// is kept as integers: w_i = ceil(max(l_i, 0) 2^Q) and its inclusive prefix sum.
//
// Three launches: one workgroup per mode forms C_n, L, L^{-1} and P (O(I_n R_n^2)
// work, latency bound); a rows kernel with many workgroups stages blocks of
// factor rows in LDS and multiplies them by L^{-T} (the same kernel forms
// A(n) V_n for the exact update); one workgroup per mode then scans the
// integer weights.
#include "tk_internal.h"

namespace tk {
namespace {

struct FactorPtrs {
  const void* p[kMaxOrder];
};

template <class T>
__device__ inline double ld(const T* a, int64_t i) {
  return static_cast<double>(a[i]);
}

// buf[e] = src[e] for e < n (FP64), NV loads in flight per thread (indices
// clamped into range so that the loads issue together)
template <int NV, class T>
__device__ inline void stage_rows(const T* src, int64_t n, double* buf) {
  for (int64_t e0 = threadIdx.x; e0 < n; e0 += NV * kBlock) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int64_t e = e0 + k * kBlock;
      v[k] = ld(src, e < n ? e : n - 1);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int64_t e = e0 + k * kBlock;
      if (e < n) buf[e] = v[k];
    }
  }
}

// LDS budget: two R x R FP64 buffers (64 KB at R = 64).
template <class T>
__global__ __launch_bounds__(kBlock) void leverage_kernel(Geom g, FactorPtrs fp, double* Lg,
                                                          double* Linvg, double* Pg,
                                                          int32_t* status) {
  // row chunks of A across both halves; then C and L (lower, in place) in the
  // first, L^{-1} in the second
  __shared__ double buf2[2 * kMaxRank * kMaxRank];
  double* bufC = buf2;
  double* bufA = buf2 + kMaxRank * kMaxRank;
  __shared__ int bad;
  __shared__ double thr;

  const int n = blockIdx.x;
  const int tid = threadIdx.x;
  const int R = g.ranks[n];
  const int64_t I = g.dims[n];
  const T* A = static_cast<const T*>(fp.p[n]);
  const int E = R * (R + 1) / 2;

  // ---- C = A^T A (lower triangle, FP64), rows streamed through LDS.  With
  // E <= 256 entries, thread (e, grp) takes entry e over the rows i = grp mod
  // G (G = 256 / E groups) and the groups are added in order at the end;
  // otherwise each thread takes entries tid, tid + 256, ... over all rows.
  constexpr int kMaxPer = (kMaxRank * (kMaxRank + 1) / 2 + kBlock - 1) / kBlock;
  const bool grouped = E <= kBlock;
  const int G = grouped ? kBlock / E : 1;
  const int grp = grouped ? tid / E : 0;
  const int e0 = grouped ? tid % E : tid;
  double acc[kMaxPer];
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) acc[k] = 0.0;
  const int64_t chunk_rows = (2 * kMaxRank * kMaxRank) / R;
  for (int64_t r0 = 0; r0 < I; r0 += chunk_rows) {
    const int64_t rows = (I - r0 < chunk_rows) ? (I - r0) : chunk_rows;
    __syncthreads();
    stage_rows<32>(A + r0 * R, rows * R, buf2);  // one round trip for a full chunk
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
      const int e = e0 + k * kBlock;
      if (e < E && grp < G && (k == 0 || !grouped)) {
        // e -> (a, b), b <= a
        int a = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= e) ++a;
        while (a * (a + 1) / 2 > e) --a;
        const int b = e - a * (a + 1) / 2;
        // four independent chains over the rows, added in a fixed order
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t i = grp;
        for (; i + 3 * G < rows; i += 4 * G) {
          s0 = fma(buf2[i * R + a], buf2[i * R + b], s0);
          s1 = fma(buf2[(i + G) * R + a], buf2[(i + G) * R + b], s1);
          s2 = fma(buf2[(i + 2 * G) * R + a], buf2[(i + 2 * G) * R + b], s2);
          s3 = fma(buf2[(i + 3 * G) * R + a], buf2[(i + 3 * G) * R + b], s3);
        }
        for (; i < rows; i += G) s0 = fma(buf2[i * R + a], buf2[i * R + b], s0);
        acc[k] += (s0 + s1) + (s2 + s3);
      }
    }
  }
  __syncthreads();
  if (grouped) {
    // groups in order: bufA[grp][e] -> thread e
    bufA[tid] = (grp < G) ? acc[0] : 0.0;
    __syncthreads();
    if (tid < E) {
      double v = 0.0;
      for (int k = 0; k < G; ++k) v += bufA[k * E + tid];
      acc[0] = v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) {
    const int e = tid + k * kBlock;
    if (e < E && (k == 0 || !grouped)) {
      int a = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      while (a * (a + 1) / 2 > e) --a;
      const int b = e - a * (a + 1) / 2;
      bufC[a * R + b] = acc[k];
      bufC[b * R + a] = acc[k];
    }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int a = 0; a < R; ++a) mx = fmax(mx, bufC[a * R + a]);
    thr = static_cast<double>(R) * 0x1p-52 * mx;
    if (!(mx > 0.0)) bad = 1;
  }
  __syncthreads();

  // ---- Cholesky C = L L^T (right-looking, one column per step)
  for (int j = 0; j < R; ++j) {
    if (tid == 0) {
      double piv = bufC[j * R + j];
      if (!(piv > thr)) {
        bad = 1;
        piv = 1.0;
      }
      bufC[j * R + j] = sqrt(piv);
    }
    __syncthreads();
    const double ljj = bufC[j * R + j];
    for (int i = j + 1 + tid; i < R; i += kBlock) bufC[i * R + j] /= ljj;
    __syncthreads();
    const int m = R - j - 1;  // trailing size
    for (int e = tid; e < m * m; e += kBlock) {
      const int i = j + 1 + e / m;
      const int c = j + 1 + e % m;
      if (c <= i) bufC[i * R + c] = fma(-bufC[i * R + j], bufC[c * R + j], bufC[i * R + c]);
    }
    __syncthreads();
  }

  // ---- L^{-1} by columns (thread c solves L x = e_c)
  if (tid < R) {
    const int c = tid;
    for (int i = 0; i < R; ++i) bufA[i * R + c] = 0.0;
    bufA[c * R + c] = 1.0 / bufC[c * R + c];
    for (int i = c + 1; i < R; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s = fma(bufC[i * R + k], bufA[k * R + c], s);
      bufA[i * R + c] = -s / bufC[i * R + i];
    }
  }
  __syncthreads();
  double* L = Lg + g.roff[n];
  double* Li = Linvg + g.roff[n];
  double* P = Pg + g.roff[n];
  for (int e = tid; e < R * R; e += kBlock) {
    const int a = e / R, b = e % R;
    L[e] = (b <= a) ? bufC[e] : 0.0;
    Li[e] = (b <= a) ? bufA[e] : 0.0;
    // P = (L^T L)^{-1} = L^{-1} L^{-T}
    double s = 0.0;
    const int kmax = a < b ? a : b;
    for (int k = 0; k <= kmax; ++k) s = fma(bufA[a * R + k], bufA[b * R + k], s);
    P[e] = s;
  }

  if (tid == 0 && bad) atomicMax(status, static_cast<int32_t>(TK_E_RANK_DEFICIENT));
}

// Rows times a per-mode R x R matrix: out[i][c] = sum_k A(n)[i][k] M[k][c], with
// M row major at Mg + roff[n] (trans = 0) or M[k][c] = Mg[roff[n] + c R + k]
// (trans = 1).  kModeRows rows per workgroup, staged in LDS with a padded
// stride; workgroups walk the modes in order.  With `weights`, also the row
// score l_i = ||out[i]||^2 and the integer weight ceil(max(l_i, 0) 2^Q).
constexpr int kModeRows = 16;

__host__ __device__ inline int64_t mode_row_blocks(int64_t I) {
  return (I + kModeRows - 1) / kModeRows;
}

template <class T>
__global__ __launch_bounds__(kBlock) void mode_rows_kernel(Geom g, FactorPtrs fp, const double* Mg,
                                                           int trans, double* out64, float* out32,
                                                           double* scores, uint64_t* weights,
                                                           double qscale) {
  __shared__ double Ms[kMaxRank * kMaxRank];
  __shared__ double As[kModeRows * (kMaxRank + 1)];
  __shared__ double Ss[kModeRows * (kMaxRank + 1)];
  const int tid = threadIdx.x;
  int n = 0;
  int64_t b = blockIdx.x;
  for (; n < g.order; ++n) {
    const int64_t nb = mode_row_blocks(g.dims[n]);
    if (b < nb) break;
    b -= nb;
  }
  if (n >= g.order) return;  // uniform over the workgroup
  const int R = g.ranks[n];
  const int Rp = R + 1;
  const int64_t r0 = b * kModeRows;
  const int rows = static_cast<int>(g.dims[n] - r0 < kModeRows ? g.dims[n] - r0 : kModeRows);
  const T* A = static_cast<const T*>(fp.p[n]) + r0 * R;
  const double* M = Mg + g.roff[n];
  for (int e = tid; e < R * R; e += kBlock) {
    const int u = e / R, v = e % R;
    Ms[trans ? v * R + u : e] = M[e];
  }
  for (int e = tid; e < rows * R; e += kBlock) As[(e / R) * Rp + e % R] = ld(A, e);
  __syncthreads();
  double* o64 = out64 + g.qoff[n] + r0 * R;
  float* o32 = out32 ? out32 + g.qoff[n] + r0 * R : nullptr;
  for (int e = tid; e < rows * R; e += kBlock) {
    const int i = e / R, c = e % R;
    double s = 0.0;
    for (int k = 0; k < R; ++k) s = fma(As[i * Rp + k], Ms[k * R + c], s);
    o64[e] = s;
    if (o32) o32[e] = static_cast<float>(s);
    Ss[i * Rp + c] = s * s;
  }
  if (!weights) return;
  __syncthreads();
  if (tid < rows) {
    double l = 0.0;
    for (int c = 0; c < R; ++c) l += Ss[tid * Rp + c];
    if (scores) scores[g.off[n] + r0 + tid] = l;
    const double lc = l > 0.0 ? l : 0.0;
    weights[g.off[n] + r0 + tid] = static_cast<uint64_t>(ceil(lc * qscale));
  }
}

// Inclusive prefix sum of each mode's integer weights (order independent:
// integer adds), one workgroup per mode: per 256-entry block a wave scan by
// shuffles, then the wave totals.
__global__ __launch_bounds__(kBlock) void weight_scan_kernel(Geom g, uint64_t* cdf) {
  __shared__ uint64_t wsum[kBlock / 64];
  const int n = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t I = g.dims[n];
  uint64_t* cd = cdf + g.off[n];
  uint64_t carry = 0;
  for (int64_t base = 0; base < I; base += kBlock) {
    const int64_t i = base + tid;
    uint64_t v = (i < I) ? cd[i] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    uint64_t before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < I) cd[i] = v + before;
    for (int w = 0; w < kBlock / 64; ++w) carry += wsum[w];
    __syncthreads();
  }
}

}  // namespace

namespace {

// In-place inclusive prefix sum of len uint64 entries by one workgroup of
// kBlock threads (integer adds: any order gives the same table).
__device__ void block_scan_u64(uint64_t* cd, int64_t len, uint64_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t carry = 0;
  for (int64_t base = 0; base < len; base += kBlock) {
    const int64_t i = base + tid;
    uint64_t v = (i < len) ? cd[i] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    uint64_t before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < len) cd[i] = v + before;
    for (int w = 0; w < kBlock / 64; ++w) carry += wsum[w];
    __syncthreads();
  }
}

// Ridge-score mixture of K (Sec. 2 SVD form applied to K's SVD): with
// C_n = V_n Lambda_n V_n^T and W_n = A(n) V_n, column c of U_n is
// W_n[:, c] / sqrt(Lambda_n[c]).  Workgroup j builds the table of global
// column j (mode n, column c) at qoff[n] + c I_n: weights
// ceil(W[i][c]^2 / Lambda[c] 2^Q), then their inclusive prefix sums.  A
// numerically zero eigenvalue (<= R 2^-52 max) gets an all-zero column.
__global__ __launch_bounds__(kBlock) void ridge_col_kernel(Geom g, const double* __restrict__ lamm,
                                                           const double* __restrict__ W,
                                                           uint64_t* __restrict__ ccdf,
                                                           double qscale) {
  __shared__ uint64_t wsum[kBlock / 64];
  int n = 0, c = blockIdx.x;
  while (c >= g.ranks[n]) c -= g.ranks[n++];
  const int R = g.ranks[n];
  const int64_t I = g.dims[n];
  double mx = 0.0;
  for (int a = 0; a < R; ++a) mx = fmax(mx, lamm[n * kMaxRank + a]);
  const double lc = lamm[n * kMaxRank + c];
  const bool zero = !(lc > static_cast<double>(R) * 0x1p-52 * mx);
  uint64_t* cd = ccdf + g.qoff[n] + static_cast<int64_t>(c) * I;
  const double* w = W + g.qoff[n] + c;
  for (int64_t i = threadIdx.x; i < I; i += kBlock) {
    const double v = w[i * R];
    const double u2 = zero ? 0.0 : (v * v) / lc;
    cd[i] = static_cast<uint64_t>(ceil(u2 * qscale));
  }
  __syncthreads();
  block_scan_u64(cd, I, wsum);
}

// Tuple table: pi_t = prod_n Lambda_n[t_n] / (prod + lambda) (the product in
// mode order; 0 when it is not positive), weights ceil(pi_t 2^Q), their
// inclusive prefix sums, and d_eff = sum_t pi_t (per-thread sums over
// t = tid + k kBlock, then added in thread order).
__global__ __launch_bounds__(kBlock) void ridge_tuple_kernel(Geom g, const double* __restrict__ lamm,
                                                             double lambda,
                                                             uint64_t* __restrict__ tcdf,
                                                             double* __restrict__ deff,
                                                             double qscale) {
  __shared__ uint64_t wsum[kBlock / 64];
  __shared__ double part[kBlock];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int64_t t = tid; t < g.d; t += kBlock) {
    int64_t rem = t;
    int dig[kMaxOrder];
    for (int n = g.order - 1; n >= 0; --n) {
      dig[n] = static_cast<int>(rem % g.ranks[n]);
      rem /= g.ranks[n];
    }
    double prod = 1.0;
    for (int n = 0; n < g.order; ++n) prod = prod * lamm[n * kMaxRank + dig[n]];
    const double pi = prod > 0.0 ? prod / (prod + lambda) : 0.0;
    acc += pi;
    tcdf[t] = static_cast<uint64_t>(ceil(pi * qscale));
  }
  part[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int k = 0; k < kBlock; ++k) sum += part[k];
    *deff = sum;
  }
  block_scan_u64(tcdf, g.d, wsum);
}

// Rows of the augmented whitened tables: one thread per table entry of ga.
__global__ __launch_bounds__(kBlock) void aug_tables_kernel(Geom g, Geom ga,
                                                            const double* __restrict__ Q64,
                                                            const double* __restrict__ Linv,
                                                            double sqrt_lambda,
                                                            double* __restrict__ Q64a) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= ga.total_q) return;
  int n = 0;
  while (n + 1 < ga.order && e >= ga.qoff[n + 1]) ++n;
  const int R = ga.ranks[n];
  const int64_t i = (e - ga.qoff[n]) / R;
  const int r = static_cast<int>((e - ga.qoff[n]) % R);
  double v;
  if (i < g.dims[n]) {
    v = Q64[g.qoff[n] + i * R + r];
  } else {
    // ridge row k: entry r of L_n^{-1} e_k (L_n^{-1} row-major at roff)
    const int64_t k = i - g.dims[n];
    v = Linv[g.roff[n] + static_cast<int64_t>(r) * R + k];
    if (n == 0) v *= sqrt_lambda;
  }
  Q64a[e] = v;
}

}  // namespace

void launch_ridge_tables(const Geom& g, const double* lamm, const double* W, double lambda,
                         uint64_t* tcdf, uint64_t* ccdf, double* deff, hipStream_t st, int qbits) {
  const double qscale = ldexp(1.0, qbits);
  hipLaunchKernelGGL(ridge_col_kernel, dim3(g.sum_r), dim3(kBlock), 0, st, g, lamm, W, ccdf,
                     qscale);
  hipLaunchKernelGGL(ridge_tuple_kernel, dim3(1), dim3(kBlock), 0, st, g, lamm, lambda, tcdf, deff,
                     qscale);
}

void launch_aug_tables(const Geom& g, const Geom& ga, const double* Q64, const double* Linv,
                       double lambda, double* Q64a, hipStream_t st) {
  hipLaunchKernelGGL(aug_tables_kernel, dim3(static_cast<unsigned>(cdiv(ga.total_q, kBlock))),
                     dim3(kBlock), 0, st, g, ga, Q64, Linv, sqrt(lambda), Q64a);
}

void launch_leverage(const Geom& g, const void* const* factors, tk_dtype dt, double* scores,
                     uint64_t* cdf, double* L, double* Linv, double* P, double* Q64, float* Q32,
                     int32_t* status, hipStream_t st, int qbits) {
  FactorPtrs fp;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  if (dt == TK_F64)
    hipLaunchKernelGGL(leverage_kernel<double>, dim3(g.order), dim3(kBlock), 0, st, g, fp, L, Linv,
                       P, status);
  else
    hipLaunchKernelGGL(leverage_kernel<float>, dim3(g.order), dim3(kBlock), 0, st, g, fp, L, Linv,
                       P, status);
  launch_mode_rows(g, factors, dt, Linv, 1, Q64, Q32, scores, cdf, st, qbits);
  hipLaunchKernelGGL(weight_scan_kernel, dim3(g.order), dim3(kBlock), 0, st, g, cdf);
}

void launch_mode_rows(const Geom& g, const void* const* factors, tk_dtype dt, const double* M,
                      int trans, double* out64, float* out32, double* scores, uint64_t* weights,
                      hipStream_t st, int qbits) {
  const double qscale = ldexp(1.0, qbits);
  FactorPtrs fp;
  int64_t blocks = 0;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  for (int n = 0; n < g.order; ++n) blocks += mode_row_blocks(g.dims[n]);
  if (blocks == 0) return;
  if (dt == TK_F64)
    hipLaunchKernelGGL(mode_rows_kernel<double>, dim3(blocks), dim3(kBlock), 0, st, g, fp, M,
                       trans, out64, out32, scores, weights, qscale);
  else
    hipLaunchKernelGGL(mode_rows_kernel<float>, dim3(blocks), dim3(kBlock), 0, st, g, fp, M, trans,
                       out64, out32, scores, weights, qscale);
}

}  // namespace tk
