// Factor leverage scores, whitened factor rows and integer sampling tables.
//
// Alg. 3 first step: the statistical leverage score of row i of A(n) is
// l_i = a_i (A^T A)^+ a_i^T (Sec. 2, ridge score at lambda = 0).  With the
// FP64 Cholesky factor C_n = A^T A = L L^T this is l_i = ||L^{-1} a_i^T||^2,
// and q_i = L^{-1} a_i^T is row i of the whitened factor Q_n = A L^{-T},
// whose columns are orthonormal.  The per-mode CDF of the proof of Thm 4.2
// is kept as integers: w_i = ceil(max(l_i, 0) 2^Q) and its inclusive prefix sum.
//
// One workgroup per mode: the mode's work is O(I_n R_n^2) and latency bound.
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

// LDS budget: two R x R FP64 buffers (64 KB at R = 64).
template <class T>
__global__ __launch_bounds__(kBlock) void leverage_kernel(Geom g, FactorPtrs fp, double* scores,
                                                          uint64_t* cdf, double* Lg,
                                                          double* Linvg, double* Pg, double* Q64,
                                                          float* Q32, int32_t* status) {
  __shared__ double bufC[kMaxRank * kMaxRank];  // C, then L (lower) in place
  __shared__ double bufA[kMaxRank * kMaxRank];  // row chunks of A, then L^{-1}
  __shared__ int bad;
  __shared__ double thr;

  const int n = blockIdx.x;
  const int tid = threadIdx.x;
  const int R = g.ranks[n];
  const int64_t I = g.dims[n];
  const T* A = static_cast<const T*>(fp.p[n]);
  const int E = R * (R + 1) / 2;

  // ---- C = A^T A (lower triangle, FP64), rows streamed through LDS
  constexpr int kMaxPer = (kMaxRank * (kMaxRank + 1) / 2 + kBlock - 1) / kBlock;
  double acc[kMaxPer];
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) acc[k] = 0.0;
  const int64_t chunk_rows = (kMaxRank * kMaxRank) / R;
  for (int64_t r0 = 0; r0 < I; r0 += chunk_rows) {
    const int64_t rows = (I - r0 < chunk_rows) ? (I - r0) : chunk_rows;
    __syncthreads();
    for (int64_t e = tid; e < rows * R; e += kBlock) bufA[e] = ld(A, r0 * R + e);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
      const int e = tid + k * kBlock;
      if (e < E) {
        // e -> (a, b), b <= a
        int a = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= e) ++a;
        while (a * (a + 1) / 2 > e) --a;
        const int b = e - a * (a + 1) / 2;
        double s = acc[k];
        for (int64_t i = 0; i < rows; ++i) s = fma(bufA[i * R + a], bufA[i * R + b], s);
        acc[k] = s;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) {
    const int e = tid + k * kBlock;
    if (e < E) {
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

  // ---- whitened rows, scores, integer weights (one wave per row, lane = column)
  double* sc = scores ? scores + g.off[n] : nullptr;
  uint64_t* cd = cdf + g.off[n];
  double* q64 = Q64 + g.qoff[n];
  float* q32 = Q32 + g.qoff[n];
  const int wave = tid >> 6, lane = tid & 63;
  for (int64_t i = wave; i < I; i += kBlock / 64) {
    double q = 0.0;
    if (lane < R) {
      for (int k = 0; k <= lane; ++k) q = fma(bufA[lane * R + k], ld(A, i * R + k), q);
      q64[i * R + lane] = q;
      q32[i * R + lane] = static_cast<float>(q);
    }
    double l = q * q;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (lane == 0) {
      if (sc) sc[i] = l;
      const double lc = l > 0.0 ? l : 0.0;
      cd[i] = static_cast<uint64_t>(ceil(lc * static_cast<double>(1ull << TK_Q_BITS)));
    }
  }
  __syncthreads();

  // ---- inclusive prefix sum of the weights (integer, order independent)
  uint64_t* sbuf = reinterpret_cast<uint64_t*>(bufC);  // L already stored
  uint64_t carry = 0;
  for (int64_t base = 0; base < I; base += kBlock) {
    const int64_t i = base + tid;
    uint64_t v = (i < I) ? cd[i] : 0;
    sbuf[tid] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      uint64_t add = (tid >= off) ? sbuf[tid - off] : 0;
      __syncthreads();
      sbuf[tid] += add;
      __syncthreads();
    }
    if (i < I) cd[i] = sbuf[tid] + carry;
    carry += sbuf[kBlock - 1];
    __syncthreads();
  }
  if (tid == 0 && bad) atomicMax(status, static_cast<int32_t>(TK_E_RANK_DEFICIENT));
}

}  // namespace

void launch_leverage(const Geom& g, const void* const* factors, tk_dtype dt, double* scores,
                     uint64_t* cdf, double* L, double* Linv, double* P, double* Q64, float* Q32,
                     int32_t* status, hipStream_t st) {
  FactorPtrs fp;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  if (dt == TK_F64)
    hipLaunchKernelGGL(leverage_kernel<double>, dim3(g.order), dim3(kBlock), 0, st, g, fp,
                       scores, cdf, L, Linv, P, Q64, Q32, status);
  else
    hipLaunchKernelGGL(leverage_kernel<float>, dim3(g.order), dim3(kBlock), 0, st, g, fp,
                       scores, cdf, L, Linv, P, Q64, Q32, status);
}

}  // namespace tk
