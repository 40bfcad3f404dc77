// Exact core update, factor update and loss (Alg. 2 and Sec. 2).
//
// Exact core: the proof of Lemma 4.1 diagonalises K^T K + lambda I with the
// per-mode eigendecompositions C_n = A(n)^T A(n) = V_n Lambda_n V_n^T, so
//   G = ((K^T vec X) x_n V_n^T / ((x) Lambda_n + lambda)) x_n V_n
// with K^T vec X = X x_1 A(1)^T ... x_N A(N)^T: one streaming pass over X,
// the rest is core-sized.  Eigendecompositions are cyclic Jacobi sweeps in
// round-robin (parallel) order, one workgroup per mode.
#include "tk_internal.h"
#include "tk_mfma.h"

namespace tk {
namespace {

struct FPtrs {
  const void* p[kMaxOrder];
};

template <class T>
__device__ inline double ldv(const T* a, int64_t i) {
  return static_cast<double>(a[i]);
}

// C = A^T A for one mode (FP64), into LDS buffer C (R x R, full).  With
// E = R^2 <= 256 entries, thread (e, grp) takes entry e over the rows
// i = grp mod G (G = 256 / E) and the groups are added in order at the end;
// otherwise each thread takes entries tid, tid + 256, ... over all rows.
template <class T>
__device__ void mode_gram(const T* A, int64_t I, int R, double* C, double* buf) {
  const int tid = threadIdx.x;
  const int E = R * R;
  const bool grouped = E <= kBlock;
  const int G = grouped ? kBlock / E : 1;
  const int grp = grouped ? tid / E : 0;
  const int e0 = grouped ? tid % E : tid;
  double gacc = 0.0;  // grouped partial of entry e0
  for (int e = tid; e < E; e += kBlock) C[e] = 0.0;
  const int64_t chunk_rows = (kMaxRank * kMaxRank) / R;
  for (int64_t r0 = 0; r0 < I; r0 += chunk_rows) {
    const int64_t rows = (I - r0 < chunk_rows) ? (I - r0) : chunk_rows;
    __syncthreads();
    {
      // eight loads in flight per thread (indices clamped into range)
      const int64_t n = rows * R;
      const T* src = A + r0 * R;
      for (int64_t q0 = tid; q0 < n; q0 += 8 * kBlock) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int64_t q = q0 + k * kBlock;
          v[k] = ldv(src, q < n ? q : n - 1);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int64_t q = q0 + k * kBlock;
          if (q < n) buf[q] = v[k];
        }
      }
    }
    __syncthreads();
    if (grouped) {
      if (grp < G) {
        const int a = e0 / R, b = e0 % R;
        double s0 = 0.0, s1 = 0.0;
        int64_t i = grp;
        for (; i + G < rows; i += 2 * G) {
          s0 = fma(buf[i * R + a], buf[i * R + b], s0);
          s1 = fma(buf[(i + G) * R + a], buf[(i + G) * R + b], s1);
        }
        if (i < rows) s0 = fma(buf[i * R + a], buf[i * R + b], s0);
        gacc += s0 + s1;
      }
    } else {
      for (int e = tid; e < E; e += kBlock) {
        const int a = e / R, b = e % R;
        double s = C[e];
        for (int64_t i = 0; i < rows; ++i) s = fma(buf[i * R + a], buf[i * R + b], s);
        C[e] = s;
      }
    }
  }
  __syncthreads();
  if (grouped) {
    buf[tid] = grp < G ? gacc : 0.0;
    __syncthreads();
    if (tid < E) {
      double v = 0.0;
      for (int k = 0; k < G; ++k) v += buf[k * E + tid];
      C[tid] = v;
    }
  }
  __syncthreads();
}

// Per mode: C_n and its eigenpairs (V_n, Lambda_n).  Each Jacobi step rotates
// the disjoint pairs of one round-robin round: the rotations are chosen from
// the current matrix, then every 2 x 2 block (pair k1 rows, pair k2 columns) is
// transformed in place by its own thread, rows first, then columns, as are the
// pairs of columns of V.  W_n = A(n) V_n is formed by the rows kernel after.
template <class T>
__global__ __launch_bounds__(kBlock) void eig_modes_kernel(Geom g, FPtrs fp, double* Vg,
                                                           double* lamg, double* Cg) {
  __shared__ double S[kMaxRank * kMaxRank];
  __shared__ double V[kMaxRank * kMaxRank];
  __shared__ double buf[kMaxRank * kMaxRank];
  __shared__ double cs[kMaxRank / 2][2];
  __shared__ int pq[kMaxRank / 2][2];
  __shared__ double red[2][kBlock / 64];
  const int n = blockIdx.x;
  const int tid = threadIdx.x;
  const int R = g.ranks[n];
  const int64_t I = g.dims[n];
  const T* A = static_cast<const T*>(fp.p[n]);
  mode_gram(A, I, R, S, buf);
  if (Cg)
    for (int e = tid; e < R * R; e += kBlock) Cg[g.roff[n] + e] = S[e];
  for (int e = tid; e < R * R; e += kBlock) V[e] = (e / R == e % R) ? 1.0 : 0.0;
  __syncthreads();
  const int Rp = R + (R & 1);  // even player count (index R is a dummy when R is odd)
  const int npairs = Rp / 2;
  for (int sweep = 0; sweep < 30 && R > 1; ++sweep) {
    // convergence test: off-diagonal against diagonal Frobenius mass
    double o = 0.0, dg = 0.0;
    for (int e = tid; e < R * R; e += kBlock) {
      const double v = S[e];
      if (e / R == e % R)
        dg = fma(v, v, dg);
      else
        o = fma(v, v, o);
    }
    for (int off = 32; off > 0; off >>= 1) {
      o += __shfl_xor(o, off, 64);
      dg += __shfl_xor(dg, off, 64);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = o;
      red[1][tid >> 6] = dg;
    }
    __syncthreads();
    double offn = 0.0, diagn = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      offn += red[0][w];
      diagn += red[1][w];
    }
    if (offn <= 1e-30 * diagn) break;
    for (int step = 0; step < Rp - 1; ++step) {
      if (tid < npairs) {
        const int k = tid;
        int p, q;
        auto ring = [&](int j) { return ((j + step) % (Rp - 1)) + 1; };
        if (k == 0) {
          p = 0;
          q = ring(0);
        } else {
          p = ring(k);
          q = ring(Rp - 1 - k);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < R) {
          const double apq = S[p * R + q];
          if (apq != 0.0) {
            const double tau = (S[q * R + q] - S[p * R + p]) / (2.0 * apq);
            const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                          : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pq[k][0] = p;
        pq[k][1] = q;
        cs[k][0] = c;
        cs[k][1] = s;
      }
      __syncthreads();
      // 2 x 2 blocks of S: rows (p1, q1) <- (c1 p1 - s1 q1, s1 p1 + c1 q1), then
      // columns (p2, q2) the same with (c2, s2); an index >= R is absent.
      const int nb = npairs * npairs;
      for (int e = tid; e < nb + npairs * R; e += kBlock) {
        if (e < nb) {
          const int k1 = e / npairs, k2 = e % npairs;
          const int p1 = pq[k1][0], q1 = pq[k1][1], p2 = pq[k2][0], q2 = pq[k2][1];
          const double c1 = cs[k1][0], s1 = cs[k1][1], c2 = cs[k2][0], s2 = cs[k2][1];
          const bool h1 = q1 < R, h2 = q2 < R;
          const double b00 = S[p1 * R + p2];
          const double b01 = h2 ? S[p1 * R + q2] : 0.0;
          const double b10 = h1 ? S[q1 * R + p2] : 0.0;
          const double b11 = (h1 && h2) ? S[q1 * R + q2] : 0.0;
          // rows
          const double r00 = h1 ? c1 * b00 - s1 * b10 : b00;
          const double r01 = h1 ? c1 * b01 - s1 * b11 : b01;
          const double r10 = s1 * b00 + c1 * b10;
          const double r11 = s1 * b01 + c1 * b11;
          // columns
          S[p1 * R + p2] = h2 ? c2 * r00 - s2 * r01 : r00;
          if (h2) S[p1 * R + q2] = s2 * r00 + c2 * r01;
          if (h1) S[q1 * R + p2] = h2 ? c2 * r10 - s2 * r11 : r10;
          if (h1 && h2) S[q1 * R + q2] = s2 * r10 + c2 * r11;
        } else {
          const int k = (e - nb) / R, i = (e - nb) % R;
          const int p = pq[k][0], q = pq[k][1];
          if (q < R) {
            const double c = cs[k][0], s = cs[k][1];
            const double a = V[i * R + p], b = V[i * R + q];
            V[i * R + p] = c * a - s * b;
            V[i * R + q] = s * a + c * b;
          }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += kBlock) Vg[g.roff[n] + e] = V[e];
  for (int a = tid; a < R; a += kBlock) lamg[n * kMaxRank + a] = S[a * R + a];
}

// B[r] /= (prod_n Lambda_n[r_n] + lambda)
__global__ void kron_scale_kernel(Geom g, const double* __restrict__ lam, double lambda,
                                  double* __restrict__ B) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= g.d) return;
  double p = 1.0;
  int64_t a = r;
  for (int n = g.order - 1; n >= 0; --n) {
    const int R = g.ranks[n];
    p *= lam[n * kMaxRank + a % R];
    a /= R;
  }
  B[r] = B[r] / (p + lambda);
}

// partial sums of squares
template <class T>
__global__ __launch_bounds__(kBlock) void sq_reduce_kernel(int64_t n, const T* __restrict__ x,
                                                           double* __restrict__ part) {
  __shared__ double red[kBlock];
  double a = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double v = static_cast<double>(x[i]);
    a = fma(v, v, a);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Residual over X, last mode expanded on FP64 MFMA: xhat[p][i] = H[p,:] . A_N[i,:]
// with H = G x_1 A(1) ... x_{N-1} A(N-1) (P x R_N).  A wave owns 16 rows p (its
// slice of H is the A operand, held in registers) and walks 64-column groups;
// A_N for a chunk of columns is staged in LDS as the B operand (Bs[c][r],
// padded stride rnp, zero beyond R_N).  X is read in the accumulator layout
// (register v of lane l: row l / 16 + 4 v, column l % 16 of a 16 x 16 block).
constexpr int kLossCols = 64;

template <class T, int K4>
__global__ __launch_bounds__(kBlock) void loss_stream_kernel(Geom g, const T* __restrict__ X,
                                                             const uint32_t* __restrict__ mask,
                                                             const double* __restrict__ H,
                                                             const double* __restrict__ AN,
                                                             int64_t P, int cc, int rnp,
                                                             double* __restrict__ psq,
                                                             double* __restrict__ pcnt) {
  extern __shared__ double Bs[];
  __shared__ double red[2][kBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int RN = g.ranks[g.order - 1];
  const int64_t IN = g.dims[g.order - 1];
  const int64_t nrb = (P + 15) / 16;
  double a = 0.0, cnt = 0.0;
  for (int64_t c0 = 0; c0 < IN; c0 += cc) {
    const int cw = static_cast<int>(IN - c0 < cc ? IN - c0 : cc);
    __syncthreads();  // the previous chunk's LDS reads are done
    for (int e = tid; e < cc * rnp; e += kBlock) {
      const int c = e / rnp, r = e % rnp;
      Bs[e] = (c < cw && r < RN) ? AN[(c0 + c) * RN + r] : 0.0;
    }
    __syncthreads();
    for (int64_t rb = static_cast<int64_t>(blockIdx.x) * 4 + wave; rb < nrb;
         rb += static_cast<int64_t>(gridDim.x) * 4) {
      const int64_t p0 = rb * 16;
      double aop[K4];
#pragma unroll
      for (int ks = 0; ks < K4; ++ks) {
        const int r = 4 * ks + lk;
        aop[ks] = (p0 + lr < P && r < RN) ? H[(p0 + lr) * RN + r] : 0.0;
      }
      for (int cb = 0; cb < cw; cb += kLossCols) {
        T xv[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t row = p0 + lk + 4 * v;
            const int col = cb + 16 * t + lr;
            const bool ok = row < P && col < cw;
            xv[t][v] = X[ok ? row * IN + c0 + col : 0];
          }
        doublex4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < K4; ++ks) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                aop[ks], Bs[(cb + 16 * t + lr) * rnp + 4 * ks + lk], acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t row = p0 + lk + 4 * v;
            const int col = cb + 16 * t + lr;
            bool ok = row < P && col < cw;
            if (ok && mask) {
              const int64_t e = row * IN + c0 + col;
              ok = (mask[e >> 5] >> (e & 31)) & 1u;
            }
            if (ok) {
              const double res = static_cast<double>(xv[t][v]) - acc[t][v];
              a = fma(res, res, a);
              cnt += 1.0;
            }
          }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    cnt += __shfl_xor(cnt, off, 64);
  }
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sc = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      sa += red[0][w];
      sc += red[1][w];
    }
    psq[blockIdx.x] = sa;
    pcnt[blockIdx.x] = sc;
  }
}

__global__ void loss_final_kernel(const double* psq, const double* pcnt, int64_t np,
                                  const double* preg, int64_t nreg, double lambda, double* out) {
  if (threadIdx.x != 0) return;
  double sq = 0.0, cnt = 0.0, reg = 0.0;
  for (int64_t i = 0; i < np; ++i) {
    sq += psq[i];
    cnt += pcnt[i];
  }
  for (int64_t i = 0; i < nreg; ++i) reg += preg[i];
  out[0] = fma(lambda, reg, sq);
  out[1] = sq;
  out[2] = cnt;
}

// out[i][a] = sum_{p,q} U[p][i][q] V[p][a][q]
__global__ __launch_bounds__(kBlock) void unfold_contract_kernel(const double* __restrict__ U,
                                                                 const double* __restrict__ V,
                                                                 int64_t P, int64_t I, int64_t A,
                                                                 int64_t Q, double* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= I * A) return;
  const int64_t i = e / A, a = e % A;
  double s = 0.0;
  for (int64_t p = 0; p < P; ++p)
    for (int64_t q = 0; q < Q; ++q) s = fma(U[(p * I + i) * Q + q], V[(p * A + a) * Q + q], s);
  out[e] = s;
}

// A(n) = rhs (KKt + lambda I)^{-1}, rows independent; one workgroup factors, all rows solve.
template <class T>
__global__ __launch_bounds__(kBlock) void factor_solve_kernel(const double* __restrict__ KKt,
                                                              const double* __restrict__ rhs,
                                                              int64_t I, int R, double lambda,
                                                              T* __restrict__ out,
                                                              int32_t* status) {
  __shared__ double L[kMaxRank * kMaxRank];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < R * R; e += kBlock) L[e] = KKt[e] + ((e / R == e % R) ? lambda : 0.0);
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    if (tid == 0) {
      double piv = L[j * R + j];
      if (!(piv > 0.0)) {
        bad = 1;
        piv = 1.0;
      }
      L[j * R + j] = sqrt(piv);
    }
    __syncthreads();
    const double ljj = L[j * R + j];
    for (int i = j + 1 + tid; i < R; i += kBlock) L[i * R + j] /= ljj;
    __syncthreads();
    const int m = R - j - 1;
    for (int e = tid; e < m * m; e += kBlock) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) L[i * R + c] = fma(-L[i * R + j], L[c * R + j], L[i * R + c]);
    }
    __syncthreads();
  }
  if (tid == 0 && bad && blockIdx.x == 0) atomicMax(status, static_cast<int32_t>(TK_E_NOT_SPD));
  // each wave solves rows; lane-serial substitution (R <= 64)
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + tid; i < I;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double y[kMaxRank];
    for (int a = 0; a < R; ++a) {
      double s = rhs[i * R + a];
      for (int c = 0; c < a; ++c) s = fma(-L[a * R + c], y[c], s);
      y[a] = s / L[a * R + a];
    }
    for (int a = R - 1; a >= 0; --a) {
      double s = y[a];
      for (int c = a + 1; c < R; ++c) s = fma(-L[c * R + a], y[c], s);
      y[a] = s / L[a * R + a];
    }
    for (int a = 0; a < R; ++a) out[i * R + a] = static_cast<T>(y[a]);
  }
}

// C_n = A(n)^T A(n) for every mode (factor update Gram terms)
template <class T>
__global__ __launch_bounds__(kBlock) void gram_modes_kernel(Geom g, FPtrs fp, double* Cg) {
  __shared__ double S[kMaxRank * kMaxRank];
  __shared__ double buf[kMaxRank * kMaxRank];
  const int n = blockIdx.x;
  mode_gram(static_cast<const T*>(fp.p[n]), g.dims[n], g.ranks[n], S, buf);
  for (int e = threadIdx.x; e < g.ranks[n] * g.ranks[n]; e += kBlock) Cg[g.roff[n] + e] = S[e];
}

}  // namespace

void launch_eig_modes(const Geom& g, const void* const* factors, tk_dtype dt, double* V,
                      double* lam, double* W, double* C, hipStream_t st) {
  FPtrs fp;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  if (dt == TK_F64)
    hipLaunchKernelGGL(eig_modes_kernel<double>, dim3(g.order), dim3(kBlock), 0, st, g, fp, V, lam,
                       C);
  else
    hipLaunchKernelGGL(eig_modes_kernel<float>, dim3(g.order), dim3(kBlock), 0, st, g, fp, V, lam,
                       C);
  if (W) launch_mode_rows(g, factors, dt, V, 0, W, nullptr, nullptr, nullptr, st);
}

namespace {

// Cor. B.1: with sigma_max(A(n))^2 the largest eigenvalue of C_n,
// out = {1/beta bound, prod_n sigma_max^2, beta', s}; s = ceil(k / beta)
// with k = 4 d (1 + c) max{420 ln(4d/delta), 1/(delta eps)} formed on the host.
__global__ void masked_bound_kernel(Geom g, const double* __restrict__ lam_modes, double lambda,
                                    double k, double one_plus_c, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double prod = 1.0;
  for (int n = 0; n < g.order; ++n) {
    double mx = 0.0;
    for (int a = 0; a < g.ranks[n]; ++a) mx = fmax(mx, lam_modes[n * kMaxRank + a]);
    prod *= mx;
  }
  const double inv_beta = 2.0 + prod / lambda;
  out[0] = inv_beta;
  out[1] = prod;
  out[2] = (1.0 / inv_beta) / one_plus_c;
  out[3] = ceil(k * inv_beta);
}

}  // namespace

void launch_masked_bound(const Geom& g, const double* lam_modes, double lambda, double k,
                         double one_plus_c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(masked_bound_kernel, dim3(1), dim3(64), 0, st, g, lam_modes, lambda, k,
                     one_plus_c, out);
}

void launch_gram_modes(const Geom& g, const void* const* factors, tk_dtype dt, double* C,
                       hipStream_t st) {
  FPtrs fp;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  if (dt == TK_F64)
    hipLaunchKernelGGL(gram_modes_kernel<double>, dim3(g.order), dim3(kBlock), 0, st, g, fp, C);
  else
    hipLaunchKernelGGL(gram_modes_kernel<float>, dim3(g.order), dim3(kBlock), 0, st, g, fp, C);
}

void launch_kron_scale(const Geom& g, const double* lam_modes, double lambda, double* B,
                       hipStream_t st) {
  hipLaunchKernelGGL(kron_scale_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, g, lam_modes, lambda, B);
}

void launch_sq_reduce(int64_t n, const void* x, tk_dtype dt, double* part, int64_t nparts,
                      hipStream_t st) {
  if (dt == TK_F64)
    hipLaunchKernelGGL(sq_reduce_kernel<double>, dim3(static_cast<unsigned>(nparts)), dim3(kBlock),
                       0, st, n, static_cast<const double*>(x), part);
  else
    hipLaunchKernelGGL(sq_reduce_kernel<float>, dim3(static_cast<unsigned>(nparts)), dim3(kBlock),
                       0, st, n, static_cast<const float*>(x), part);
}

template <class T>
void loss_stream_dispatch(int k4, dim3 grid, size_t lds, hipStream_t st, const Geom& g,
                          const T* X, const uint32_t* mask, const double* H, const double* AN,
                          int64_t P, int cc, int rnp, double* psq, double* pcnt) {
#define TK_LOSS_CASE(K)                                                                        \
  case K:                                                                                      \
    hipLaunchKernelGGL((loss_stream_kernel<T, K>), grid, dim3(kBlock), lds, st, g, X, mask, H, \
                       AN, P, cc, rnp, psq, pcnt);                                             \
    break;
  switch (k4) {
    TK_LOSS_CASE(1)
    TK_LOSS_CASE(2)
    TK_LOSS_CASE(4)
    TK_LOSS_CASE(8)
    TK_LOSS_CASE(16)
  }
#undef TK_LOSS_CASE
}

void launch_loss_stream(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                        const double* H, const double* AN, double* part_sq, double* part_cnt,
                        int64_t nparts, hipStream_t st) {
  // k-steps of 4 ranks, rounded up to a power of two (the operands are zero-padded)
  const int RN = g.ranks[g.order - 1];
  int k4 = 1;
  while (4 * k4 < RN) k4 *= 2;
  // A_N chunk in LDS: at most 48 KB, whole 64-column groups, chunks of equal size
  const int64_t IN = g.dims[g.order - 1];
  const int rnp = 4 * k4 + 1;
  const int64_t in64 = cdiv(IN, kLossCols) * kLossCols;
  const int64_t maxc = (6144 / rnp) / kLossCols * kLossCols;
  const int64_t nch = cdiv(in64, maxc);
  const int cc = static_cast<int>(cdiv(cdiv(in64, nch), kLossCols) * kLossCols);
  const size_t lds = static_cast<size_t>(cc) * rnp * sizeof(double);
  const int64_t P = g.numel / IN;
  const dim3 grid(static_cast<unsigned>(nparts));
  if (dt == TK_F64)
    loss_stream_dispatch(k4, grid, lds, st, g, static_cast<const double*>(X), mask, H, AN, P, cc,
                         rnp, part_sq, part_cnt);
  else
    loss_stream_dispatch(k4, grid, lds, st, g, static_cast<const float*>(X), mask, H, AN, P, cc,
                         rnp, part_sq, part_cnt);
}

void launch_loss_final(const double* part_sq, const double* part_cnt, int64_t nparts,
                       const double* part_reg, int64_t nreg, double lambda, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, part_sq, part_cnt, nparts,
                     part_reg, nreg, lambda, out);
}

void launch_unfold_contract(const double* U, const double* V, int64_t P, int64_t I, int64_t A,
                            int64_t Q, double* out, hipStream_t st) {
  hipLaunchKernelGGL(unfold_contract_kernel, dim3(static_cast<unsigned>(cdiv(I * A, kBlock))),
                     dim3(kBlock), 0, st, U, V, P, I, A, Q, out);
}

void launch_factor_solve(const double* KKt, const double* rhs, int64_t I, int R, double lambda,
                         void* out, tk_dtype dt, int32_t* status, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(cdiv(I, kBlock) < 64 ? cdiv(I, kBlock) : 64);
  if (dt == TK_F64)
    hipLaunchKernelGGL(factor_solve_kernel<double>, dim3(grid), dim3(kBlock), 0, st, KKt, rhs, I, R,
                       lambda, static_cast<double*>(out), status);
  else
    hipLaunchKernelGGL(factor_solve_kernel<float>, dim3(grid), dim3(kBlock), 0, st, KKt, rhs, I, R,
                       lambda, static_cast<float*>(out), status);
}

}  // namespace tk
