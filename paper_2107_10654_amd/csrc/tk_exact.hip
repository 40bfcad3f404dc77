// Exact core update, factor update and loss (Alg. 2 and Sec. 2).
//
// Exact core: the proof of Lemma 4.1 diagonalises K^T K + lambda I with the
// per-mode eigendecompositions C_n = A(n)^T A(n) = V_n Lambda_n V_n^T, so
//   G = ((K^T vec X) x_n V_n^T / ((x) Lambda_n + lambda)) x_n V_n
// with K^T vec X = X x_1 A(1)^T ... x_N A(N)^T: one streaming pass over X,
// the rest is core-sized.  Eigendecompositions are cyclic Jacobi sweeps in
// round-robin (parallel) order, one workgroup per mode.
#include "tk_internal.h"

namespace tk {
namespace {

struct FPtrs {
  const void* p[kMaxOrder];
};

template <class T>
__device__ inline double ldv(const T* a, int64_t i) {
  return static_cast<double>(a[i]);
}

// C = A^T A for one mode (FP64), into LDS buffer C (R x R, full)
template <class T>
__device__ void mode_gram(const T* A, int64_t I, int R, double* C, double* buf) {
  const int tid = threadIdx.x;
  const int E = R * R;
  for (int e = tid; e < E; e += kBlock) C[e] = 0.0;
  const int64_t chunk_rows = (kMaxRank * kMaxRank) / R;
  for (int64_t r0 = 0; r0 < I; r0 += chunk_rows) {
    const int64_t rows = (I - r0 < chunk_rows) ? (I - r0) : chunk_rows;
    __syncthreads();
    for (int64_t e = tid; e < rows * R; e += kBlock) buf[e] = ldv(A, r0 * R + e);
    __syncthreads();
    for (int e = tid; e < E; e += kBlock) {
      const int a = e / R, b = e % R;
      double s = C[e];
      for (int64_t i = 0; i < rows; ++i) s = fma(buf[i * R + a], buf[i * R + b], s);
      C[e] = s;
    }
  }
  __syncthreads();
}

// Per mode: C_n, eigenpairs (V_n, Lambda_n), W_n = A(n) V_n.
template <class T>
__global__ __launch_bounds__(kBlock) void eig_modes_kernel(Geom g, FPtrs fp, double* Vg,
                                                           double* lamg, double* Wg, double* Cg) {
  __shared__ double S[kMaxRank * kMaxRank];
  __shared__ double V[kMaxRank * kMaxRank];
  __shared__ double buf[kMaxRank * kMaxRank];
  __shared__ double cs[kMaxRank / 2][2];
  __shared__ int pq[kMaxRank / 2][2];
  __shared__ double offn, diagn;
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
    // convergence test
    if (tid == 0) {
      double o = 0.0, dg = 0.0;
      for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b) {
          const double v = S[a * R + b];
          if (a == b)
            dg += v * v;
          else
            o += v * v;
        }
      offn = o;
      diagn = dg;
    }
    __syncthreads();
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
      // rows: (row_p, row_q) <- (c row_p - s row_q, s row_p + c row_q)
      for (int e = tid; e < npairs * R; e += kBlock) {
        const int k = e / R, j = e % R;
        const int p = pq[k][0], q = pq[k][1];
        if (q < R) {
          const double c = cs[k][0], s = cs[k][1];
          const double a = S[p * R + j], b = S[q * R + j];
          S[p * R + j] = c * a - s * b;
          S[q * R + j] = s * a + c * b;
        }
      }
      __syncthreads();
      // columns of S and V
      for (int e = tid; e < npairs * R; e += kBlock) {
        const int k = e / R, i = e % R;
        const int p = pq[k][0], q = pq[k][1];
        if (q < R) {
          const double c = cs[k][0], s = cs[k][1];
          double a = S[i * R + p], b = S[i * R + q];
          S[i * R + p] = c * a - s * b;
          S[i * R + q] = s * a + c * b;
          a = V[i * R + p];
          b = V[i * R + q];
          V[i * R + p] = c * a - s * b;
          V[i * R + q] = s * a + c * b;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += kBlock) Vg[g.roff[n] + e] = V[e];
  for (int a = tid; a < R; a += kBlock) lamg[n * kMaxRank + a] = S[a * R + a];
  // W = A V (I x R)
  double* W = Wg + g.qoff[n];
  for (int64_t e = tid; e < I * R; e += kBlock) {
    const int64_t i = e / R;
    const int b = static_cast<int>(e % R);
    double s = 0.0;
    for (int a = 0; a < R; ++a) s = fma(ldv(A, i * R + a), V[a * R + b], s);
    W[e] = s;
  }
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

// residual over X: xhat[p][i] = H[p,:] . A_N[i,:]
template <class T>
__global__ __launch_bounds__(kBlock) void loss_stream_kernel(Geom g, const T* __restrict__ X,
                                                             const uint32_t* __restrict__ mask,
                                                             const double* __restrict__ H,
                                                             const double* __restrict__ AN,
                                                             double* __restrict__ psq,
                                                             double* __restrict__ pcnt) {
  __shared__ double red[2][kBlock];
  const int N = g.order;
  const int RN = g.ranks[N - 1];
  const int64_t IN = g.dims[N - 1];
  double a = 0.0, c = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < g.numel;
       e += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (mask && !((mask[e >> 5] >> (e & 31)) & 1u)) continue;
    const int64_t p = e / IN, i = e % IN;
    double xh = 0.0;
    for (int r = 0; r < RN; ++r) xh = fma(H[p * RN + r], AN[i * RN + r], xh);
    const double res = static_cast<double>(X[e]) - xh;
    a = fma(res, res, a);
    c += 1.0;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = c;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psq[blockIdx.x] = red[0][0];
    pcnt[blockIdx.x] = red[1][0];
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
                       W, C);
  else
    hipLaunchKernelGGL(eig_modes_kernel<float>, dim3(g.order), dim3(kBlock), 0, st, g, fp, V, lam,
                       W, C);
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

void launch_loss_stream(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                        const double* H, const double* AN, double* part_sq, double* part_cnt,
                        int64_t nparts, hipStream_t st) {
  if (dt == TK_F64)
    hipLaunchKernelGGL(loss_stream_kernel<double>, dim3(static_cast<unsigned>(nparts)),
                       dim3(kBlock), 0, st, g, static_cast<const double*>(X), mask, H, AN, part_sq,
                       part_cnt);
  else
    hipLaunchKernelGGL(loss_stream_kernel<float>, dim3(static_cast<unsigned>(nparts)), dim3(kBlock),
                       0, st, g, static_cast<const float*>(X), mask, H, AN, part_sq, part_cnt);
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
