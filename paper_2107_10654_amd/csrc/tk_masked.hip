// Exact core update over the observed entries of a masked tensor.
//
// The core step of Alg. 2 with missing entries uses the design rows of the
// observed entries only (the masked design of Sec. 4.2):
//   (K~^T K~ + lambda I) g = K~^T x~.
// In the eigenbasis of C_n = A(n)^T A(n) = V_n Lambda_n V_n^T (proof of
// Lemma 4.1), with W_n = A(n) V_n, K_W = (x)_n W_n, D = diag(mask) and
// y = ((x)_n V_n)^T g, the system reads
//   (K_W^T D K_W + lambda I) y = K_W^T D x,
// and the unmasked operator K_W^T K_W + lambda I = (x)_n Lambda_n + lambda I
// is diagonal; it preconditions conjugate gradients.  A product with the
// masked operator maps y up the chain of modes 0..N-2
// (H = y x_0 W_0 ... x_{N-2} W_{N-2}), applies W_{N-1}^T D_f W_{N-1} to each
// fibre f along the last mode (the masked tensor is never formed), and
// contracts back down with W_n^T.
#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kMChunk = 64;  // rows of W_{N-1} staged in LDS per step

__device__ inline bool observed(const uint32_t* mask, int64_t flat) {
  return (mask[flat >> 5] >> (flat & 31)) & 1u;
}

// out[f][r] = sum_{i observed} X[f * I + i] W[i][r]   (one thread per fibre)
template <class T, int RMAX>
__global__ __launch_bounds__(kBlock) void masked_rhs_kernel(const T* __restrict__ X,
                                                            const uint32_t* __restrict__ mask,
                                                            int64_t P, int64_t I,
                                                            const double* __restrict__ W, int R,
                                                            double* __restrict__ out) {
  __shared__ double Ws[kMChunk][RMAX];
  const int64_t f = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool ok = f < P;
  double z[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) z[r] = 0.0;
  for (int64_t i0 = 0; i0 < I; i0 += kMChunk) {
    const int ic = static_cast<int>((I - i0) < kMChunk ? (I - i0) : kMChunk);
    __syncthreads();
    for (int e = threadIdx.x; e < kMChunk * RMAX; e += kBlock) {
      const int i = e / RMAX, r = e % RMAX;
      Ws[i][r] = (i < ic && r < R) ? W[(i0 + i) * R + r] : 0.0;
    }
    __syncthreads();
    if (ok) {
      const int64_t base = f * I + i0;
      for (int i = 0; i < ic; ++i) {
        const int64_t flat = base + i;
        const double x = observed(mask, flat) ? static_cast<double>(X[flat]) : 0.0;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) z[r] = fma(x, Ws[i][r], z[r]);
      }
    }
  }
  if (ok)
    for (int r = 0; r < R; ++r) out[f * R + r] = z[r];
}

// out[f] = W^T D_f W h[f]   (one thread per fibre; h, out: P x R)
template <int RMAX>
__global__ __launch_bounds__(kBlock) void masked_normal_kernel(const double* __restrict__ H,
                                                               const uint32_t* __restrict__ mask,
                                                               int64_t P, int64_t I,
                                                               const double* __restrict__ W, int R,
                                                               double* __restrict__ out,
                                                               const int32_t* done) {
  if (done && *done) return;
  __shared__ double Ws[kMChunk][RMAX];
  const int64_t f = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool ok = f < P;
  double h[RMAX], z[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    h[r] = (ok && r < R) ? H[f * R + r] : 0.0;
    z[r] = 0.0;
  }
  for (int64_t i0 = 0; i0 < I; i0 += kMChunk) {
    const int ic = static_cast<int>((I - i0) < kMChunk ? (I - i0) : kMChunk);
    __syncthreads();
    for (int e = threadIdx.x; e < kMChunk * RMAX; e += kBlock) {
      const int i = e / RMAX, r = e % RMAX;
      Ws[i][r] = (i < ic && r < R) ? W[(i0 + i) * R + r] : 0.0;
    }
    __syncthreads();
    if (ok) {
      const int64_t base = f * I + i0;
      for (int i = 0; i < ic; ++i) {
        if (!observed(mask, base + i)) continue;
        double u = 0.0;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) u = fma(Ws[i][r], h[r], u);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) z[r] = fma(u, Ws[i][r], z[r]);
      }
    }
  }
  if (ok)
    for (int r = 0; r < R; ++r) out[f * R + r] = z[r];
}

// preconditioner diagonal prod_n Lambda_n[r_n] + lambda
__device__ inline double kron_diag(const Geom& g, const double* lam, double lambda, int64_t r) {
  double p = 1.0;
  int64_t a = r;
  for (int n = g.order - 1; n >= 0; --n) {
    const int R = g.ranks[n];
    p *= lam[n * kMaxRank + a % R];
    a /= R;
  }
  return p + lambda;
}

constexpr int kCg = 1024;

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kCg / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// y = b / diag
__global__ __launch_bounds__(kBlock) void pcg_guess_kernel(Geom g, const double* __restrict__ lam,
                                                           double lambda,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ y) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (r < g.d) y[r] = b[r] / kron_diag(g, lam, lambda, r);
}

// scal: [0] r.z, [1] ||b||, [2] relative residual, [3] iterations
// r = b - (q + lambda y); z = r / diag; p = z
__global__ __launch_bounds__(kCg) void pcg_start_kernel(Geom g, const double* __restrict__ lam,
                                                        double lambda, double tol,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ r,
                                                        double* __restrict__ p, double* scal,
                                                        int32_t* done) {
  __shared__ double red[kCg];
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int64_t i = threadIdx.x; i < g.d; i += kCg) {
    const double ri = b[i] - fma(lambda, y[i], q[i]);
    const double zi = ri / kron_diag(g, lam, lambda, i);
    r[i] = ri;
    p[i] = zi;
    rz = fma(ri, zi, rz);
    rr = fma(ri, ri, rr);
    bb = fma(b[i], b[i], bb);
  }
  rz = block_sum(rz, red);
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    const double bn = sqrt(bb);
    const double rel = bn > 0.0 ? sqrt(rr) / bn : sqrt(rr);
    scal[0] = rz;
    scal[1] = bn;
    scal[2] = rel;
    scal[3] = 0.0;
    *done = (rel <= tol) ? 1 : 0;
  }
}

// One conjugate-gradient step after q = (masked operator without lambda) p.
__global__ __launch_bounds__(kCg) void pcg_step_kernel(Geom g, const double* __restrict__ lam,
                                                       double lambda, double tol,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ y,
                                                       double* __restrict__ r,
                                                       double* __restrict__ p, double* scal,
                                                       int32_t* done) {
  if (*done) return;
  __shared__ double red[kCg];
  __shared__ double sh[2];
  double pq = 0.0;
  for (int64_t i = threadIdx.x; i < g.d; i += kCg) pq = fma(p[i], fma(lambda, p[i], q[i]), pq);
  pq = block_sum(pq, red);
  const double alpha = scal[0] / pq;
  double rr = 0.0;
  for (int64_t i = threadIdx.x; i < g.d; i += kCg) {
    y[i] = fma(alpha, p[i], y[i]);
    const double ri = r[i] - alpha * fma(lambda, p[i], q[i]);
    r[i] = ri;
    rr = fma(ri, ri, rr);
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) {
    const double rel = scal[1] > 0.0 ? sqrt(rr) / scal[1] : sqrt(rr);
    sh[0] = rel;
    scal[2] = rel;
    scal[3] += 1.0;
  }
  __syncthreads();
  if (sh[0] <= tol) {
    if (threadIdx.x == 0) *done = 1;
    return;
  }
  double rz = 0.0;
  for (int64_t i = threadIdx.x; i < g.d; i += kCg) rz = fma(r[i], r[i] / kron_diag(g, lam, lambda, i), rz);
  rz = block_sum(rz, red);
  const double beta = rz / scal[0];
  for (int64_t i = threadIdx.x; i < g.d; i += kCg)
    p[i] = fma(beta, p[i], r[i] / kron_diag(g, lam, lambda, i));
  __syncthreads();
  if (threadIdx.x == 0) scal[0] = rz;
}

__global__ void pcg_finish_kernel(const int32_t* done, int32_t* status) {
  if (threadIdx.x == 0 && !*done) atomicMax(status, static_cast<int32_t>(TK_E_NO_CONVERGE));
}

template <class T, int RMAX>
void rhs_launch(const T* X, const uint32_t* mask, int64_t P, int64_t I, const double* W, int R,
                double* out, hipStream_t st) {
  hipLaunchKernelGGL((masked_rhs_kernel<T, RMAX>), dim3(static_cast<unsigned>(cdiv(P, kBlock))),
                     dim3(kBlock), 0, st, X, mask, P, I, W, R, out);
}

template <class T>
void rhs_dispatch(const T* X, const uint32_t* mask, int64_t P, int64_t I, const double* W, int R,
                  double* out, hipStream_t st) {
  if (R <= 8) rhs_launch<T, 8>(X, mask, P, I, W, R, out, st);
  else if (R <= 16) rhs_launch<T, 16>(X, mask, P, I, W, R, out, st);
  else if (R <= 32) rhs_launch<T, 32>(X, mask, P, I, W, R, out, st);
  else rhs_launch<T, 64>(X, mask, P, I, W, R, out, st);
}

}  // namespace

void launch_masked_rhs(const void* X, tk_dtype dt, const uint32_t* mask, int64_t P, int64_t I,
                       const double* W, int R, double* out, hipStream_t st) {
  if (dt == TK_F64)
    rhs_dispatch<double>(static_cast<const double*>(X), mask, P, I, W, R, out, st);
  else
    rhs_dispatch<float>(static_cast<const float*>(X), mask, P, I, W, R, out, st);
}

void launch_masked_normal(const double* H, const uint32_t* mask, int64_t P, int64_t I,
                          const double* W, int R, double* out, const int32_t* done,
                          hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(cdiv(P, kBlock)));
  if (R <= 8)
    hipLaunchKernelGGL(masked_normal_kernel<8>, grid, dim3(kBlock), 0, st, H, mask, P, I, W, R,
                       out, done);
  else if (R <= 16)
    hipLaunchKernelGGL(masked_normal_kernel<16>, grid, dim3(kBlock), 0, st, H, mask, P, I, W, R,
                       out, done);
  else if (R <= 32)
    hipLaunchKernelGGL(masked_normal_kernel<32>, grid, dim3(kBlock), 0, st, H, mask, P, I, W, R,
                       out, done);
  else
    hipLaunchKernelGGL(masked_normal_kernel<64>, grid, dim3(kBlock), 0, st, H, mask, P, I, W, R,
                       out, done);
}

void launch_pcg_guess(const Geom& g, const double* lam, double lambda, const double* b, double* y,
                      hipStream_t st) {
  hipLaunchKernelGGL(pcg_guess_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, g, lam, lambda, b, y);
}

void launch_pcg_start(const Geom& g, const double* lam, double lambda, double tol, const double* b,
                      const double* y, const double* q, double* r, double* p, double* scal,
                      int32_t* done, hipStream_t st) {
  hipLaunchKernelGGL(pcg_start_kernel, dim3(1), dim3(kCg), 0, st, g, lam, lambda, tol, b, y, q, r,
                     p, scal, done);
}

void launch_pcg_step(const Geom& g, const double* lam, double lambda, double tol, const double* q,
                     double* y, double* r, double* p, double* scal, int32_t* done,
                     hipStream_t st) {
  hipLaunchKernelGGL(pcg_step_kernel, dim3(1), dim3(kCg), 0, st, g, lam, lambda, tol, q, y, r, p,
                     scal, done);
}

void launch_pcg_finish(const int32_t* done, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(pcg_finish_kernel, dim3(1), dim3(64), 0, st, done, status);
}

}  // namespace tk
