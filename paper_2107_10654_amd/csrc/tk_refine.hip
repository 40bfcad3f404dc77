// One FP64 iterative-refinement step for a small Kronecker dimension
// (d <= 256: at most four 64 x 64 Cholesky blocks), in a single workgroup.
//
// The sampled ridge system (whitened form) is (G_Q + lambda P) h = b_Q with
// G_Q = sum_t weff_t q_t q_t^T and P = (x)_n P_n.  The Gram is formed in
// BF16/FP32 on MFMA and factored in FP64; the refinement evaluates the
// residual in FP64 without forming G_Q:
//   r = b + sum_t q_t (xw_t - weff_t q_t . h) - lambda P h,
// whose data term the residual kernel leaves as per-workgroup partial sums.
// This step adds the partials in a fixed order, applies P mode by mode,
// measures ||r|| / ||rhs||, sets the device `done` flag once it is at most
// tol, and otherwise solves L L^T delta = r by block substitution with the
// stored diagonal-block inverses and adds delta to h.  Once `done` is set the
// step returns at entry, so the host may enqueue a fixed number of steps.
#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kRsThreads = 1024;
constexpr int kRsD = 256;
constexpr int kNb = kCholNb;  // 64
constexpr int kLd = kNb + 1;

__device__ inline double block_sum(double v, double* red) {
  // sum over the workgroup (fixed order: lanes by xor tree, then waves)
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kRsThreads / 64; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(kRsThreads) void refine_step_small_kernel(
    Geom g, const double* __restrict__ part, int64_t nparts, const double* __restrict__ P,
    const double* __restrict__ b, double lambda, const double* __restrict__ norm_ref, double tol,
    const double* __restrict__ L, const double* __restrict__ Linv_diag, double* __restrict__ h,
    int32_t* done, int32_t* steps, double* relres, int do_solve, int first) {
  // first: the initial solve h = (L L^T)^{-1} b (no partials, h taken as
  // zero and written, done cleared, no step counted)
  if (!first && *done) return;
  __shared__ double rs[kRsD], ta[kRsD], tb[kRsD], yv[kRsD], acc[kNb];
  __shared__ double red[kRsThreads];
  __shared__ double Li[kNb * kLd];
  const int tid = threadIdx.x;
  const int d = static_cast<int>(g.d);
  const int N = g.order;
  // the first diagonal-block inverse, loaded now and stored once it is needed
  double li0[kNb * kNb / kRsThreads];
#pragma unroll
  for (int q = 0; q < kNb * kNb / kRsThreads; ++q) li0[q] = Linv_diag[tid + q * kRsThreads];

  // 1. data term: sum of the workgroup partials, G groups of threads per entry
  {
    const int G = kRsThreads / d;
    const int i = tid % d, gq = tid / d;
    double v = 0.0;
    if (gq < G) {
      // eight loads in flight: parts gq, gq + G, ..., added in that order
      int64_t k = gq;
      for (; k + 7 * G < nparts; k += 8 * G) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(k + u * G) * d + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
      }
      for (; k < nparts; k += G) v += part[k * d + i];
    }
    red[tid] = v;
    if (tid < d) ta[tid] = first ? 0.0 : h[tid];
    __syncthreads();
    if (tid < d) {
      double s = 0.0;
      for (int k = 0; k < G; ++k) s += red[k * d + tid];
      rs[tid] = s;
    }
    __syncthreads();
  }
  // 2. P h, one mode at a time: t <- t x_n P_n
  double* cur = ta;
  double* nxt = tb;
  for (int n = 0; n < N; ++n) {
    const int R = g.ranks[n];
    int stride = 1;
    for (int m = n + 1; m < N; ++m) stride *= g.ranks[m];
    const double* Pn = P + g.roff[n];
    if (tid < d) {
      const int j = (tid / stride) % R;
      const int base = tid - j * stride;
      double v = 0.0;
      for (int i2 = 0; i2 < R; ++i2) v = fma(Pn[j * R + i2], cur[base + i2 * stride], v);
      nxt[tid] = v;
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  // 3. r = data + b - lambda P h, its relative norm and the convergence test
  double a2 = 0.0, n2 = 0.0;
  if (tid < d) {
    double v = rs[tid];
    if (b) v += b[tid];
    v = fma(-lambda, cur[tid], v);
    rs[tid] = v;
    a2 = v * v;
    n2 = norm_ref[tid] * norm_ref[tid];
  }
  const double sa = block_sum(a2, red);
  const double sn = block_sum(n2, red + 32);
  const double rel = sn > 0.0 ? sqrt(sa / sn) : sqrt(sa);
  const bool conv = !first && rel <= tol;
  if (tid == 0) {
    if (first) {
      *done = 0;
    } else {
      *relres = rel;
      if (conv)
        *done = 1;
      else if (do_solve)
        *steps += 1;
    }
  }
  if (conv || !(do_solve || first)) return;

  // 4. delta = (L L^T)^{-1} r by 64-row blocks; h += delta
  const int nblk = (d + kNb - 1) / kNb;
  const int row = tid & 63, pq = tid >> 6;  // 16 column groups per row
  // forward: y_i = Linv_ii (r_i - sum_{j < i} L_ij y_j)
  for (int i = 0; i < nblk; ++i) {
    const int i0 = i * kNb;
    const int rows = d - i0 < kNb ? d - i0 : kNb;
    __syncthreads();
    if (i == 0) {
#pragma unroll
      for (int q = 0; q < kNb * kNb / kRsThreads; ++q) {
        const int e = tid + q * kRsThreads;
        Li[(e >> 6) * kLd + (e & 63)] = li0[q];
      }
    } else {
      for (int e = tid; e < kNb * kNb; e += kRsThreads)
        Li[(e >> 6) * kLd + (e & 63)] = Linv_diag[static_cast<int64_t>(i) * kNb * kNb + e];
    }
    double v = 0.0;
    if (row < rows)
      for (int c = pq; c < i0; c += 16) v = fma(L[static_cast<int64_t>(i0 + row) * d + c], yv[c], v);
    red[tid] = v;
    __syncthreads();
    if (tid < kNb) {
      double s = 0.0;
      for (int k = 0; k < 16; ++k) s += red[k * 64 + tid];
      acc[tid] = tid < rows ? rs[i0 + tid] - s : 0.0;
    }
    __syncthreads();
    v = 0.0;
    for (int c = pq; c <= row; c += 16) v = fma(Li[row * kLd + c], acc[c], v);
    red[tid] = v;
    __syncthreads();
    if (tid < rows) {
      double s = 0.0;
      for (int k = 0; k < 16; ++k) s += red[k * 64 + tid];
      yv[i0 + tid] = s;
    }
  }
  // backward: x_i = Linv_ii^T (y_i - sum_{j > i} L_ji^T x_j), x kept in rs
  for (int i = nblk - 1; i >= 0; --i) {
    const int i0 = i * kNb;
    const int rows = d - i0 < kNb ? d - i0 : kNb;
    __syncthreads();
    if (i != nblk - 1)  // the last forward block is still in Li
      for (int e = tid; e < kNb * kNb; e += kRsThreads)
        Li[(e >> 6) * kLd + (e & 63)] = Linv_diag[static_cast<int64_t>(i) * kNb * kNb + e];
    double v = 0.0;
    if (row < rows)
      for (int c = i0 + kNb + pq; c < d; c += 16)
        v = fma(L[static_cast<int64_t>(c) * d + i0 + row], rs[c], v);
    red[tid] = v;
    __syncthreads();
    if (tid < kNb) {
      double s = 0.0;
      for (int k = 0; k < 16; ++k) s += red[k * 64 + tid];
      acc[tid] = tid < rows ? yv[i0 + tid] - s : 0.0;
    }
    __syncthreads();
    v = 0.0;
    for (int c = row + pq; c < kNb; c += 16) v = fma(Li[c * kLd + row], acc[c], v);
    red[tid] = v;
    __syncthreads();
    if (tid < rows) {
      double s = 0.0;
      for (int k = 0; k < 16; ++k) s += red[k * 64 + tid];
      rs[i0 + tid] = s;
      h[i0 + tid] = first ? s : h[i0 + tid] + s;
    }
  }
}

// The check of one refinement step for larger d (up to kPcD), in one
// workgroup: t = P h mode by mode, each output element from the previous
// buffer into the other (two d-vectors in dynamic LDS, and the P_n there too
// when np_lds > 0), then r = r + b - lambda t, relres = ||r|| / ||norm_ref||,
// done once relres <= tol (else steps += 1 when count_step).  r holds the
// summed data term on entry and the residual on exit.
constexpr int kPcD = 8192;
constexpr size_t kPcMaxLds = 160 * 1024;

__global__ __launch_bounds__(kRsThreads) void refine_check_p_kernel(
    Geom g, double* __restrict__ r, const double* __restrict__ h, const double* __restrict__ P,
    const double* __restrict__ b, double lambda, const double* __restrict__ norm_ref, double tol,
    int32_t* done, int32_t* steps, double* relres, int count_step, int np_lds,
    int32_t* solve_flags, double* solve_y) {
  if (*done) return;
  extern __shared__ double tbuf[];  // 2 x d, then np_lds P entries
  __shared__ double red[64];
  const int tid = threadIdx.x;
  const int d = static_cast<int>(g.d);
  const int N = g.order;
  double* cur = tbuf;
  double* nxt = tbuf + d;
  double* Ps = tbuf + 2 * d;
  for (int e = tid; e < d; e += kRsThreads) cur[e] = h[e];
  for (int e = tid; e < np_lds; e += kRsThreads) Ps[e] = P[e];
  __syncthreads();
  for (int n = 0; n < N; ++n) {
    const int R = g.ranks[n];
    int stride = 1;
    for (int m = n + 1; m < N; ++m) stride *= g.ranks[m];
    const double* Pn = (np_lds > 0 ? Ps : P) + g.roff[n];
    for (int e = tid; e < d; e += kRsThreads) {
      const int j = (e / stride) % R;
      const int base = e - j * stride;
      const double* prow = Pn + j * R;
      double v0 = 0.0, v1 = 0.0;
      int i = 0;
      for (; i + 2 <= R; i += 2) {
        v0 = fma(prow[i], cur[base + i * stride], v0);
        v1 = fma(prow[i + 1], cur[base + (i + 1) * stride], v1);
      }
      if (i < R) v0 = fma(prow[i], cur[base + i * stride], v0);
      nxt[e] = v0 + v1;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  double a2 = 0.0, n2 = 0.0;
  for (int e = tid; e < d; e += kRsThreads) {
    double v = r[e];
    if (b) v += b[e];
    v = fma(-lambda, cur[e], v);
    r[e] = v;
    a2 = fma(v, v, a2);
    n2 = fma(norm_ref[e], norm_ref[e], n2);
  }
  // the next correction solve's sentinels and tickets (unused once done)
  if (solve_y)
    for (int e = tid; e < d; e += kRsThreads)
      solve_y[e] = __longlong_as_double(static_cast<long long>(kSolvePending));
  if (solve_flags && tid < 2) solve_flags[tid] = 0;
  const double sa = block_sum(a2, red);
  const double sn = block_sum(n2, red + 32);
  if (tid == 0) {
    const double rel = sn > 0.0 ? sqrt(sa / sn) : sqrt(sa);
    *relres = rel;
    if (rel <= tol)
      *done = 1;
    else if (count_step)
      *steps += 1;
  }
}

// out = ((x)_n M_n^T) t (trans) or ((x)_n M_n) t for d <= kPcD in one
// workgroup: t and, when they fit, the M_n (mode n at roff[n]) in LDS, one
// mode after the other between two LDS vectors, the result written in the
// output precision.
__global__ __launch_bounds__(kRsThreads) void core_chain_small_kernel(Geom g,
                                                                      const double* __restrict__ t,
                                                                      const double* __restrict__ mats,
                                                                      int trans, int np_lds,
                                                                      void* out, int out_f64) {
  extern __shared__ double tbuf[];  // 2 x d, then np_lds matrix entries
  const int tid = threadIdx.x;
  const int d = static_cast<int>(g.d);
  const int N = g.order;
  double* cur = tbuf;
  double* nxt = tbuf + d;
  double* Ms = tbuf + 2 * d;
  for (int e = tid; e < d; e += kRsThreads) cur[e] = t[e];
  for (int e = tid; e < np_lds; e += kRsThreads) Ms[e] = mats[e];
  __syncthreads();
  for (int n = 0; n < N; ++n) {
    const int R = g.ranks[n];
    int stride = 1;
    for (int m = n + 1; m < N; ++m) stride *= g.ranks[m];
    const double* Mn = (np_lds > 0 ? Ms : mats) + g.roff[n];
    // entry (j, i) of the applied matrix: M_n[j][i], or M_n[i][j] when trans
    const int sj = trans ? 1 : R, si = trans ? R : 1;
    for (int e = tid; e < d; e += kRsThreads) {
      const int j = (e / stride) % R;
      const int base = e - j * stride;
      double v0 = 0.0, v1 = 0.0;
      int i = 0;
      for (; i + 2 <= R; i += 2) {
        v0 = fma(Mn[j * sj + i * si], cur[base + i * stride], v0);
        v1 = fma(Mn[j * sj + (i + 1) * si], cur[base + (i + 1) * stride], v1);
      }
      if (i < R) v0 = fma(Mn[j * sj + i * si], cur[base + i * stride], v0);
      nxt[e] = v0 + v1;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  for (int e = tid; e < d; e += kRsThreads) {
    if (out_f64)
      static_cast<double*>(out)[e] = cur[e];
    else
      static_cast<float*>(out)[e] = static_cast<float>(cur[e]);
  }
}

}  // namespace

// two d-vectors of kPcD doubles (128 KB) always fit; the M_n join them when
// there is room
bool core_chain_small_ok(const Geom& g) { return g.d <= kPcD; }

void launch_core_chain_small(const Geom& g, const double* t, const double* mats, bool trans,
                             void* out, tk_dtype dt, hipStream_t st) {
  int64_t np = 0;
  for (int n = 0; n < g.order; ++n) np += static_cast<int64_t>(g.ranks[n]) * g.ranks[n];
  size_t lds = 2 * sizeof(double) * static_cast<size_t>(g.d);
  int np_lds = 0;
  if (lds + sizeof(double) * static_cast<size_t>(np) + 64 * sizeof(double) <= kPcMaxLds) {
    np_lds = static_cast<int>(np);
    lds += sizeof(double) * static_cast<size_t>(np);
  }
  // dynamic LDS above the 64 KB default (gfx950: 160 KB per CU)
  ensure_dyn_lds(reinterpret_cast<const void*>(&core_chain_small_kernel),
                 static_cast<int>(kPcMaxLds - 64 * sizeof(double)));
  hipLaunchKernelGGL(core_chain_small_kernel, dim3(1), dim3(kRsThreads), lds, st, g, t, mats,
                     trans ? 1 : 0, np_lds, out, dt == TK_F64 ? 1 : 0);
}

bool refine_small_ok(const Geom& g) { return g.d <= kRsD; }

bool refine_check_p_ok(const Geom& g) { return g.d <= kPcD; }

void launch_refine_check_p(const Geom& g, double* r, const double* h, const double* P,
                           const double* b, double lambda, const double* norm_ref, double tol,
                           int32_t* done, int32_t* steps, double* relres, int count_step,
                           hipStream_t st, int32_t* solve_flags, double* solve_y) {
  // the P_n (sum_n R_n^2 entries, mode n at roff[n]) join the two vectors in
  // LDS when all fit
  int64_t np = 0;
  for (int n = 0; n < g.order; ++n) np += static_cast<int64_t>(g.ranks[n]) * g.ranks[n];
  size_t lds = 2 * sizeof(double) * static_cast<size_t>(g.d);
  int np_lds = 0;
  if (lds + sizeof(double) * static_cast<size_t>(np) + 64 * sizeof(double) <= kPcMaxLds) {
    np_lds = static_cast<int>(np);
    lds += sizeof(double) * static_cast<size_t>(np);
  }
  // dynamic LDS above the 64 KB default (gfx950: 160 KB per CU)
  ensure_dyn_lds(reinterpret_cast<const void*>(&refine_check_p_kernel),
                 static_cast<int>(kPcMaxLds - 64 * sizeof(double)));
  hipLaunchKernelGGL(refine_check_p_kernel, dim3(1), dim3(kRsThreads), lds, st, g, r, h, P, b,
                     lambda, norm_ref, tol, done, steps, relres, count_step, np_lds, solve_flags,
                     solve_y);
}

void launch_refine_step_small(const Geom& g, const double* part, int64_t nparts, const double* P,
                              const double* b, double lambda, const double* norm_ref, double tol,
                              const double* L, const double* Linv_diag, double* h, int32_t* done,
                              int32_t* steps, double* relres, int do_solve, hipStream_t st,
                              int first) {
  hipLaunchKernelGGL(refine_step_small_kernel, dim3(1), dim3(kRsThreads), 0, st, g, part, nparts,
                     P, b, lambda, norm_ref, tol, L, Linv_diag, h, done, steps, relres, do_solve,
                     first);
}

}  // namespace tk
