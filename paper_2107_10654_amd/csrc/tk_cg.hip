// Conjugate-gradient solve of the FP64 sketched normal equations.
//
// Alg. 1 solves its sketched ridge problem through the normal equations
// (proof of Thm 4.2): M h = b with M = sum_t w_t q_t q_t^T + lambda P
// symmetric positive definite, here given by its lower triangle (d x d,
// row-major).  In the whitened coordinates the design has orthonormal
// columns, and leverage-score sampling makes the sketch a subspace embedding
// of that column space (the leverage-sampling tool of the appendix on the
// structural conditions, Missing Analysis of Sec. 3): every eigenvalue of the
// sketched Gram lies near 1, so with s well above d conjugate gradients reach
// FP64 accuracy after a few tens of products with M.  The caller runs the
// Cholesky factorisation only when this solve reports no convergence.
//
// One persistent launch runs every iteration.  Per iteration:
//   S  each workgroup multiplies its lower 64 x 64 tiles M_IJ by the search
//      direction p = r + beta p_prev (formed on the fly from r and p_prev):
//      the row part M_IJ p_J and, off the diagonal, the column part
//      M_IJ^T p_I (diagonal tiles: strictly lower part transposed), written
//      to per-tile partials; each workgroup also writes its own entries of p;
//   R  each workgroup sums the partials of its own entries of q = M p in a
//      fixed order, and its share of p.q;
//   U  alpha = r.r / p.q (the shares summed in a fixed order by every
//      workgroup alike), h += alpha p, r -= alpha q on its own entries, and
//      its share of the new r.r;
// with a grid-wide barrier after each.  Every sum has a fixed order, so the
// result does not depend on timing.  Data that other workgroups read (p, r,
// partials, shares) is written through to memory and read with agent-scope
// loads, since the L2 of one XCD does not see another's writes.
#include <string.h>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kCt = 64;          // tile edge
constexpr int kCld = kCt + 1;    // padded LDS row
constexpr int kCgMaxOwn = 256;   // entries of h, r, p owned by one workgroup
constexpr int kCgMaxBlocks = 256;  // d <= 64 * 256
constexpr int kCgTerms = (kCgMaxBlocks + 1 + 15) / 16;  // partial terms per thread of an entry
constexpr long kCgSpinLimit = 1L << 20;
// stop once ||r|| <= kCgTol ||b|| (the recursively updated residual)
constexpr double kCgTol = 1e-14;

struct CgArgs {
  const double* M;   // lower triangle, d x d row-major
  const double* b;
  double* h;         // out: solution (b when the iteration did not converge)
  double* r;         // residual (shared)
  double* pbuf;      // two direction vectors (previous, current), 2 d
  double* rowpart;   // [tile][64]
  double* colpart;   // [tile][64]
  double* shares;    // [2][grid]: p.q and r.r shares
  int32_t* sync;     // [0] barrier arrivals, [1] abort word
  int32_t* cg_done;  // out: 1 when converged
  int32_t* steps;    // out: iterations taken
  double* relres;    // out: final ||r|| / ||b|| of the recursion
  double* min_pivot; // out: 0 (no factorisation ran) when converged
  int32_t* status;
  int64_t d, nb, ntiles, own;  // own: entries per workgroup
  int32_t max_iter;
};

__device__ inline double cload(const double* p) {
  return __longlong_as_double(static_cast<long long>(__hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ inline void cstore(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cg_complete_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ inline double dir(double r, double beta, double pprev) { return fma(beta, pprev, r); }
__device__ inline int64_t tri(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Sum of one value per thread over the workgroup in a fixed tree order.
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kBlock) void cg_kernel(CgArgs a) {
  __shared__ double tile[kCt * kCld];
  __shared__ double pI[kCt], pJ[kCt];
  __shared__ double red[kBlock];
  __shared__ double csum[4][kCt];
  __shared__ double own_p[kCgMaxOwn], own_q[kCgMaxOwn], own_h[kCgMaxOwn];
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  const int G = gridDim.x, w = blockIdx.x;
  const int64_t d = a.d, nb = a.nb;
  const int64_t e0 = w * a.own;
  const int64_t ne = (e0 + a.own < d ? e0 + a.own : d) - e0 > 0
                         ? (e0 + a.own < d ? e0 + a.own : d) - e0 : 0;
  const int64_t t0 = w * a.ntiles / G, t1 = (w + 1) * a.ntiles / G;
  double* sh_pq = a.shares;
  double* sh_rr = a.shares + G;
  int32_t* abort = a.sync + 1;
  int target = 0;
  bool failed = false;
  auto barrier = [&]() {
    cg_complete_stores();
    __syncthreads();
    target += G;
    if (tid == 0) {
      __hip_atomic_fetch_add(a.sync, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      long spins = 0;
      int ok = 1;
      while (__hip_atomic_load(a.sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kCgSpinLimit) {
          __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      ok_s = ok;
    }
    __syncthreads();
    failed = failed || !ok_s;
  };
  // sum of the grid's shares, the same fixed order in every workgroup
  auto grid_sum = [&](const double* sh) {
    double v = 0.0;
    for (int i = tid; i < G; i += kBlock) v += cload(sh + i);
    return block_sum(v, red);
  };

  // ---- start: h = 0, r = b, p_prev = 0, shares of b.b
  double part = 0.0;
  for (int64_t i = tid; i < ne; i += kBlock) {
    const double bi = a.b[e0 + i];
    cstore(a.r + e0 + i, bi);
    cstore(a.pbuf + e0 + i, 0.0);
    own_h[i] = 0.0;
    part += bi * bi;
  }
  {
    const double s = block_sum(part, red);
    if (tid == 0) cstore(sh_rr + w, s);
  }
  barrier();
  const double bb = grid_sum(sh_rr);
  double rr = bb;
  double beta = 0.0;
  int cur = 0;  // pbuf half holding p_prev
  int it = 0;
  bool conv = !(bb > 0.0);
  // tile staging roles: row tid / 4, columns 16 (tid % 4) .. + 16
  const int srow = tid >> 2, scol = (tid & 3) * 16;
  while (!conv && !failed && it < a.max_iter) {
    const double* pprev = a.pbuf + cur * d;
    double* pnext = a.pbuf + (cur ^ 1) * d;
    // ---- S: own entries of p, then the tile products
    for (int64_t i = tid; i < ne; i += kBlock) {
      const double pv = dir(cload(a.r + e0 + i), beta, cload(pprev + e0 + i));
      own_p[i] = pv;
      cstore(pnext + e0 + i, pv);
    }
    // tiles t0 .. t1 - 1 in row-major lower order; the next tile's M entries
    // and r, p_prev values load into registers while the current one is used
    int64_t ti = 0, tj = 0;
    if (t0 < t1) {
      ti = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(t0) + 1.0) - 1.0) * 0.5);
      while ((ti + 1) * (ti + 2) / 2 <= t0) ++ti;
      while (ti * (ti + 1) / 2 > t0) --ti;
      tj = t0 - ti * (ti + 1) / 2;
    }
    double v[16];
    double vr = 0.0, vp = 0.0;
    auto fetch = [&](int64_t fi, int64_t fj) {
      const int64_t r0 = fi * kCt, c0 = fj * kCt;
      const int64_t row = r0 + srow;
      const double* src = a.M + row * d + c0 + scol;
      if (fi != fj && row < d && c0 + scol + 16 <= d && (d & 1) == 0) {
#pragma unroll
        for (int e = 0; e < 16; e += 2) {
          const double2 x = *reinterpret_cast<const double2*>(src + e);
          v[e] = x.x;
          v[e + 1] = x.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int64_t col = c0 + scol + e;
          v[e] = (row < d && col < d && (fi != fj || col <= row)) ? src[e] : 0.0;
        }
      }
      if (tid < 2 * kCt) {
        const int64_t x = tid < kCt ? c0 + tid : r0 + tid - kCt;
        vr = x < d ? cload(a.r + x) : 0.0;
        vp = x < d ? cload(pprev + x) : 0.0;
      }
    };
    if (t0 < t1) fetch(ti, tj);
    for (int64_t tau = t0; tau < t1; ++tau) {
      const bool diag = ti == tj;
      if (tid < kCt)
        pJ[tid] = dir(vr, beta, vp);
      else if (tid < 2 * kCt)
        pI[tid - kCt] = dir(vr, beta, vp);
#pragma unroll
      for (int e = 0; e < 16; ++e) tile[srow * kCld + scol + e] = v[e];
      __syncthreads();
      // next tile
      if (++tj > ti) {
        ++ti;
        tj = 0;
      }
      if (tau + 1 < t1) fetch(ti, tj);
      // row part: sum_c M[row][c] pJ[c] over the 4 threads of the row
      double rs = 0.0;
#pragma unroll
      for (int e = 0; e < 16; ++e) rs = fma(tile[srow * kCld + scol + e], pJ[scol + e], rs);
      rs += __shfl_xor(rs, 1, 64);
      rs += __shfl_xor(rs, 2, 64);
      if ((tid & 3) == 0) cstore(a.rowpart + tau * kCt + srow, rs);
      // column part: sum_row M[row][c] pI[row] (diagonal tile: rows below c only)
      {
        const int c = tid & 63, rg = tid >> 6;
        double cs = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int rr_ = rg * 16 + i;
          const double m = (!diag || rr_ > c) ? tile[rr_ * kCld + c] : 0.0;
          cs = fma(m, pI[rr_], cs);
        }
        csum[rg][c] = cs;
      }
      __syncthreads();
      if (tid < kCt)
        cstore(a.colpart + tau * kCt + tid,
               ((csum[0][tid] + csum[1][tid]) + csum[2][tid]) + csum[3][tid]);
      __syncthreads();
    }
    barrier();
    // ---- R: own entries of q = M p, share of p.q
    // 16 threads per entry: thread z of entry i sums terms z, z + 16, ... of
    // [rowpart(I, 0..I), colpart(I..nb-1, I)], then the 16 in a fixed tree
    part = 0.0;
    for (int64_t base = 0; base < ne; base += kBlock / 16) {
      const int64_t i = base + (tid >> 4);
      const int z = tid & 15;
      double s = 0.0;
      if (i < ne) {
        const int64_t gi = e0 + i;
        const int64_t I = gi / kCt, o = gi % kCt;
        const int64_t nt = nb + 1;
        double t[kCgTerms];  // all loads issued before the sum
#pragma unroll
        for (int q = 0; q < kCgTerms; ++q) {
          const int64_t u = z + 16 * q;
          const double* src = u <= I ? a.rowpart + tri(I, u) * kCt + o
                                     : a.colpart + tri(I + (u - I - 1), I) * kCt + o;
          t[q] = u < nt ? cload(src) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kCgTerms; ++q) s += t[q];
      }
      s += __shfl_xor(s, 8, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 1, 64);
      if (i < ne && z == 0) {
        own_q[i] = s;
      }
    }
    __syncthreads();
    for (int64_t i = tid; i < ne; i += kBlock) part = fma(own_p[i], own_q[i], part);
    {
      const double s = block_sum(part, red);
      if (tid == 0) cstore(sh_pq + w, s);
    }
    barrier();
    // ---- U: alpha, h and r on own entries, share of r.r
    const double pq = grid_sum(sh_pq);
    const double alpha = rr / pq;
    part = 0.0;
    for (int64_t i = tid; i < ne; i += kBlock) {
      own_h[i] = fma(alpha, own_p[i], own_h[i]);
      const double rv = fma(-alpha, own_q[i], cload(a.r + e0 + i));
      cstore(a.r + e0 + i, rv);
      part = fma(rv, rv, part);
    }
    {
      const double s = block_sum(part, red);
      if (tid == 0) cstore(sh_rr + w, s);
    }
    barrier();
    const double rr_new = grid_sum(sh_rr);
    beta = rr_new / rr;
    rr = rr_new;
    cur ^= 1;
    ++it;
    conv = rr <= kCgTol * kCgTol * bb;
    if (!(pq > 0.0)) break;  // not positive definite in this direction: leave it to the factorisation
  }
  // ---- finish: h, or b again when the iteration did not converge
  for (int64_t i = tid; i < ne; i += kBlock) a.h[e0 + i] = conv ? own_h[i] : a.b[e0 + i];
  if (w == 0 && tid == 0) {
    *a.cg_done = conv ? 1 : 0;
    *a.steps = it;
    *a.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (conv) *a.min_pivot = 0.0;
  }
  if (failed && tid == 0) atomicMax(a.status, static_cast<int32_t>(TK_E_HIP));
}

}  // namespace

bool cg_ok(int64_t d) { return d >= 1024 && d <= int64_t(kCgMaxBlocks) * kCt; }

size_t cg_bytes(int64_t d) {
  const int64_t nb = cdiv(d, kCt);
  const int64_t nt = nb * (nb + 1) / 2;
  Carver c(nullptr);
  (void)c.take<double>(2 * d);            // pbuf
  (void)c.take<double>(nt * kCt);         // rowpart
  (void)c.take<double>(nt * kCt);         // colpart
  (void)c.take<double>(2 * 1024);         // shares
  (void)c.take<int32_t>(64);              // sync words
  (void)c.take<int32_t>(1);               // done
  return c.used;
}

void launch_cg(const double* M, int64_t d, const double* b, double* h, double* r, void* ws,
               int32_t* steps, double* relres, double* min_pivot, int32_t* status,
               int max_iter, hipStream_t st) {
  const int64_t nb = cdiv(d, kCt);
  const int64_t nt = nb * (nb + 1) / 2;
  Carver c(ws);
  CgArgs a;
  a.pbuf = c.take<double>(2 * d);
  a.rowpart = c.take<double>(nt * kCt);
  a.colpart = c.take<double>(nt * kCt);
  a.shares = c.take<double>(2 * 1024);
  a.sync = c.take<int32_t>(64);
  a.cg_done = c.take<int32_t>(1);
  // one workgroup per compute unit, all resident together (the barriers wait
  // on every workgroup of the launch)
  int grid = device_cu_count();
  const int res = resident_grid(reinterpret_cast<const void*>(cg_kernel), kBlock, 0);
  if (res > 0 && grid > res) grid = res;
  if (grid > 1024) grid = 1024;
  if (grid > nt) grid = static_cast<int>(nt);
  int64_t own = cdiv(d, grid);
  if (own > kCgMaxOwn) own = kCgMaxOwn;
  grid = static_cast<int>(cdiv(d, own));
  a.M = M;
  a.b = b;
  a.h = h;
  a.r = r;
  a.steps = steps;
  a.relres = relres;
  a.min_pivot = min_pivot;
  a.status = status;
  a.d = d;
  a.nb = nb;
  a.ntiles = nt;
  a.own = own;
  a.max_iter = max_iter;
  launch_fill_i32(64, 0, a.sync, st);
  hipLaunchKernelGGL(cg_kernel, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, st, a);
}

const int32_t* cg_done_word(void* ws, int64_t d) {
  const int64_t nb = cdiv(d, kCt);
  const int64_t nt = nb * (nb + 1) / 2;
  Carver c(ws);
  (void)c.take<double>(2 * d);
  (void)c.take<double>(nt * kCt);
  (void)c.take<double>(nt * kCt);
  (void)c.take<double>(2 * 1024);
  (void)c.take<int32_t>(64);
  return c.take<int32_t>(1);
}

}  // namespace tk
