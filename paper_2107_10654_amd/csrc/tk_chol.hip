// FP64 Cholesky factorisation and triangular solves of the sketched system
// (Gram + lambda P) h = rhs.  The proof of Thm 4.2 solves the sketched
// normal equations with a pseudo-inverse; the system here is positive
// definite for lambda > 0, so a Cholesky factorisation is the direct solver.
//
// Blocked right-looking algorithm with 64 x 64 tiles, three launches per
// block column: factor the diagonal tile (and invert it), solve the tiles
// below it with the inverse, update the trailing lower triangle on FP64
// MFMA.  The triangular solves use one launch each: workgroups take block
// rows in ticket order and wait (bounded spin) for the rows they depend on.
#include "tk_internal.h"

namespace tk {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;
constexpr int NB = kCholNb;
constexpr int LDA = NB + 1;

// ---- diagonal tile: L_kk and its inverse
// Blocked over four 16-column panels.  Wave 0 factors (and inverts) each
// 16 x 16 diagonal panel in registers, lane r owning row r, with lane
// shuffles in place of barriers; the workgroup then solves the rows below the
// panel and updates the trailing triangle.  The 64 x 64 inverse is assembled
// from the four 16 x 16 inverses block row by block row.
constexpr int PB = 16;
__global__ __launch_bounds__(kBlock) void chol_diag_kernel(double* __restrict__ M, int64_t d,
                                                           int64_t k,
                                                           double* __restrict__ Linv_diag,
                                                           double* min_pivot, int32_t* status) {
  __shared__ double A[NB * LDA];
  __shared__ double Li[NB * LDA];
  __shared__ double Tm[NB * (PB + 1)];
  __shared__ int bad;
  __shared__ double pmin;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t o = k * NB;
  const int b = static_cast<int>((d - o) < NB ? (d - o) : NB);
  for (int i = ty; i < NB; i += 16)
    for (int j = tx; j < NB; j += 16) {
      A[i * LDA + j] = (i < b && j <= i) ? M[(o + i) * d + o + j] : (i == j ? 1.0 : 0.0);
      Li[i * LDA + j] = 0.0;
    }
  if (tid == 0) {
    bad = 0;
    pmin = 1e308;
  }
  __syncthreads();
  for (int p = 0; p < NB / PB; ++p) {
    const int c0 = p * PB;
    // (1) factor the 16 x 16 diagonal panel and invert it (wave 0, lane r = row r)
    if (wave == 0) {
      const int r = lane & 15;
      double a[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) a[c] = (c <= r) ? A[(c0 + r) * LDA + c0 + c] : 0.0;
      double pm = 1e308;
      bool nb_ = false;
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        double pj = __shfl(a[j], j, 64);
        if (!(pj > 0.0)) {
          nb_ = true;
          pj = 1.0;
        }
        const double ljj = sqrt(pj);
        pm = fmin(pm, ljj);
        const double lj = (r == j) ? ljj : (r > j ? a[j] / ljj : 0.0);
        a[j] = (r >= j) ? lj : 0.0;
#pragma unroll
        for (int c = j + 1; c < PB; ++c) {
          const double lc = __shfl(lj, c, 64);
          if (r >= c) a[c] = fma(-lj, lc, a[c]);
        }
      }
      // inverse: lane r computes column r, x[i] for i >= r
      double x[PB];
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        double sacc = (i == r) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) {
          const double liq = __shfl(a[q], i, 64);  // L[i][q] from lane i
          sacc = fma(-liq, x[q], sacc);
        }
        const double lii = __shfl(a[i], i, 64);
        x[i] = (i >= r) ? sacc / lii : 0.0;
      }
      if (lane < PB) {
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          A[(c0 + r) * LDA + c0 + c] = (c <= r) ? a[c] : 0.0;
          Li[(c0 + c) * LDA + c0 + r] = x[c];  // column r of the inverse
        }
      }
      if (lane == 0) {
        if (nb_) bad = 1;
        pmin = fmin(pmin, pm);
      }
    }
    __syncthreads();
    const int below = NB - (c0 + PB);
    if (below > 0) {
      // (2) rows below: X = A[c0+16:, c0:c0+16] Li_pp^T
      for (int e = tid; e < below * PB; e += kBlock) {
        const int rr = c0 + PB + (e >> 4), c = e & 15;
        double sacc = 0.0;
#pragma unroll
        for (int m = 0; m < PB; ++m)
          sacc = fma(A[rr * LDA + c0 + m], Li[(c0 + c) * LDA + c0 + m], sacc);
        Tm[(rr - c0 - PB) * (PB + 1) + c] = sacc;
      }
      __syncthreads();
      for (int e = tid; e < below * PB; e += kBlock) {
        const int rr = c0 + PB + (e >> 4), c = e & 15;
        A[rr * LDA + c0 + c] = Tm[(rr - c0 - PB) * (PB + 1) + c];
      }
      __syncthreads();
      // (3) trailing update of the lower triangle
      for (int i = c0 + PB + ty; i < NB; i += 16)
        for (int j = c0 + PB + tx; j <= i; j += 16) {
          double sacc = A[i * LDA + j];
#pragma unroll
          for (int m = 0; m < PB; ++m)
            sacc = fma(-A[i * LDA + c0 + m], A[j * LDA + c0 + m], sacc);
          A[i * LDA + j] = sacc;
        }
      __syncthreads();
    }
  }
  // (4) off-diagonal blocks of the inverse: Li_ij = -Li_ii sum_{q=j}^{i-1} L_iq Li_qj
  for (int bi = 1; bi < NB / PB; ++bi) {
    // S_j = sum_q L_{bi,q} Li_{q,j} for every block column j < bi (into Tm rows j*16..)
    for (int e = tid; e < bi * PB * PB; e += kBlock) {
      const int bj = e >> 8, rr = (e >> 4) & 15, c = e & 15;
      double sacc = 0.0;
      for (int q = bj * PB; q < bi * PB; ++q)
        sacc = fma(A[(bi * PB + rr) * LDA + q], Li[q * LDA + bj * PB + c], sacc);
      Tm[(bj * PB + rr) * (PB + 1) + c] = sacc;
    }
    __syncthreads();
    for (int e = tid; e < bi * PB * PB; e += kBlock) {
      const int bj = e >> 8, rr = (e >> 4) & 15, c = e & 15;
      double sacc = 0.0;
#pragma unroll
      for (int m = 0; m < PB; ++m)
        sacc = fma(Li[(bi * PB + rr) * LDA + bi * PB + m], Tm[(bj * PB + m) * (PB + 1) + c], sacc);
      Li[(bi * PB + rr) * LDA + bj * PB + c] = -sacc;
    }
    __syncthreads();
  }
  double* Lo = Linv_diag + k * NB * NB;
  for (int i = ty; i < NB; i += 16)
    for (int j = tx; j < NB; j += 16) {
      Lo[i * NB + j] = (j <= i) ? Li[i * LDA + j] : 0.0;
      if (i < b && j <= i) M[(o + i) * d + o + j] = A[i * LDA + j];
    }
  if (tid == 0) {
    if (bad) atomicMax(status, static_cast<int32_t>(TK_E_NOT_SPD));
    // min pivot: monotone update through integer compare of non-negative doubles
    atomicMin(reinterpret_cast<unsigned long long*>(min_pivot),
              static_cast<unsigned long long>(__double_as_longlong(pmin)));
  }
}

// ---- panel: L_ik = A_ik L_kk^{-T} for block rows i > k
__global__ __launch_bounds__(kBlock) void chol_trsm_kernel(double* __restrict__ M, int64_t d,
                                                           int64_t k,
                                                           const double* __restrict__ Linv_diag) {
  __shared__ double Li[NB * LDA];
  __shared__ double A[NB * LDA];
  const int tid = threadIdx.x;
  const int64_t i0 = (k + 1 + blockIdx.x) * NB;
  const int64_t o = k * NB;
  const int rows = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  const double* L = Linv_diag + k * NB * NB;
  for (int e = tid; e < NB * NB; e += kBlock) {
    const int i = e / NB, j = e % NB;
    Li[i * LDA + j] = L[e];
    A[i * LDA + j] = i < rows ? M[(i0 + i) * d + o + j] : 0.0;
  }
  __syncthreads();
  // X[r][c] = sum_{m <= c} A[r][m] Li[c][m]; each thread 4 x 4 outputs
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  double acc[4][4] = {};
  for (int m = 0; m < NB; ++m) {
    double a[4], l[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      a[x] = A[(tr + x) * LDA + m];
      l[x] = Li[(tc + x) * LDA + m];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], l[y], acc[x][y]);
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (tr + x < rows) M[(i0 + tr + x) * d + o + tc + y] = acc[x][y];
}

// ---- trailing update: M_ij -= L_ik L_jk^T for k < j <= i (FP64 MFMA 16x16x4)
__global__ __launch_bounds__(kBlock) void chol_syrk_kernel(double* __restrict__ M, int64_t d,
                                                           int64_t k) {
  __shared__ double La[NB * LDA];
  __shared__ double Lb[NB * LDA];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int64_t tau = blockIdx.x;
  int64_t a = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(tau) + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= tau) ++a;
  while (a * (a + 1) / 2 > tau) --a;
  const int64_t bb = tau - a * (a + 1) / 2;
  const int64_t bi = k + 1 + a, bj = k + 1 + bb;
  const int64_t i0 = bi * NB, j0 = bj * NB, o = k * NB;
  const int ri = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  const int rj = static_cast<int>((d - j0) < NB ? (d - j0) : NB);
  for (int e = tid; e < NB * NB; e += kBlock) {
    const int i = e / NB, j = e % NB;
    La[i * LDA + j] = i < ri ? M[(i0 + i) * d + o + j] : 0.0;
    Lb[i * LDA + j] = i < rj ? M[(j0 + i) * d + o + j] : 0.0;
  }
  __syncthreads();
  // waves 2 x 2, each 32 x 32 = 2 x 2 MFMA 16 x 16 blocks
  const int wr = wave >> 1, wc = wave & 1;
  doublex4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = doublex4{0, 0, 0, 0};
  for (int kk = 0; kk < NB; kk += 4) {
    const int kc = kk + lane / 16;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const double av = La[(wr * 32 + x * 16 + lane % 16) * LDA + kc];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const double bv = Lb[(wc * 32 + y * 16 + lane % 16) * LDA + kc];
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[x][y], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 16x16x4 accumulator: register v of lane l holds row l / 16 + 4 v
        const int r = wr * 32 + x * 16 + lane / 16 + 4 * v;
        const int c = wc * 32 + y * 16 + lane % 16;
        if (r < ri && c < rj && (bi != bj || c <= r)) {
          double* p = &M[(i0 + r) * d + j0 + c];
          *p -= acc[x][y][v];
        }
      }
}

// ---- triangular solves with ticket-ordered block rows
constexpr long kSpinLimit = 1L << 22;

__device__ inline bool wait_flag(const int32_t* f) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > kSpinLimit) return false;
  }
  return true;
}

// forward: L y = b.  flags[0] ticket, flags[2 + i] row-ready flags.
// Thread (r, q): row r of the block row, column quarter q of each dependency
// block.  The L block of the next dependency is loaded before waiting on its
// flag, so a link of the dependency chain costs a flag hop and a few FMAs.
__global__ __launch_bounds__(kBlock) void trsv_lower_kernel(const double* __restrict__ L,
                                                            const double* __restrict__ Linv_diag,
                                                            int64_t d, const double* __restrict__ b,
                                                            double* y, int32_t* flags,
                                                            const int32_t* done, int32_t* status) {
  if (done && *done) return;
  __shared__ int64_t row_blk;
  __shared__ double Li[NB * LDA];
  __shared__ double acc_s[NB];
  __shared__ double part[4][NB];
  __shared__ int ok;
  const int tid = threadIdx.x;
  if (tid == 0) {
    row_blk = atomicAdd(&flags[0], 1);
    ok = 1;
  }
  __syncthreads();
  const int64_t i = row_blk;
  const int64_t i0 = i * NB;
  const int rows = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  const int r = tid & 63, q = tid >> 6;
  {
    const double* src = Linv_diag + i * NB * NB;
    for (int e = tid; e < NB * NB; e += kBlock) Li[(e >> 6) * LDA + (e & 63)] = src[e];
  }
  const double* Lrow = L + (i0 + (r < rows ? r : 0)) * d + q * 16;
  double cur[16], nxt[16];
  if (i > 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) cur[c] = Lrow[c];
  }
  double acc = 0.0;
  for (int64_t j = 0; j < i; ++j) {
    if (j + 1 < i) {
#pragma unroll
      for (int c = 0; c < 16; ++c) nxt[c] = Lrow[(j + 1) * NB + c];
    }
    if (tid == 0 && ok) {
      if (!wait_flag(&flags[2 + j])) ok = 0;
    }
    __syncthreads();
    if (!ok) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const double* yj = y + j * NB + q * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc = fma(cur[c], yj[c], acc);
#pragma unroll
    for (int c = 0; c < 16; ++c) cur[c] = nxt[c];
  }
  part[q][r] = acc;
  __syncthreads();
  if (tid < NB) {
    const double bv = tid < rows ? b[i0 + tid] : 0.0;
    acc_s[tid] = bv - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
  }
  __syncthreads();
  // y_i = Li acc: row r, four partial sums over c
  {
    const int rr = tid >> 2, pp = tid & 3;
    double v = 0.0;
    for (int c = pp; c <= rr; c += 4) v = fma(Li[rr * LDA + c], acc_s[c], v);
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    if (pp == 0 && rr < rows) y[i0 + rr] = v;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_store(&flags[2 + i], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (!ok) atomicMax(status, static_cast<int32_t>(TK_E_HIP));
  }
}

// backward: L^T x = y.  flags[1] ticket, flags[2 + nblk + i] flags.
__global__ __launch_bounds__(kBlock) void trsv_upper_kernel(const double* __restrict__ L,
                                                            const double* __restrict__ Linv_diag,
                                                            int64_t d, int64_t nblk,
                                                            const double* __restrict__ y,
                                                            double* x, int32_t* flags,
                                                            const int32_t* done, int32_t* status) {
  if (done && *done) return;
  __shared__ int64_t row_blk;
  __shared__ double Li[NB * LDA];
  __shared__ double acc_s[NB];
  __shared__ double part[4][NB];
  __shared__ int ok;
  const int tid = threadIdx.x;
  if (tid == 0) {
    row_blk = nblk - 1 - atomicAdd(&flags[1], 1);
    ok = 1;
  }
  __syncthreads();
  const int64_t i = row_blk;
  const int64_t i0 = i * NB;
  const int rows = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  int32_t* fl = flags + 2 + nblk;
  {
    const double* src = Linv_diag + i * NB * NB;
    for (int e = tid; e < NB * NB; e += kBlock) Li[(e >> 6) * LDA + (e & 63)] = src[e];
  }
  // acc[r] = sum_{j > i} sum_c L[j0 + c][i0 + r] x[j0 + c]; thread (r, quarter q of c)
  const int r = tid & 63, q = tid >> 6;
  const int rc = r < rows ? r : 0;
  auto load_blk = [&](int64_t j, double* v) {
    const int64_t j0 = j * NB;
    const int rj = static_cast<int>((d - j0) < NB ? (d - j0) : NB);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = q * 16 + c;
      v[c] = cc < rj ? L[(j0 + cc) * d + i0 + rc] : 0.0;
    }
  };
  double cur[16], nxt[16];
  if (i < nblk - 1) load_blk(nblk - 1, cur);
  double acc = 0.0;
  for (int64_t j = nblk - 1; j > i; --j) {
    if (j - 1 > i) load_blk(j - 1, nxt);
    if (tid == 0 && ok) {
      if (!wait_flag(&fl[j])) ok = 0;
    }
    __syncthreads();
    if (!ok) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int64_t j0 = j * NB;
    const int rj = static_cast<int>((d - j0) < NB ? (d - j0) : NB);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = q * 16 + c;
      if (cc < rj) acc = fma(cur[c], x[j0 + cc], acc);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) cur[c] = nxt[c];
  }
  part[q][r] = acc;
  __syncthreads();
  if (tid < NB) {
    const double yv = tid < rows ? y[i0 + tid] : 0.0;
    acc_s[tid] = yv - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
  }
  __syncthreads();
  // x_i = Li^T acc: x[r] = sum_{c >= r} Li[c][r] acc[c]
  {
    const int rr = tid >> 2, pp = tid & 3;
    double v = 0.0;
    for (int c = rr + pp; c < rows; c += 4) v = fma(Li[c * LDA + rr], acc_s[c], v);
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    if (pp == 0 && rr < rows) x[i0 + rr] = v;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_store(&fl[i], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (!ok) atomicMax(status, static_cast<int32_t>(TK_E_HIP));
  }
}

__global__ void fill_flags_kernel(int32_t* f, int64_t n, const int32_t* done) {
  if (done && *done) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) f[i] = 0;
}

}  // namespace

void launch_cholesky(double* M, int64_t d, double* Linv_diag, double* min_pivot, int32_t* status,
                     hipStream_t st) {
  const int64_t nblk = cdiv(d, NB);
  for (int64_t k = 0; k < nblk; ++k) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(kBlock), 0, st, M, d, k, Linv_diag,
                       min_pivot, status);
    const int64_t below = nblk - k - 1;
    if (below > 0) {
      hipLaunchKernelGGL(chol_trsm_kernel, dim3(static_cast<unsigned>(below)), dim3(kBlock), 0, st,
                         M, d, k, static_cast<const double*>(Linv_diag));
      hipLaunchKernelGGL(chol_syrk_kernel, dim3(static_cast<unsigned>(below * (below + 1) / 2)),
                         dim3(kBlock), 0, st, M, d, k);
    }
  }
}

void launch_chol_solve(const double* L, const double* Linv_diag, int64_t d, double* x,
                       double* y_tmp, int32_t* flags, const int32_t* done, int32_t* status,
                       hipStream_t st) {
  const int64_t nblk = cdiv(d, NB);
  const int64_t nf = 2 * nblk + 2;
  hipLaunchKernelGGL(fill_flags_kernel, dim3(static_cast<unsigned>(cdiv(nf, kBlock))), dim3(kBlock),
                     0, st, flags, nf, done);
  hipLaunchKernelGGL(trsv_lower_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, st, L,
                     Linv_diag, d, static_cast<const double*>(x), y_tmp, flags, done, status);
  hipLaunchKernelGGL(trsv_upper_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, st, L,
                     Linv_diag, d, nblk, static_cast<const double*>(y_tmp), x, flags, done, status);
}

}  // namespace tk
