// FP64 Cholesky factorisation and triangular solves of the sketched system
// (Gram + lambda P) h = rhs.  The proof of Thm 4.2 solves the sketched
// normal equations with a pseudo-inverse; the system here is positive
// definite for lambda > 0, so a Cholesky factorisation is the direct solver.
//
// Left-looking factorisation over 64 x 64 tiles in one persistent launch:
// one workgroup runs the chain of diagonal tiles (factor, inverse, next
// tile) while the others form the remaining tiles and the chain's partial
// sums, each tile written once and published by a flag.  The triangular
// solves use one launch each: workgroups take block rows in ticket order and
// wait (bounded spin) for the values they depend on.
#include "tk_internal.h"

namespace tk {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;
constexpr int NB = kCholNb;
constexpr int LDA = NB + 1;

// ---- diagonal tile: L_kk and its inverse
// Blocked over four 16-column panels.  Wave 0 factors each 16 x 16 diagonal
// panel in registers, lane r owning row r (each 16-lane row of the wave holds a
// copy), with DPP row broadcasts in place of barriers, and eliminates the
// panel's inverse alongside.  The rows below the panel, the trailing triangle
// and the off-diagonal blocks of the 64 x 64 inverse are 16 x 16 FP64 MFMA
// block products, done by the other waves while wave 0 factors the next panel
// where the dependencies allow.
constexpr int PB = 16;

// value of v in lane c of this lane's 16-lane row (c a constant after unrolling):
// the 64-bit DPP row broadcast, one vector move, so the panel factor keeps its
// broadcasts out of scalar registers (no readlane hazards or spills)
template <int C>
__device__ inline double row_bcast(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, 0x150 + C, 0xF, 0xF, true);
}
__device__ inline double row_value(double v, int c) {
  switch (c) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
  }
}

// Newton steps for 1 / sqrt(x) from the hardware estimate y (each step
// doubles the correct bits), in place of a square root followed by IEEE
// divisions on the factorisation's serial chain
__device__ inline double rsqrt_refine(double x, double y) {
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Factor the 16 x 16 diagonal panel at (c0, c0) of A and invert it into Li
// (one wave).  Lane (g, r) = (lane / 16, lane % 16) holds row r of the panel;
// the four 16-lane rows repeat the factorisation, and each eliminates its own
// four columns 4 g .. 4 g + 3 of the inverse: Z, the forward elimination of
// L Z' = I without the final row scaling, so row j of the inverse is
// Z[j] / L[j][j].  The column after the pivot is updated first and its
// reciprocal square root estimate issued before the rest of the pivot's
// updates, which then hide that estimate's latency; the Newton steps follow
// them (the scheduling barriers keep this order).
__device__ __attribute__((always_inline)) inline void panel_factor(double* A, double* Li, int c0,
                                                                  int lane, int* bad_s,
                                                                  double* pmin_s) {
  const int r = lane & 15, g = lane >> 4;
  double a[PB];
#pragma unroll
  for (int c = 0; c < PB; ++c) a[c] = (c <= r) ? A[(c0 + r) * LDA + c0 + c] : 0.0;
  double z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = (4 * g + k == r) ? 1.0 : 0.0;
  double pm = 1e308;
  bool nb_ = false;
  double yr = 1.0;  // 1 / L[r][r]
  double pj = row_value(a[0], 0);
  if (!(pj > 0.0)) {
    nb_ = true;
    pj = 1.0;
  }
  double y = rsqrt_refine(pj, __builtin_amdgcn_rsq(pj));
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    const double ljj = pj * y;
    pm = fmin(pm, ljj);
    const double lj = (r == j) ? ljj : (r > j ? a[j] * y : 0.0);
    a[j] = (r >= j) ? lj : 0.0;
    if (r == j) yr = y;
    double pn = 1.0, yn = 1.0;
    if (j + 1 < PB) {
      // entries above the diagonal (c > r) are never read again and are
      // zeroed when their column is reached, so no select is needed here
      a[j + 1] = fma(-lj, row_value(lj, j + 1), a[j + 1]);
      pn = row_value(a[j + 1], j + 1);
      if (!(pn > 0.0)) {
        nb_ = true;
        pn = 1.0;
      }
      yn = __builtin_amdgcn_rsq(pn);
    }
    __builtin_amdgcn_sched_barrier(0);
    // the broadcasts first, each into its own register, so that they issue
    // back to back instead of each waiting for the previous product
    double bl[PB], bz[4];
#pragma unroll
    for (int c = j + 2; c < PB; ++c) bl[c] = row_value(lj, c);
#pragma unroll
    for (int k = 0; k < 4; ++k) bz[k] = row_value(z[k], j);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = j + 2; c < PB; ++c) a[c] = fma(-lj, bl[c], a[c]);
    // rows below j: Z[r] -= L[r][j] (Z[j] / L[j][j]); Z[j] is final here and
    // zero past column j
    const double mj = (r > j) ? lj * y : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = fma(-mj, bz[k], z[k]);
    __builtin_amdgcn_sched_barrier(0);
    if (j + 1 < PB) {
      y = rsqrt_refine(pn, yn);
      pj = pn;
    }
  }
  if (g == 0) {
#pragma unroll
    for (int c = 0; c < PB; ++c) A[(c0 + r) * LDA + c0 + c] = (c <= r) ? a[c] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) Li[(c0 + r) * LDA + c0 + 4 * g + k] = z[k] * yr;  // row r
  if (lane == 0) {
    if (nb_) *bad_s = 1;
    *pmin_s = fmin(*pmin_s, pm);
  }
}

// rows below panel c0, block at row R: X = A[R.., c0:c0+16] Li_pp^T, written
// over its own operand (the wave reads all of it first)
__device__ inline void rows_below(double* A, const double* Li, int c0, int R, int lr, int lk) {
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < PB / 4; ++kk)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(R + lr) * LDA + c0 + 4 * kk + lk],
                                               Li[(c0 + lr) * LDA + c0 + 4 * kk + lk], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) A[(R + lk + 4 * v) * LDA + c0 + lr] = acc[v];
}

// trailing update of block (R, C) by panel c0: A_RC -= L_R,p L_C,p^T (a
// diagonal block is updated whole; its upper half is never read)
__device__ inline void trail_block(double* A, int c0, int R, int C, int lr, int lk) {
  doublex4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = A[(R + lk + 4 * v) * LDA + C + lr];
#pragma unroll
  for (int kk = 0; kk < PB / 4; ++kk)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-A[(R + lr) * LDA + c0 + 4 * kk + lk],
                                               A[(C + lr) * LDA + c0 + 4 * kk + lk], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) A[(R + lk + 4 * v) * LDA + C + lr] = acc[v];
}

// off-diagonal block (bi, bj) of the inverse, Li_ij = -Li_ii sum_{q=j}^{i-1} L_iq Li_qj,
// from the finished block rows of L and earlier block rows of the inverse
__device__ inline void inv_block(const double* A, double* Li, int bi, int bj, int lr, int lk) {
  doublex4 sacc = {0.0, 0.0, 0.0, 0.0};
  for (int q = bj; q < bi; ++q)
#pragma unroll
    for (int kk = 0; kk < PB / 4; ++kk)
      sacc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(bi * PB + lr) * LDA + q * PB + 4 * kk + lk],
                                                  Li[(q * PB + 4 * kk + lk) * LDA + bj * PB + lr],
                                                  sacc, 0, 0, 0);
  // the accumulator's register v holds row 4 v + lk of the sum in lane
  // (lk, lr): exactly the B operand of the k-slice v
  doublex4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < PB / 4; ++kk)
    o = __builtin_amdgcn_mfma_f64_16x16x4f64(-Li[(bi * PB + lr) * LDA + bi * PB + 4 * kk + lk],
                                             sacc[kk], o, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) Li[(bi * PB + lk + 4 * v) * LDA + bj * PB + lr] = o[v];
}

// Factor and invert the 64 x 64 block held in LDS A (lower triangle; rows past
// the matrix hold the identity): on return A holds L and Li holds L^{-1}.
// Li must be zero and *bad / *pmin initialised.  Entries of A above the
// diagonal are scratch (never read).
//
// Blocked over four 16-column panels p.  Wave 0 factors panel p while waves
// 1..3 finish what panel p - 1 left: its trailing update (all blocks but the
// next diagonal one, which wave 0 updated itself right after the rows below)
// and block row p - 1 of the inverse.  Then the rows below panel p are
// 16 x 16 FP64 MFMA products, one block per wave.  Each phase touches blocks
// the concurrent one does not, and a barrier separates a block's producer from
// its readers.
__device__ __attribute__((always_inline)) inline void diag_factor(double* A, double* Li, int* bad_s,
                                                                double* pmin_s) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // FP64 MFMA 16x16x4 operand lanes: row / column lr, k-slice lk; accumulator
  // register v holds row lk + 4 v, column lr
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int NP = NB / PB;
  for (int p = 0; p < NP; ++p) {
    const int c0 = p * PB;
    if (wave == 0) {
      panel_factor(A, Li, c0, lane, bad_s, pmin_s);
    } else if (p > 0) {
      // panel p - 1's trailing blocks (i, j), p <= j <= i < NP, but (p, p);
      // then the blocks (p - 1, bj), bj < p - 1, of the inverse
      const int m = NP - p;
      const int ntr = m * (m + 1) / 2 - 1;
      const int nitems = ntr + (p - 1);
      for (int t = wave - 1; t < nitems; t += kBlock / 64 - 1) {
        if (t < ntr) {
          const int u = t + 1;
          int i = 0;
          while ((i + 1) * (i + 2) / 2 <= u) ++i;
          const int j = u - i * (i + 1) / 2;
          trail_block(A, c0 - PB, c0 + i * PB, c0 + j * PB, lr, lk);
        } else {
          inv_block(A, Li, p - 1, t - ntr, lr, lk);
        }
      }
    }
    __syncthreads();
    const int nbl = NP - 1 - p;  // 16-row blocks below the panel
    if (nbl > 0) {
      if (wave < nbl) rows_below(A, Li, c0, c0 + PB + wave * PB, lr, lk);
      __syncthreads();
      // the next diagonal block, which the next panel factor needs first
      if (wave == 0) trail_block(A, c0, c0 + PB, c0 + PB, lr, lk);
    }
  }
  // the last block row of the inverse
  if (wave < NP - 1) inv_block(A, Li, NP - 1, wave, lr, lk);
  __syncthreads();
}

// acc (2 x 2 blocks of 16 x 16 per wave, FP64 MFMA 16x16x4) = X Y^T over 64
// columns, X and Y 64 x 64 in LDS (row stride LDA)
__device__ inline void tile_gemm_nt(const double* X, const double* Y, doublex4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = doublex4{0, 0, 0, 0};
  for (int kk = 0; kk < NB; kk += 4) {
    const int kc = kk + lane / 16;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const double av = X[(wr * 32 + x * 16 + lane % 16) * LDA + kc];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const double bv = Y[(wc * 32 + y * 16 + lane % 16) * LDA + kc];
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[x][y], 0, 0, 0);
      }
    }
  }
}

// (row, col) of accumulator register v of block (x, y): FP64 16x16x4 puts
// row l / 16 + 4 v, column l % 16 of the 16 x 16 block in lane l
__device__ inline int acc_r(int x, int v) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 32 + x * 16 + lane / 16 + 4 * v;
}
__device__ inline int acc_c(int y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 32 + y * 16 + lane % 16;
}

// ---- left-looking dataflow factorisation in one persistent launch
// With S_ij = A_ij - sum_{k < j} L_ik L_jk^T over lower 64 x 64 tiles:
//  * the workgroup that starts first (ticket 0) runs the chain of the
//    factorisation, column by column: S_jj
//    (its last term L_{j,j-1} L_{j,j-1}^T from the tile it made itself, still in
//    LDS), the factor and inverse of S_jj, then the next tile
//    L_{j+1,j} = S_{j+1,j} L_jj^{-T}, which it keeps in LDS for the next column;
//    both tiles are published together;
//  * the other workgroups take tickets, column by column j, for the tiles
//    L_ij = S_ij L_jj^{-T}, i >= j + 2, then for the finished S_{j+2,j+1} (its
//    last term, with the chain's tile L_{j+1,j}) and for the partial sums of
//    column j + 2 (S_{j+2,j+2} and S_{j+3,j+2} over k <= j), all left in a
//    scratch area for the chain.
// Each tile is written once, then its flag is raised; published tiles are read
// with agent-scope coherent loads, so no cache invalidation is needed.  A
// ticketed task waits only on smaller tickets or on chain tiles of earlier
// columns, and the chain at column j only on tickets of columns j - 2 and
// j - 1.  Tickets are taken when a workgroup starts, so every wait is on a
// workgroup that is already running and never gives up its compute unit:
// the launch drains whatever the dispatch order or the number of co-resident
// workgroups.  Every wait is still bounded (TK_E_HIP past the limit, the task
// then goes on).
constexpr int kFlagStride = 32;  // one flag per 128-byte line
__device__ inline int64_t tile_flag_index(int64_t i, int64_t j) {
  return (i * (i + 1) / 2 + j) * kFlagStride;
}

// Bounded wait for a published tile: relaxed agent-scope polls, spaced out.
// The limit (~2^18 polls of ~0.2 us) is far above the longest legitimate wait
// (the chain's progress over all columns, a few ms); the first wait to run out
// raises *abort, which ends every other wait of the launch at once.
constexpr long kFlowSpinLimit = 1L << 18;
__device__ inline bool wait_tile(const int32_t* f, int32_t* abort) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(8);
    if (++spins > kFlowSpinLimit) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// A published tile entry: read coherently at agent scope (no cached copy from
// before the tile's flag).
__device__ inline double load_tile(const double* p) {
  return __longlong_as_double(static_cast<long long>(__hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}

// dst (64 x 64 in LDS, row stride LDA) = rows [r0, r0 + rows) of column block k
// of M, zero past `rows`
__device__ inline void stage_tile(const double* M, int64_t d, int64_t r0, int rows, int64_t k,
                                  double* dst) {
  const int tid = threadIdx.x;
  double v[NB * NB / kBlock];
#pragma unroll
  for (int q = 0; q < NB * NB / kBlock; ++q) {
    const int e = tid + q * kBlock;
    const int r = e / NB, c = e % NB;
    v[q] = load_tile(&M[(r0 + (r < rows ? r : rows - 1)) * d + k * NB + c]);
  }
#pragma unroll
  for (int q = 0; q < NB * NB / kBlock; ++q) {
    const int e = tid + q * kBlock;
    const int r = e / NB, c = e % NB;
    dst[r * LDA + c] = r < rows ? v[q] : 0.0;
  }
}

// S (accumulator layout) -= X Y^T, X and Y 64 x 64 in LDS
__device__ inline void sub_gemm_nt(const double* X, const double* Y, double (&S)[2][2][4]) {
  doublex4 acc[2][2];
  tile_gemm_nt(X, Y, acc);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) S[x][y][v] -= acc[x][y][v];
}

// S = A_ij (rows / columns clamped; entries past them are never used)
__device__ inline void load_block(const double* M, int64_t d, int64_t i0, int ri, int64_t j0,
                                  int rj, double (&S)[2][2][4]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_r(x, v), c = acc_c(y);
        S[x][y][v] = M[(i0 + (r < ri ? r : ri - 1)) * d + j0 + (c < rj ? c : rj - 1)];
      }
}

// Published data is stored with agent-scope atomic stores, which write through
// this XCD's L2 to the device's coherence point, and read with agent-scope
// atomic loads (load_tile).  Such a store is visible to every reader once it has
// completed, so a publisher waits for its own stores to complete (s_waitcnt) and
// then raises the flag: no L2 writeback fence is needed, which would write back
// every dirty line of the XCD's L2 at each publication.
__device__ inline void pub_store(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// M rows [i0, i0 + ri) of column block j = S Li^T, S in the accumulator layout
// staged through X; Li (64 x 64) in LDS
__device__ inline void apply_inverse_store(double* M, int64_t d, int64_t i0, int ri, int64_t j0,
                                           const double (&S)[2][2][4], double* X,
                                           const double* Li) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_r(x, v), c = acc_c(y);
        X[r * LDA + c] = r < ri ? S[x][y][v] : 0.0;
      }
  __syncthreads();
  doublex4 acc[2][2];
  tile_gemm_nt(X, Li, acc);  // sum_m S[r][m] Li[c][m]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_r(x, v), c = acc_c(y);
        if (r < ri) pub_store(&M[(i0 + r) * d + j0 + c], acc[x][y][v]);
      }
}

// Wait until every memory operation this wave issued has completed.
__device__ inline void complete_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Raise a tile's flag once every thread's (write-through) stores to it completed.
__device__ inline void publish_tile(int32_t* flag) {
  complete_stores();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// tickets of column j: tiles (i, j) for i >= j + 2, then the finished
// S_{j+2,j+1} and the partial sums of column j + 2
__host__ __device__ inline int64_t chol_column_tickets(int64_t nblk, int64_t j) {
  const int64_t tiles = nblk - j - 2 > 0 ? nblk - j - 2 : 0;
  return tiles + (j + 2 < nblk ? 2 : 0);
}
__host__ __device__ inline int64_t chol_flow_tasks(int64_t nblk) {
  int64_t n = 0;
  for (int64_t j = 0; j < nblk; ++j) n += chol_column_tickets(nblk, j);
  return n;
}

// S (accumulator layout) as a row-major 64 x 64 tile in device memory, published
// with write-through stores (rows past `rows` zero)
__device__ inline void store_block_pub(double* dst, int ld, int rows, const double (&S)[2][2][4]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_r(x, v), c = acc_c(y);
        pub_store(&dst[r * ld + c], r < rows ? S[x][y][v] : 0.0);
      }
}

// S (accumulator layout) as a row-major 64 x 64 tile (rows past `rows` zero)
__device__ inline void store_block(double* dst, int ld, int rows, const double (&S)[2][2][4]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_r(x, v), c = acc_c(y);
        dst[r * ld + c] = r < rows ? S[x][y][v] : 0.0;
      }
}

// pre: scratch; column c's partial sums at blocks 2c (S_cc) and 2c + 1
// (S_{c+1,c}, then finished in place)
__global__ __launch_bounds__(kBlock, 1) void chol_flow_kernel(double* __restrict__ M, int64_t d,
                                                              int64_t nblk,
                                                              double* __restrict__ Linv_diag,
                                                              double* __restrict__ pre,
                                                              double* min_pivot, int32_t* status,
                                                              int32_t* flags,
                                                              const int32_t* skip) {
  if (skip && *skip != 0) return;  // the system was already solved
  __shared__ double smem[4 * NB * LDA];
  double* La = smem;
  double* Lb = smem + NB * LDA;
  double* Lc = smem + 2 * NB * LDA;
  double* Ld = smem + 3 * NB * LDA;
  __shared__ int64_t task_s;
  __shared__ int bad;
  __shared__ double pmin;
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  int32_t* tile_flag = flags + kFlagStride;  // flags[0] is the ticket, flags[1] the abort word
  int32_t* pre_flag = tile_flag + (nblk * (nblk + 1) / 2) * kFlagStride;
  int32_t* post_flag = pre_flag + nblk * kFlagStride;  // S_{c+1,c} finished
  bool failed = false;
  auto rows_of = [&](int64_t b) {
    return static_cast<int>((d - b * NB) < NB ? (d - b * NB) : NB);
  };
  // tid 0 waits for the flags, then the workgroup goes on together
  int32_t* abort = flags + 1;  // in the ticket's line
  auto wait2 = [&](const int32_t* fa, const int32_t* fb) {
    if (tid == 0)
      ok_s = (wait_tile(fa, abort) && (fb == nullptr || wait_tile(fb, abort))) ? 1 : 0;
    __syncthreads();
    failed = failed || !ok_s;
  };
  // Roles come from the ticket counter, in the order workgroups start: ticket 0
  // runs the chain, ticket k >= 1 runs task k - 1.  Every wait is then on work
  // held by a workgroup that has already started (the chain, or a smaller
  // ticket), never on one that may still be queued for a compute unit.
  if (tid == 0) task_s = atomicAdd(&flags[0], 1);
  __syncthreads();
  if (task_s == 0) {
    // ---------------- the chain (Lc holds L_{j,j-1} from the previous column)
    __builtin_amdgcn_s_setprio(3);
    double Sd_next[2][2][4];  // partial sums of the next diagonal tile
    for (int64_t j = 0; j < nblk; ++j) {
      const int64_t j0 = j * NB;
      const int rj = rows_of(j);
      const bool next = j + 1 < nblk;
      const int64_t i10 = (j + 1) * NB;
      const int r1 = next ? rows_of(j + 1) : 0;
      double Sd[2][2][4];
      if (j >= 2) {
        // loaded during the previous column (with its S_{j,j-1})
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) Sd[x][y][v] = Sd_next[x][y][v];
      } else {
        load_block(M, d, j0, rj, j0, rj, Sd);
      }
      if (j >= 1) sub_gemm_nt(Lc, Lc, Sd);  // L_{j,j-1} L_{j,j-1}^T
      // factor and invert S_jj (rows past d hold the identity)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = acc_r(x, v), c = acc_c(y);
            La[r * LDA + c] = (r < rj && c <= r) ? Sd[x][y][v] : (r == c ? 1.0 : 0.0);
            Lb[r * LDA + c] = 0.0;
          }
      if (tid == 0) {
        bad = 0;
        pmin = 1e308;
      }
      __syncthreads();
      diag_factor(La, Lb, &bad, &pmin);
      {
        // this thread's entries (ty + 16 a, tx + 16 b): all LDS reads first,
        // then the stores
        double* Lo = Linv_diag + j * NB * NB;
        double lo_v[4][4], m_v[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int r = ty + 16 * a, c = tx + 16 * b;
            lo_v[a][b] = (c <= r) ? Lb[r * LDA + c] : 0.0;
            m_v[a][b] = La[r * LDA + c];
          }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int r = ty + 16 * a;
          double* Mrow = M + (j0 + r) * d + j0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int c = tx + 16 * b;
            pub_store(&Lo[r * NB + c], lo_v[a][b]);
            if (r < rj && c <= r) pub_store(&Mrow[c], m_v[a][b]);
          }
        }
      }
      if (tid == 0) {
        if (bad) atomicMax(status, static_cast<int32_t>(TK_E_NOT_SPD));
        atomicMin(reinterpret_cast<unsigned long long*>(min_pivot),
                  static_cast<unsigned long long>(__double_as_longlong(pmin)));
      }
      if (!next) {
        publish_tile(&tile_flag[tile_flag_index(j, j)]);
        break;
      }
      // S_{j+1,j}: A_{1,0}, or the scratch block its ticketed task finished
      double Sn[2][2][4];
      if (j >= 1) wait2(&post_flag[j * kFlagStride], nullptr);
      // (j, j) is published now (its stores have had the wait to complete), so
      // that the tiles of column j start before this column's last tile
      publish_tile(&tile_flag[tile_flag_index(j, j)]);
      if (j >= 1) {
        const double* P1 = pre + (2 * j + 1) * NB * NB;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              Sn[x][y][v] = load_tile(&P1[acc_r(x, v) * NB + acc_c(y)]);
      } else {
        load_block(M, d, i10, r1, j0, rj, Sn);
      }
      // L_{j+1,j} = S_{j+1,j} Li_jj^T: stored, kept in Lc, published as (j + 1, j)
      __syncthreads();  // every wave is done reading Lc (the previous tile)
      store_block(Ld, LDA, r1, Sn);
      __syncthreads();
      doublex4 acc[2][2];
      tile_gemm_nt(Ld, Lb, acc);
      if (j >= 1) {
        // the partial sums of S_{j+1,j+1}: their loads complete with this
        // tile's stores below
        wait2(&pre_flag[(j + 1) * kFlagStride], nullptr);
        const double* P0 = pre + (2 * (j + 1)) * NB * NB;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              Sd_next[x][y][v] = load_tile(&P0[acc_r(x, v) * NB + acc_c(y)]);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = acc_r(x, v), c = acc_c(y);
            const double val = r < r1 ? acc[x][y][v] : 0.0;
            Lc[r * LDA + c] = val;
            if (r < r1) pub_store(&M[(i10 + r) * d + j0 + c], val);
          }
      complete_stores();
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(&tile_flag[tile_flag_index(j + 1, j)], 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  } else {
    // ---------------- ticketed tasks
    const int64_t ntasks = chol_flow_tasks(nblk);
    for (bool first = true;; first = false) {
      if (!first) {
        __syncthreads();  // the previous task is done with LDS and task_s
        if (tid == 0) task_s = atomicAdd(&flags[0], 1);
        __syncthreads();
      }
      const int64_t t = task_s - 1;
      if (t >= ntasks) break;
      int64_t j = 0, start = 0;
      for (;;) {
        const int64_t cnt = chol_column_tickets(nblk, j);
        if (t < start + cnt) break;
        start += cnt;
        ++j;
      }
      const int64_t off = t - start;
      const int64_t ntile = nblk - j - 2 > 0 ? nblk - j - 2 : 0;
      if (off == ntile) {
        // finished S_{c+1,c}, c = j + 1: its partial sums (or A for c = 1) minus
        // L_{c+1,j} L_{c,j}^T, the second tile being the chain's
        const int64_t c = j + 1, c0 = c * NB, n0 = (c + 1) * NB;
        const int rc = rows_of(c), rn = rows_of(c + 1);
        double* P1 = pre + (2 * c + 1) * NB * NB;
        double S[2][2][4];
        if (c >= 2) {
          wait2(&pre_flag[c * kFlagStride], nullptr);
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                S[x][y][v] = load_tile(&P1[acc_r(x, v) * NB + acc_c(y)]);
        } else {
          load_block(M, d, n0, rn, c0, rc, S);
        }
        wait2(&tile_flag[tile_flag_index(c + 1, j)], &tile_flag[tile_flag_index(c, j)]);
        stage_tile(M, d, n0, rn, j, La);
        stage_tile(M, d, c0, rc, j, Lb);
        __syncthreads();
        sub_gemm_nt(La, Lb, S);
        store_block_pub(P1, NB, NB, S);
        publish_tile(&post_flag[c * kFlagStride]);
      } else if (off < ntile) {
        // tile (i, j), i >= j + 2 (block j is full)
        const int64_t i = j + 2 + off, i0 = i * NB, j0 = j * NB;
        const int ri = rows_of(i);
        double S[2][2][4];
        load_block(M, d, i0, ri, j0, NB, S);
        for (int64_t k = 0; k < j; ++k) {
          wait2(&tile_flag[tile_flag_index(i, k)], &tile_flag[tile_flag_index(j, k)]);
          stage_tile(M, d, i0, ri, k, La);
          stage_tile(M, d, j0, NB, k, Lb);
          __syncthreads();
          sub_gemm_nt(La, Lb, S);
          __syncthreads();
        }
        wait2(&tile_flag[tile_flag_index(j, j)], nullptr);
        {
          const double* Li = Linv_diag + j * NB * NB;
          double vl[NB * NB / kBlock];
#pragma unroll
          for (int q = 0; q < NB * NB / kBlock; ++q) vl[q] = load_tile(&Li[tid + q * kBlock]);
#pragma unroll
          for (int q = 0; q < NB * NB / kBlock; ++q) {
            const int e = tid + q * kBlock;
            Lb[(e / NB) * LDA + e % NB] = vl[q];
          }
        }
        apply_inverse_store(M, d, i0, ri, j0, S, La, Lb);
        publish_tile(&tile_flag[tile_flag_index(i, j)]);
      } else {
        // partial sums of column c = j + 2 over k <= j
        const int64_t c = j + 2, c0 = c * NB;
        const int rc = rows_of(c);
        const bool next = c + 1 < nblk;
        const int64_t n0 = (c + 1) * NB;
        const int rn = next ? rows_of(c + 1) : 0;
        double Sd[2][2][4], Sn[2][2][4];
        load_block(M, d, c0, rc, c0, rc, Sd);
        if (next) load_block(M, d, n0, rn, c0, rc, Sn);
        for (int64_t k = 0; k <= j; ++k) {
          wait2(&tile_flag[tile_flag_index(c, k)],
                next ? &tile_flag[tile_flag_index(c + 1, k)] : nullptr);
          stage_tile(M, d, c0, rc, k, La);
          if (next) stage_tile(M, d, n0, rn, k, Lb);
          __syncthreads();
          sub_gemm_nt(La, La, Sd);
          if (next) sub_gemm_nt(Lb, La, Sn);
          __syncthreads();
        }
        store_block_pub(pre + (2 * c) * NB * NB, NB, NB, Sd);
        if (next) store_block_pub(pre + (2 * c + 1) * NB * NB, NB, NB, Sn);
        publish_tile(&pre_flag[c * kFlagStride]);
      }
    }
  }
  if (tid == 0 && failed) atomicMax(status, static_cast<int32_t>(TK_E_HIP));
}

int chol_flow_grid(int64_t nblk, int max_grid) {
  const int cus = device_cu_count();
  const int64_t ntasks = chol_flow_tasks(nblk);
  int64_t g = cus;  // one workgroup per CU: the serial panel factor keeps its SIMD
  if (max_grid > 0 && max_grid < g) g = max_grid < 2 ? 2 : max_grid;
  return static_cast<int>(1 + ntasks < g ? 1 + ntasks : g);  // the chain + ticketed tasks
}

__global__ void chol_flags_kernel(int32_t* f, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) f[i] = 0;
}

// ---- triangular solves with ticket-ordered block rows
// Workgroups take 64-row blocks in ticket order.  A solved block is published
// by storing its values (agent-scope atomic stores) over a sentinel that no
// arithmetic produces; a consumer thread polls exactly the 16 values it needs
// (agent-scope atomic loads), so a link of the dependency chain costs one
// visibility hop and the block's own work -- no flag, fence or barrier.
// Waits are bounded: after kSpinLimit polls a block reports TK_E_HIP and
// uses 0, so every workgroup still finishes and publishes.
constexpr long kSpinLimit = 1L << 22;
constexpr unsigned long long kPending = kSolvePending;

// v[c] = p[c] for c < n (0 beyond), waiting until all n are published
__device__ inline bool load_published(const double* p, int n, double* v) {
  long spins = 0;
  bool pending = true;
  while (pending) {
    pending = false;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const unsigned long long u =
          c < n ? __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p + c),
                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                : 0ull;
      pending = pending || (u == kPending);
      v[c] = __longlong_as_double(static_cast<long long>(u));
    }
    if (pending) {
      if (++spins > kSpinLimit) {
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0.0;
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return true;
}

// The chain matrices of the two solves, one pair per 64-row block i (their
// last dependency folded into one product, so that a block finishes the rest
// of its row before that dependency is published):
//   forward  y_i = Li_ii (b_i - sum_{j < i-1} L_ij y_j) - Wl_i y_{i-1},  Wl_i = Li_ii L_{i,i-1}
//   backward x_i = Li_ii^T (y_i - sum_{j > i+1} L_ji^T x_j) - Wu_i x_{i+1},
//            Wu_i = Li_ii^T L_{i+1,i}^T
// Both 64 x 64 products per block on FP64 MFMA, stored row-major after the
// diagonal-block inverses (Wl at nblk blocks past Linv_diag, Wu at 2 nblk).
__global__ __launch_bounds__(kBlock) void chol_chain_kernel(const double* __restrict__ M,
                                                            int64_t d, int64_t nblk,
                                                            double* __restrict__ Linv_diag,
                                                            const int32_t* skip) {
  if (skip && *skip != 0) return;
  __shared__ double X[NB * LDA];
  __shared__ double Y[NB * LDA];
  const int tid = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int64_t i0 = i * NB;
  const double* Li = Linv_diag + i * NB * NB;
  auto store = [&](double* W, const doublex4 (&acc)[2][2]) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) W[acc_r(x, v) * NB + acc_c(y)] = acc[x][y][v];
  };
  if (i >= 1) {
    // X = Li_ii, Y[c][m] = L_{i,i-1}[m][c] (rows past d are zero)
    const int ri = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
    for (int e = tid; e < NB * NB; e += kBlock) {
      const int r = e >> 6, c = e & 63;
      X[r * LDA + c] = Li[e];
      Y[c * LDA + r] = r < ri ? M[(i0 + r) * d + i0 - NB + c] : 0.0;
    }
    __syncthreads();
    doublex4 acc[2][2];
    tile_gemm_nt(X, Y, acc);
    store(Linv_diag + (nblk + i) * NB * NB, acc);
    __syncthreads();
  }
  if (i + 1 < nblk) {
    // X[r][m] = Li_ii[m][r], Y[c][m] = L_{i+1,i}[c][m] (rows past d are zero)
    const int64_t n0 = i0 + NB;
    const int rn = static_cast<int>((d - n0) < NB ? (d - n0) : NB);
    for (int e = tid; e < NB * NB; e += kBlock) {
      const int r = e >> 6, c = e & 63;
      X[c * LDA + r] = Li[e];
      Y[r * LDA + c] = r < rn ? M[(n0 + r) * d + i0 + c] : 0.0;
    }
    __syncthreads();
    doublex4 acc[2][2];
    tile_gemm_nt(X, Y, acc);
    store(Linv_diag + (2 * nblk + i) * NB * NB, acc);
  }
}

// forward: L y = b, b read from x; x is left holding the sentinel for the
// backward solve.  flags[0] is the ticket.  Thread (r, q): row r of the block,
// column quarter q of each dependency block and of the chain product.
__global__ __launch_bounds__(kBlock) void trsv_lower_kernel(const double* __restrict__ L,
                                                            const double* __restrict__ Linv_diag,
                                                            int64_t d, int64_t nblk, double* x,
                                                            double* y, int32_t* flags,
                                                            const int32_t* done, int32_t* status) {
  if (done && *done) return;
  __shared__ int64_t row_blk;
  __shared__ double Li[NB * LDA];
  __shared__ double acc_s[NB];
  __shared__ double part[4][NB];
  __shared__ double u_s[NB];
  __shared__ double chain[4][NB];
  const int tid = threadIdx.x;
  if (tid == 0) row_blk = atomicAdd(&flags[0], 1);
  __syncthreads();
  const int64_t i = row_blk;
  const int64_t i0 = i * NB;
  const int rows = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  const int r = tid & 63, q = tid >> 6;
  // this thread's part of the chain matrix Wl_i: row r, columns of quarter q
  double wrow[16];
  if (i >= 1) {
    const double* W = Linv_diag + (nblk + i) * NB * NB + r * NB + q * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) wrow[c] = W[c];
  }
  {
    const double* src = Linv_diag + i * NB * NB;
    for (int e = tid; e < NB * NB; e += kBlock) Li[(e >> 6) * LDA + (e & 63)] = src[e];
  }
  const double bv = (q == 0 && r < rows) ? x[i0 + r] : 0.0;
  const double* Lrow = L + (i0 + (r < rows ? r : 0)) * d + q * 16;
  double cur[16], nxt[16];
  if (i > 1) {
#pragma unroll
    for (int c = 0; c < 16; ++c) cur[c] = Lrow[c];
  }
  double acc = 0.0;
  bool ok = true;
  for (int64_t j = 0; j + 1 < i; ++j) {  // every dependency but the last (all full blocks)
    if (j + 2 < i) {
#pragma unroll
      for (int c = 0; c < 16; ++c) nxt[c] = Lrow[(j + 1) * NB + c];
    }
    double yv[16];
    ok = load_published(y + j * NB + q * 16, 16, yv) && ok;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc = fma(cur[c], yv[c], acc);
#pragma unroll
    for (int c = 0; c < 16; ++c) cur[c] = nxt[c];
  }
  part[q][r] = acc;
  __syncthreads();
  if (tid < NB) acc_s[tid] = bv - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
  if (q == 0 && r < rows) pub_store(x + i0 + r, __longlong_as_double(kPending));
  __syncthreads();
  // u = Li acc: row rr, four partial sums over c
  {
    const int rr = tid >> 2, pp = tid & 3;
    double u = 0.0;
    for (int c = pp; c <= rr; c += 4) u = fma(Li[rr * LDA + c], acc_s[c], u);
    u += __shfl_xor(u, 1, 64);
    u += __shfl_xor(u, 2, 64);
    if (pp == 0) u_s[rr] = u;
  }
  // y_i = u - Wl_i y_{i-1} once block i - 1 is published: each wave waits for
  // its own quarter of y_{i-1}
  double v = 0.0;
  if (i >= 1) {
    double yv[16];
    ok = load_published(y + (i - 1) * NB + q * 16, 16, yv) && ok;
#pragma unroll
    for (int c = 0; c < 16; ++c) v = fma(wrow[c], yv[c], v);
  }
  chain[q][r] = v;
  __syncthreads();
  if (q == 0 && r < rows)
    pub_store(y + i0 + r, u_s[r] - ((chain[0][r] + chain[1][r]) + (chain[2][r] + chain[3][r])));
  if (!ok) atomicMax(status, static_cast<int32_t>(TK_E_HIP));
}

// backward: L^T x = y.  flags[1] is the ticket (blocks from the last).
__global__ __launch_bounds__(kBlock) void trsv_upper_kernel(const double* __restrict__ L,
                                                            const double* __restrict__ Linv_diag,
                                                            int64_t d, int64_t nblk,
                                                            const double* __restrict__ y,
                                                            double* x, int32_t* flags,
                                                            const int32_t* done, int32_t* status,
                                                            double* accum) {
  if (done && *done) return;
  __shared__ int64_t row_blk;
  __shared__ double Li[NB * LDA];
  __shared__ double acc_s[NB];
  __shared__ double part[4][NB];
  __shared__ double u_s[NB];
  __shared__ double chain[4][NB];
  const int tid = threadIdx.x;
  if (tid == 0) row_blk = nblk - 1 - atomicAdd(&flags[1], 1);
  __syncthreads();
  const int64_t i = row_blk;
  const int64_t i0 = i * NB;
  const int rows = static_cast<int>((d - i0) < NB ? (d - i0) : NB);
  const int r = tid & 63, q = tid >> 6;
  // this thread's part of the chain matrix Wu_i: row r, columns of quarter q
  double wrow[16];
  if (i + 1 < nblk) {
    const double* W = Linv_diag + (2 * nblk + i) * NB * NB + r * NB + q * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) wrow[c] = W[c];
  }
  {
    const double* src = Linv_diag + i * NB * NB;
    for (int e = tid; e < NB * NB; e += kBlock) Li[(e >> 6) * LDA + (e & 63)] = src[e];
  }
  // acc[r] = sum_{j > i+1} sum_c L[j0 + c][i0 + r] x[j0 + c]; thread (r, quarter q of c)
  const int rc = r < rows ? r : 0;
  auto load_blk = [&](int64_t j, double* v) {
    const int64_t j0 = j * NB;
    const int rj = static_cast<int>((d - j0) < NB ? (d - j0) : NB);
    double t[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = q * 16 + c;
      t[c] = L[(j0 + (cc < rj ? cc : rj - 1)) * d + i0 + rc];
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = (q * 16 + c) < rj ? t[c] : 0.0;
  };
  auto published_count = [&](int64_t j, int quarter) {
    const int64_t j0 = j * NB;
    const int rj = static_cast<int>((d - j0) < NB ? (d - j0) : NB);
    const int n = rj - quarter * 16;
    return n < 0 ? 0 : (n > 16 ? 16 : n);
  };
  double cur[16], nxt[16];
  if (i + 2 < nblk) load_blk(nblk - 1, cur);
  double acc = 0.0;
  bool ok = true;
  for (int64_t j = nblk - 1; j > i + 1; --j) {  // every dependency but the last
    if (j - 1 > i + 1) load_blk(j - 1, nxt);
    double xv[16];
    ok = load_published(x + j * NB + q * 16, published_count(j, q), xv) && ok;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc = fma(cur[c], xv[c], acc);
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
  // u = Li^T acc: u[rr] = sum_{c >= rr} Li[c][rr] acc[c]
  {
    const int rr = tid >> 2, pp = tid & 3;
    double u = 0.0;
    for (int c = rr + pp; c < rows; c += 4) u = fma(Li[c * LDA + rr], acc_s[c], u);
    u += __shfl_xor(u, 1, 64);
    u += __shfl_xor(u, 2, 64);
    if (pp == 0) u_s[rr] = u;
  }
  // x_i = u - Wu_i x_{i+1} once block i + 1 is published: each wave waits for
  // its own quarter of x_{i+1}
  double v = 0.0;
  if (i + 1 < nblk) {
    double xv[16];
    ok = load_published(x + (i + 1) * NB + q * 16, published_count(i + 1, q), xv) && ok;
#pragma unroll
    for (int c = 0; c < 16; ++c) v = fma(wrow[c], xv[c], v);
  }
  chain[q][r] = v;
  __syncthreads();
  if (q == 0 && r < rows) {
    const double xv = u_s[r] - ((chain[0][r] + chain[1][r]) + (chain[2][r] + chain[3][r]));
    pub_store(x + i0 + r, xv);
    if (accum) accum[i0 + r] += xv;
  }
  if (!ok) atomicMax(status, static_cast<int32_t>(TK_E_HIP));
}

// tickets to 0 and y to the sentinel
__global__ void solve_init_kernel(int32_t* flags, double* y, int64_t d, const int32_t* done) {
  if (done && *done) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < 2) flags[i] = 0;
  if (i < d) y[i] = __longlong_as_double(static_cast<long long>(kPending));
}

}  // namespace

void launch_cholesky(double* M, int64_t d, double* Linv_diag, double* min_pivot, int32_t* status,
                     int32_t* flags, hipStream_t st, int max_grid, const int32_t* skip) {
  const int64_t nblk = cdiv(d, NB);
  int32_t* ff = flags + 2;  // flags[0..1] are the solves' tickets
  const int64_t nflags = (1 + nblk * (nblk + 1) / 2 + 2 * nblk) * kFlagStride;
  hipLaunchKernelGGL(chol_flags_kernel, dim3(static_cast<unsigned>(cdiv(nflags, kBlock))),
                     dim3(kBlock), 0, st, ff, nflags);
  double* pre = Linv_diag + 3 * nblk * NB * NB;  // past the inverses and chain matrices
  hipLaunchKernelGGL(chol_flow_kernel, dim3(static_cast<unsigned>(chol_flow_grid(nblk, max_grid))),
                     dim3(kBlock), 0, st, M, d, nblk, Linv_diag, pre, min_pivot, status, ff, skip);
  hipLaunchKernelGGL(chol_chain_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, st,
                     static_cast<const double*>(M), d, nblk, Linv_diag, skip);
}

void launch_chol_solve(const double* L, const double* Linv_diag, int64_t d, double* x,
                       double* y_tmp, int32_t* flags, const int32_t* done, int32_t* status,
                       hipStream_t st, double* accum, bool prepared) {
  const int64_t nblk = cdiv(d, NB);
  if (!prepared)
    hipLaunchKernelGGL(solve_init_kernel, dim3(static_cast<unsigned>(cdiv(d, kBlock))),
                       dim3(kBlock), 0, st, flags, y_tmp, d, done);
  hipLaunchKernelGGL(trsv_lower_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, st, L,
                     Linv_diag, d, nblk, x, y_tmp, flags, done, status);
  hipLaunchKernelGGL(trsv_upper_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, st, L,
                     Linv_diag, d, nblk, static_cast<const double*>(y_tmp), x, flags, done, status,
                     accum);
}

}  // namespace tk
