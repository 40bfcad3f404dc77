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
// The recurrence is the single-reduction form of conjugate gradients
// (Chronopoulos and Gear): with s_i = M r_i, gamma_i = r_i.r_i and
// delta_i = r_i.s_i, both dot products of an iteration come from one
// reduction,
//   beta_i = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = r_i + beta_i p_{i-1},  w_i = s_i + beta_i w_{i-1}  (w_i = M p_i),
//   h_{i+1} = h_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i w_i,
// the same iterates as the textbook form in exact arithmetic.
//
// One persistent launch runs every iteration in two phases:
//   S  each workgroup forms r_{i+1} on the entries its tiles need (from r_i,
//      s_i, w_{i-1} and the scalars, the same arithmetic as the entries'
//      owners) and multiplies its lower 64 x 64 tiles M_IJ by it: the row part
//      M_IJ r_J and the column part M_IJ^T r_I (diagonal tiles: the strictly
//      lower part transposed) go to per-tile partials.  Owners of entries
//      also update h, p, w, r there.  The next tiles' M entries and vector
//      values load while the current tile is used (two tiles ahead);
//   R  each workgroup sums the partials of its own entries of s_{i+1} in a
//      fixed order, and publishes its shares of gamma and delta; every
//      workgroup then adds all shares in the same order.
// No grid-wide barrier separates the phases: a partial or a share starts as
// an empty pattern (a signalling NaN that no arithmetic produces) and its
// reader polls until the value replaces it.  The reader of a partial clears
// it again after reading; shares rotate over three rounds, a workgroup
// clearing its slot of round j - 1 once it has every share of round j.  A
// workgroup publishes its shares only after its other stores of the phase
// have completed, so a complete set of shares also means that every vector
// entry of the phase is in memory (the argument is spelled out at
// share_wait).  Every sum has a fixed order and every workgroup sums the
// shares alike, so the result does not depend on timing.  Data that other
// workgroups read is written through to memory and read with agent-scope
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
constexpr int kCgSyncWords = 32;  // arrival count and abort word, each on its own line
// Resident tiles: a workgroup with at most kResReg + kResLds tiles keeps them
// on chip for every iteration, kResReg in registers and kResLds in LDS.
constexpr int kResReg = 8;
constexpr int kResLds = 1;
constexpr int kMaxRes = kResReg + kResLds;
constexpr int kMaxVb = 2 * kMaxRes;           // distinct vector blocks of those tiles
constexpr int kVbPer = kMaxVb * kCt / kBlock;  // their entries per thread

struct CgArgs {
  const double* M;   // lower triangle, d x d row-major
  const double* b;
  double* h;         // out: solution (b when the iteration did not converge)
  double* rbuf;      // r_i, two halves of d
  double* sbuf;      // s_i = M r_i, two halves
  double* wbuf;      // w_i = M p_i, two halves
  double* rowpart;   // [tile][64], plus a spare slot
  double* colpart;   // [tile][64], plus a spare slot
  double* shares;    // [3 rounds][gamma, delta][grid] shares
  int32_t* sync;     // [0] arrivals, [16] abort word
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
// The empty pattern of a partial or share that has not been written yet.
constexpr unsigned long long kCgEmpty = 0x7FF4C0DE5EED0001ULL;
__device__ inline bool cg_empty(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v)) == kCgEmpty;
}
__device__ inline void cg_clear(double* p) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), kCgEmpty, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int64_t tri(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }
__device__ inline void tile_of(int64_t t, int64_t& i, int64_t& j) {
  i = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(t) + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  j = t - i * (i + 1) / 2;
}

// The vector recurrences of one entry, shared by its owner and every reader:
// w_i = s_i + beta w_{i-1}, r_{i+1} = r_i - alpha w_i.
struct Next {
  double w, r;
};
__device__ inline Next next_entry(double r, double s, double wprev, double alpha, double beta) {
  const double w = fma(beta, wprev, s);
  return {w, fma(-alpha, w, r)};
}

// x from another lane of the same 16-lane row (DPP control CTRL).
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned int>(lo)));
}
// Sum over the 16 lanes of a row, in every lane: rotations by 8 and 4, then
// the quad swaps of 2 and 1 (a fixed order).
__device__ inline double row16_sum(double x) {
  x += dpp_f64<0x128>(x);  // row_ror:8
  x += dpp_f64<0x124>(x);  // row_ror:4
  x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  return x;
}

// Sums of two values per thread over the workgroup, in a fixed order: lane 0
// of each wave sums its wave by a butterfly, then the four wave sums are
// added in wave order (red: 8 doubles).
__device__ inline void block_sum2(double& x, double& y, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_xor(x, o, 64);
    y += __shfl_xor(y, o, 64);
  }
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    red[tid >> 6] = x;
    red[4 + (tid >> 6)] = y;
  }
  __syncthreads();
  x = ((red[0] + red[1]) + red[2]) + red[3];
  y = ((red[4] + red[5]) + red[6]) + red[7];
  __syncthreads();
}

// One tile's operands in registers: this thread's 16 entries of M_IJ and, for
// threads < 128, the vector values at position tid (block J) or tid - 64
// (block I) of the tile.
struct TileRegs {
  double v[16];
  double r, s, w;
};

// FULL: d is a multiple of 64, every tile is whole and its entries load as
// 16-byte vectors without conditions (the diagonal tiles' upper parts are
// zeroed on their way to LDS).  RES (with FULL): the workgroup's tiles are
// read from memory once and stay in registers and LDS; the vector blocks
// they need are formed into LDS once per iteration.
template <bool FULL, bool RES>
__global__ __launch_bounds__(kBlock, 1) void cg_kernel(CgArgs a) {
  __shared__ double tile[kCt * kCld];
  __shared__ double tres[RES ? kResLds : 1][RES ? 16 * kBlock : 1];
  __shared__ double vblk[RES ? kMaxVb : 1][kCt];
  __shared__ double csum_all[RES ? kMaxRes : 1][16][kCt];  // per row group of 4 rows
  __shared__ int slot_of[RES ? 2 * kMaxRes : 1];  // [k]: slot of tile k's J block, [kMaxRes + k]: I
  __shared__ int diag_of[RES ? kMaxRes : 1];
  __shared__ int64_t blk_of[RES ? kMaxVb : 1];
  __shared__ int nslot_s;
  __shared__ double vIJ[kBlock];  // tile vector values: J at [0, 64), I at [64, 128)
  __shared__ double red[kBlock];
  __shared__ double csum[4][kCt];
  __shared__ double own_h[kCgMaxOwn], own_p[kCgMaxOwn], own_r[kCgMaxOwn], own_s[kCgMaxOwn];
  __shared__ int ok_s;
  __shared__ int fail_s;
  const int tid = threadIdx.x;
  const int G = gridDim.x, wg = blockIdx.x;
  const int64_t d = a.d, nb = a.nb;
  const int64_t e0 = wg * a.own;
  const int64_t e1 = e0 + a.own < d ? e0 + a.own : d;
  const int64_t ne = e1 > e0 ? e1 - e0 : 0;
  const int64_t t0 = wg * a.ntiles / G, t1 = (wg + 1) * a.ntiles / G;
  const int srow = tid >> 2, scol = (tid & 3) * 16;  // tile roles: row, 16 columns
  const int nloc = static_cast<int>(t1 - t0);
  // shares of round rd: gamma at shg(rd)[wg], delta at shd(rd)[wg]
  auto shg = [&](int rd) { return a.shares + static_cast<int64_t>(2 * rd) * G; };
  auto shd = [&](int rd) { return a.shares + static_cast<int64_t>(2 * rd + 1) * G; };
  int32_t* arrivals = a.sync;
  int32_t* abort = a.sync + 16;
  int gen = 0;
  bool failed = false;
  // grid barrier on a monotonic arrival count
  auto barrier = [&]() __attribute__((always_inline)) {
    cg_complete_stores();
    __syncthreads();
    ++gen;
    if (tid == 0) {
      __hip_atomic_fetch_add(arrivals, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      long spins = 0;
      int ok = 1;
      while (__hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen * G) {
        // the abort word every 64 polls (one round trip per poll otherwise)
        if ((spins & 63) == 63 &&
            __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
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
  // one poll step of a wait: false once the launch is to stop (the abort word
  // is read every 64 polls; past the spin limit this workgroup raises it)
  auto poll_on = [&](long& spins) __attribute__((always_inline)) {
    ++spins;
    if ((spins & 63) == 0 &&
        __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return false;
    if (spins > kCgSpinLimit) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
  };
  // Sums of every workgroup's gamma and delta shares of round rd, the same
  // fixed order in every workgroup.  Why a complete set orders the phases:
  // a workgroup publishes its shares of round j only after all its stores of
  // the phases before have completed (r_{i+1}, w_i, s_{i+1}, the partials it
  // wrote and the ones it cleared), so once every share of round j is seen,
  // every vector entry the next S phase reads is in memory; and every other
  // workgroup has read all shares of round j - 1 (it read them before it
  // computed the shares of round j), so this workgroup's slot of round j - 1
  // can be cleared now for round j + 2.  That clear completes before this
  // workgroup publishes round j + 1, which every reader of round j + 2 has
  // seen first, so no reader finds a stale share.  The same holds for a
  // cleared partial: its tile's workgroup writes it again only after seeing
  // the shares that its reader published after clearing it.
  auto share_wait = [&](int rd, bool clear_prev, double& sg, double& sd)
      __attribute__((always_inline)) {
    double vg = 0.0, vd = 0.0;
    bool bad = false;
    for (int i = tid; i < G; i += kBlock) {
      const double* pg = shg(rd) + i;
      const double* pd = shd(rd) + i;
      double x = cload(pg), y = cload(pd);
      long spins = 0;
      while (!bad && (cg_empty(x) || cg_empty(y))) {
        if (!poll_on(spins)) {
          bad = true;
          break;
        }
        if (cg_empty(x)) x = cload(pg);
        if (cg_empty(y)) y = cload(pd);
      }
      vg += x;
      vd += y;
    }
    if (bad) fail_s = 1;
    block_sum2(vg, vd, red);
    failed = failed || fail_s != 0;
    if (clear_prev && tid == 0) {
      const int pr = (rd + 2) % 3;
      cg_clear(shg(pr) + wg);
      cg_clear(shd(pr) + wg);
    }
    sg = vg;
    sd = vd;
  };

  // vector sources of the S phase: r_{i+1} = r - alpha (s + beta w).  At the
  // start all three are b with alpha = beta = 0, which gives r_0 = b exactly.
  const double* rsrc = a.b;
  const double* ssrc = a.b;
  const double* wsrc = a.b;
  bool setup = true;
  double alpha = 0.0, beta = 0.0;
  // With FULL tiles the loads below are unconditional (a tile index past the
  // workgroup's range repeats its last tile), so the compiler can keep the
  // next tiles' loads in flight while the current one is used.
  auto fetch = [&](TileRegs& R, int64_t tau) __attribute__((always_inline)) {
    int64_t fi, fj;
    tile_of(tau, fi, fj);
    const int64_t r0 = fi * kCt, c0 = fj * kCt;
    if (FULL) {
      const int64_t x = tid < kCt ? c0 + tid : r0 + (tid & (kCt - 1));
      R.r = cload(rsrc + x);  // threads >= 128 load a value they do not use
      R.s = cload(ssrc + x);
      R.w = cload(wsrc + x);
    }
    const int64_t row = r0 + srow;
    const double* src = a.M + row * d + c0 + scol;
    if (FULL) {
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        const double2 x = *reinterpret_cast<const double2*>(src + e);
        R.v[e] = x.x;
        R.v[e + 1] = x.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t col = c0 + scol + e;
        R.v[e] = (row < d && col < d && (fi != fj || col <= row)) ? src[e] : 0.0;
      }
      R.r = R.s = R.w = 0.0;
      if (tid < 2 * kCt) {
        const int64_t x = tid < kCt ? c0 + tid : r0 + tid - kCt;
        if (x < d) {
          R.r = cload(rsrc + x);
          R.s = cload(ssrc + x);
          R.w = cload(wsrc + x);
        }
      }
    }
  };
  // one tile; real = false: a stand-in whose partials go to the spare slot
  auto process = [&](TileRegs& R, int64_t tau, bool real) __attribute__((always_inline)) {
    int64_t ti, tj;
    tile_of(tau, ti, tj);
    const bool diag = ti == tj;
    vIJ[tid] = next_entry(R.r, R.s, R.w, alpha, beta).r;  // [0, 64): J, [64, 128): I
#pragma unroll
    for (int e = 0; e < 16; ++e)
      tile[srow * kCld + scol + e] = (!FULL || !diag || scol + e <= srow) ? R.v[e] : 0.0;
    __syncthreads();
    if (FULL)
      fetch(R, tau + 2 < t1 ? tau + 2 : t1 - 1);
    else if (tau + 2 < t1)
      fetch(R, tau + 2);
    const int64_t slot = real ? tau : a.ntiles;
    // row part: sum_c M[row][c] v_J[c] over the 4 threads of the row
    double rs = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) rs = fma(tile[srow * kCld + scol + e], vIJ[scol + e], rs);
    rs += __shfl_xor(rs, 1, 64);
    rs += __shfl_xor(rs, 2, 64);
    if ((tid & 3) == 0) cstore(a.rowpart + slot * kCt + srow, rs);
    // column part: sum_row M[row][c] v_I[row] (diagonal tile: rows below c only)
    {
      const int c = tid & 63, rg = tid >> 6;
      double cs = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rw = rg * 16 + i;
        const double m = (!diag || rw > c) ? tile[rw * kCld + c] : 0.0;
        cs = fma(m, vIJ[kCt + rw], cs);
      }
      csum[rg][c] = cs;
    }
    __syncthreads();
    if (tid < kCt)
      cstore(a.colpart + slot * kCt + tid,
             ((csum[0][tid] + csum[1][tid]) + csum[2][tid]) + csum[3][tid]);
    __syncthreads();
  };
  // ---- resident tiles (RES)
  double treg[RES ? kResReg : 1][16];
  if (RES) {
    // the distinct vector blocks of the workgroup's tiles, and each tile's slots
    if (tid == 0) {
      int ns = 0;
      for (int k = 0; k < nloc; ++k) {
        int64_t ti, tj;
        tile_of(t0 + k, ti, tj);
        int sj = -1, si = -1;
        for (int q = 0; q < ns; ++q) {
          if (blk_of[q] == tj) sj = q;
          if (blk_of[q] == ti) si = q;
        }
        if (sj < 0) {
          blk_of[ns] = tj;
          sj = ns++;
        }
        if (si < 0) {
          if (ti == tj) {
            si = sj;
          } else {
            blk_of[ns] = ti;
            si = ns++;
          }
        }
        slot_of[k] = sj;
        slot_of[kMaxRes + k] = si;
        diag_of[k] = ti == tj ? 1 : 0;
      }
      nslot_s = ns;
    }
    __syncthreads();
  }
  // Resident tiles are held in 4 x 4 blocks: thread (rb, cb), rb = 4 wave +
  // lane / 16 and cb = lane % 16, keeps M[4 rb + i][4 cb + j] at 4 i + j.
  // Row sums then reduce over the 16 lanes of a row group and column sums over
  // the wave's 4 row groups (lane shuffles) and the 4 waves (LDS).
  const int rb = (tid >> 6) * 4 + ((tid >> 4) & 3), cb = tid & 15;
  // this thread's block of tile tau (diagonal tiles: upper part zero)
  auto load_tile = [&](double (&v)[16], int64_t tau) __attribute__((always_inline)) {
    int64_t fi, fj;
    tile_of(tau, fi, fj);
    const double* src = a.M + (fi * kCt + 4 * rb) * d + fj * kCt + 4 * cb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; j += 2) {
        const double2 x = *reinterpret_cast<const double2*>(src + i * d + j);
        v[4 * i + j] = (fi != fj || 4 * cb + j <= 4 * rb + i) ? x.x : 0.0;
        v[4 * i + j + 1] = (fi != fj || 4 * cb + j + 1 <= 4 * rb + i) ? x.y : 0.0;
      }
    }
  };
  auto phase_s_res = [&](double* rnext, double* wcur) __attribute__((always_inline)) {
    // the vector blocks' loads first, so that they and the owned entries'
    // loads below are in flight together (one round trip)
    const int nv = nslot_s * kCt;
    double lr[kVbPer], ls[kVbPer], lw[kVbPer];
#pragma unroll
    for (int q = 0; q < kVbPer; ++q) {
      const int e = tid + kBlock * q;
      const int ee = e < nv ? e : 0;
      const int64_t x = blk_of[ee / kCt] * kCt + (ee % kCt);
      lr[q] = cload(rsrc + x);
      ls[q] = cload(ssrc + x);
      lw[q] = cload(wsrc + x);
    }
    for (int64_t i = tid; i < ne; i += kBlock) {
      const int64_t x = e0 + i;
      if (!setup) {
        const double rv = cload(rsrc + x);
        const Next nx = next_entry(rv, cload(ssrc + x), cload(wsrc + x), alpha, beta);
        const double pv = fma(beta, own_p[i], rv);  // p_i = r_i + beta p_{i-1}
        own_p[i] = pv;
        own_h[i] = fma(alpha, pv, own_h[i]);
        own_r[i] = nx.r;
        cstore(wcur + x, nx.w);
        cstore(rnext + x, nx.r);
      } else {  // r_0 = b, w_{-1} = 0
        const double rv = rsrc[x];
        own_p[i] = 0.0;
        own_h[i] = 0.0;
        own_r[i] = rv;
        cstore(wcur + x, 0.0);
        cstore(rnext + x, rv);
      }
    }
    if (setup) {  // the tiles, once
#pragma unroll
      for (int k = 0; k < kResReg; ++k)
        if (k < nloc) load_tile(treg[k], t0 + k);
#pragma unroll
      for (int k = 0; k < kResLds; ++k) {
        if (kResReg + k < nloc) {
          double v[16];
          load_tile(v, t0 + kResReg + k);
#pragma unroll
          for (int e = 0; e < 16; ++e) tres[k][e * kBlock + tid] = v[e];  // this thread's own
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kVbPer; ++q) {
      const int e = tid + kBlock * q;
      if (e < nv) vblk[e / kCt][e % kCt] = next_entry(lr[q], ls[q], lw[q], alpha, beta).r;
    }
    __syncthreads();
    // every tile's row and column parts, no workgroup barrier between tiles;
    // row results stay in registers and column results in LDS until the
    // stores at the end
    double rsv[kMaxRes];
#pragma unroll
    for (int k = 0; k < kMaxRes; ++k) {
      rsv[k] = 0.0;
      if (k < nloc) {
        double m[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
          m[e] = k < kResReg ? treg[k < kResReg ? k : 0][e] : tres[k - kResReg][e * kBlock + tid];
        const double* vJ = vblk[slot_of[k]] + 4 * cb;
        const double* vI = vblk[slot_of[kMaxRes + k]] + 4 * rb;
        const bool dg = diag_of[k] != 0 && rb == cb;  // a block on the tile's diagonal
        double y[4], z[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          y[i] = 0.0;
#pragma unroll
          for (int j = 0; j < 4; ++j) y[i] = fma(m[4 * i + j], vJ[j], y[i]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          z[j] = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double mv = (!dg || i > j) ? m[4 * i + j] : 0.0;  // strictly lower
            z[j] = fma(mv, vI[i], z[j]);
          }
        }
        // rows: over the 16 column blocks of the row group (one 16-lane row)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = row16_sum(y[i]);
        // lane cb < 4 keeps row 4 rb + cb; the column partials of the row
        // group go to LDS, summed over the 16 row groups at the end
        rsv[k] = cb == 0 ? y[0] : cb == 1 ? y[1] : cb == 2 ? y[2] : y[3];
#pragma unroll
        for (int j = 0; j < 4; ++j) csum_all[k][rb][4 * cb + j] = z[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxRes; ++k)
      if (k < nloc && cb < 4) cstore(a.rowpart + (t0 + k) * kCt + 4 * rb + cb, rsv[k]);
    // column parts: wave w sums the 16 row groups of tiles w, w + 4, ...
    for (int k = tid >> 6; k < nloc; k += 4) {
      const int c = tid & (kCt - 1);
      double cs = 0.0;
#pragma unroll
      for (int g = 0; g < 16; ++g) cs += csum_all[k][g][c];
      cstore(a.colpart + (t0 + k) * kCt + c, cs);
    }
  };
  // S phase: the owners' updates, then the tile products
  auto phase_s = [&](double* rnext, double* wcur) __attribute__((always_inline)) {
    if (RES) {
      phase_s_res(rnext, wcur);
      return;
    }
    for (int64_t i = tid; i < ne; i += kBlock) {
      const int64_t x = e0 + i;
      if (!setup) {
        const double rv = cload(rsrc + x);
        const Next nx = next_entry(rv, cload(ssrc + x), cload(wsrc + x), alpha, beta);
        const double pv = fma(beta, own_p[i], rv);  // p_i = r_i + beta p_{i-1}
        own_p[i] = pv;
        own_h[i] = fma(alpha, pv, own_h[i]);
        own_r[i] = nx.r;
        cstore(wcur + x, nx.w);
        cstore(rnext + x, nx.r);
      } else {  // r_0 = b, w_{-1} = 0
        const double rv = rsrc[x];
        own_p[i] = 0.0;
        own_h[i] = 0.0;
        own_r[i] = rv;
        cstore(wcur + x, 0.0);
        cstore(rnext + x, rv);
      }
    }
    if (t0 >= t1) return;
    TileRegs A, B;
    fetch(A, t0);
    fetch(B, t0 + 1 < t1 ? t0 + 1 : t0);
    for (int64_t tau = t0; tau < t1; tau += 2) {
      process(A, tau, true);
      if (FULL)
        process(B, tau + 1 < t1 ? tau + 1 : tau, tau + 1 < t1);
      else if (tau + 1 < t1)
        process(B, tau + 1, true);
    }
  };
  // R phase: own entries of s = M r (sums of the partials in a fixed order);
  // 16 threads per entry, thread z summing terms z, z + 16, ... of
  // [rowpart(I, 0..I), colpart(I..nb-1, I)], then the 16 in a fixed tree.
  // Each term is polled until its tile's workgroup has written it and is
  // cleared after reading.  Ends with this workgroup's shares published in
  // round rd.
  auto term = [&](int64_t I, int64_t o, int64_t u) __attribute__((always_inline)) {
    return u <= I ? a.rowpart + tri(I, u) * kCt + o : a.colpart + tri(u - 1, I) * kCt + o;
  };
  auto phase_r = [&](double* snext, int rd) __attribute__((always_inline)) {
    bool bad = false;
    for (int64_t base = 0; base < ne; base += kBlock / 16) {
      const int64_t i = base + (tid >> 4);
      const int z = tid & 15;
      double sum = 0.0;
      if (i < ne) {
        const int64_t gi = e0 + i;
        const int64_t I = gi / kCt, o = gi % kCt;
        const int64_t nt = nb + 1;
        double t[kCgTerms];  // all loads issued before the sum
#pragma unroll
        for (int q = 0; q < kCgTerms; ++q) {
          const int64_t u = z + 16 * q;
          t[q] = u < nt ? cload(term(I, o, u)) : 0.0;
        }
        long spins = 0;
        for (;;) {
          bool pend = false;
#pragma unroll
          for (int q = 0; q < kCgTerms; ++q) pend = pend || cg_empty(t[q]);
          if (!pend || bad) break;
          if (!poll_on(spins)) {
            bad = true;
            break;
          }
#pragma unroll
          for (int q = 0; q < kCgTerms; ++q) {
            const int64_t u = z + 16 * q;
            if (u < nt && cg_empty(t[q])) t[q] = cload(term(I, o, u));
          }
        }
#pragma unroll
        for (int q = 0; q < kCgTerms; ++q) {
          const int64_t u = z + 16 * q;
          if (u < nt) cg_clear(term(I, o, u));
        }
#pragma unroll
        for (int q = 0; q < kCgTerms; ++q) sum += t[q];
      }
      sum += __shfl_xor(sum, 8, 64);
      sum += __shfl_xor(sum, 4, 64);
      sum += __shfl_xor(sum, 2, 64);
      sum += __shfl_xor(sum, 1, 64);
      if (i < ne && z == 0) {
        own_s[i] = sum;
        cstore(snext + e0 + i, sum);
      }
    }
    if (bad) fail_s = 1;
    __syncthreads();
    double pg = 0.0, pd = 0.0;
    for (int64_t i = tid; i < ne; i += kBlock) {
      pg = fma(own_r[i], own_r[i], pg);
      pd = fma(own_r[i], own_s[i], pd);
    }
    block_sum2(pg, pd, red);
    cg_complete_stores();
    __syncthreads();
    if (tid == 0 && fail_s == 0) {
      cstore(shg(rd) + wg, pg);
      cstore(shd(rd) + wg, pd);
    }
  };

  // ---- start: the partials this workgroup reads and its share slots of
  // every round empty, then the launch's one grid-wide barrier
  if (tid == 0) fail_s = 0;
  for (int64_t x = tid; x < ne * (nb + 1); x += kBlock) {
    const int64_t gi = e0 + x / (nb + 1), u = x % (nb + 1);
    cg_clear(term(gi / kCt, gi % kCt, u));
  }
  if (tid < 3) {
    cg_clear(shg(tid) + wg);
    cg_clear(shd(tid) + wg);
  }
  barrier();
  // ---- s_0 = M b, gamma_0, delta_0 (shares of round 0)
  phase_s(a.rbuf, a.wbuf + d);  // r_0 -> rbuf[0], w_{-1} = 0 -> wbuf[1]
  phase_r(a.sbuf, 0);
  double g0, del;
  share_wait(0, false, g0, del);
  double gam = g0;
  alpha = del > 0.0 ? gam / del : 0.0;
  beta = 0.0;
  int it = 0;
  bool conv = !(g0 > 0.0);
  bool broke = !conv && !(del > 0.0);
  while (!conv && !broke && !failed && it < a.max_iter) {
    const int c = it & 1;
    setup = false;
    rsrc = a.rbuf + c * d;
    ssrc = a.sbuf + c * d;
    wsrc = a.wbuf + (c ^ 1) * d;
    const int rd = (it + 1) % 3;
    phase_s(a.rbuf + (c ^ 1) * d, a.wbuf + c * d);
    phase_r(a.sbuf + (c ^ 1) * d, rd);
    double gn, dn;
    share_wait(rd, true, gn, dn);
    ++it;
    const double gprev = gam;
    gam = gn;
    conv = gn <= kCgTol * kCgTol * g0;
    if (conv) break;
    const double bn = gn / gprev;
    const double den = dn - bn * gn / alpha;
    if (!(den > 0.0)) {  // not positive definite in this direction
      broke = true;
      break;
    }
    beta = bn;
    alpha = gn / den;
  }
  // ---- finish: h, or b again when the iteration did not converge
  for (int64_t i = tid; i < ne; i += kBlock) a.h[e0 + i] = conv ? own_h[i] : a.b[e0 + i];
  if (wg == 0 && tid == 0) {
    *a.cg_done = conv ? 1 : 0;
    *a.steps = it;
    *a.relres = g0 > 0.0 ? sqrt(gam / g0) : 0.0;
    if (conv) *a.min_pivot = 0.0;
  }
  if (failed && tid == 0) atomicMax(a.status, static_cast<int32_t>(TK_E_HIP));
}

struct CgWS {
  double* rbuf;
  double* sbuf;
  double* wbuf;
  double* rowpart;
  double* colpart;
  double* shares;
  int32_t* sync;
  int32_t* done;
};

void carve_cg(Carver& c, int64_t d, CgWS& w) {
  const int64_t nb = cdiv(d, kCt);
  const int64_t nt = nb * (nb + 1) / 2;
  w.rbuf = c.take<double>(2 * d);
  w.sbuf = c.take<double>(2 * d);
  w.wbuf = c.take<double>(2 * d);
  w.rowpart = c.take<double>((nt + 1) * kCt);  // one spare tile slot
  w.colpart = c.take<double>((nt + 1) * kCt);
  w.shares = c.take<double>(3 * 2 * 1024);
  w.sync = c.take<int32_t>(kCgSyncWords);
  w.done = c.take<int32_t>(1);
}

}  // namespace

bool cg_ok(int64_t d) { return d >= 1024 && d <= int64_t(kCgMaxBlocks) * kCt; }

size_t cg_bytes(int64_t d) {
  Carver c(nullptr);
  CgWS w;
  carve_cg(c, d, w);
  return c.used;
}

void launch_cg(const double* M, int64_t d, const double* b, double* h, void* ws, int32_t* steps,
               double* relres, double* min_pivot, int32_t* status, int max_iter,
               hipStream_t st) {
  const int64_t nb = cdiv(d, kCt);
  const int64_t nt = nb * (nb + 1) / 2;
  Carver c(ws);
  CgWS w;
  carve_cg(c, d, w);
  const bool full = d % kCt == 0;
  // the grid: one workgroup per compute unit, all resident together (every
  // workgroup waits on data from the others), then tiles held on chip when
  // they fit
  int grid = device_cu_count();
  {
    const int r1 = resident_grid(reinterpret_cast<const void*>(cg_kernel<true, true>), kBlock, 0);
    const int r2 = resident_grid(reinterpret_cast<const void*>(cg_kernel<true, false>), kBlock, 0);
    const int r3 = resident_grid(reinterpret_cast<const void*>(cg_kernel<false, false>), kBlock, 0);
    int r = r1 < r2 ? r1 : r2;
    r = r < r3 ? r : r3;
    if (r > 0 && grid > r) grid = r;
  }
  if (grid > 1024) grid = 1024;
  if (grid > nt) grid = static_cast<int>(nt);
  int64_t own = cdiv(d, grid);
  if (own > kCgMaxOwn) own = kCgMaxOwn;
  grid = static_cast<int>(cdiv(d, own));
  const bool resident = full && cdiv(nt, grid) <= kMaxRes;
  CgArgs a;
  a.M = M;
  a.b = b;
  a.h = h;
  a.rbuf = w.rbuf;
  a.sbuf = w.sbuf;
  a.wbuf = w.wbuf;
  a.rowpart = w.rowpart;
  a.colpart = w.colpart;
  a.shares = w.shares;
  a.sync = w.sync;
  a.cg_done = w.done;
  a.steps = steps;
  a.relres = relres;
  a.min_pivot = min_pivot;
  a.status = status;
  a.d = d;
  a.nb = nb;
  a.ntiles = nt;
  a.own = own;
  a.max_iter = max_iter;
  launch_fill_i32(kCgSyncWords, 0, w.sync, st);
  const dim3 gd(static_cast<unsigned>(grid));
  if (resident)
    hipLaunchKernelGGL((cg_kernel<true, true>), gd, dim3(kBlock), 0, st, a);
  else if (full)
    hipLaunchKernelGGL((cg_kernel<true, false>), gd, dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((cg_kernel<false, false>), gd, dim3(kBlock), 0, st, a);
}

const int32_t* cg_done_word(void* ws, int64_t d) {
  Carver c(ws);
  CgWS w;
  carve_cg(c, d, w);
  return w.done;
}

}  // namespace tk
