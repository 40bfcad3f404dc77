// Sketched FP64 Gram grouped by the samples' index in one mode.
//
// Proof of Thm 4.2: the sketched Gram is the weighted sum of s outer products
// of whitened design rows q_t = (x)_n q^(n)_{i_n}.  Let L be the last mode
// with R_L >= 2 and d' = d / R_L.  A design index splits as r = p R_L + m
// (modes after L have rank 1), so q_t = y_t (x) e_{i_L}, with e_k the
// whitened row k of mode L and y_t[p] = prod_{n<L} q^(n)_{i_n}[digit_n(p)]
// times the single entries of the modes after L.  Collecting the samples by
// k = i_L regroups the same sum exactly:
//   sum_t w_t q_t q_t^T = sum_k B_k (x) e_k e_k^T,
//   B_k = sum_{t : i_L = k} w_t y_t y_t^T,
// which costs about s d'^2 / 2 + I_L d^2 / 2 multiply-adds instead of
// s d^2 / 2.  Three passes, all FP64:
//  1. a stable counting sort of the samples by i_L: per block of 256 samples
//     each sample's rank among the block's samples of its key and a count
//     table [key][block], an exclusive scan of that table, a scatter;
//  2. B_k on v_mfma_f64_16x16x4, one workgroup per (group, lower 64 x 64
//     tile of d' x d'), y_t formed from LDS per chunk of 32 or 64 samples of
//     the group (in their original order, so every sum has a fixed order);
//  3. M[p R_L + m][p' R_L + m'] = sum_k B_k[p][p'] e_k[m] e_k[m']
//     + lambda prod_n P_n[..][..] on the lower triangle: a GEMM over the
//     groups on v_mfma_f64_4x4x4_4b, with the ridge term's Kronecker product
//     in its epilogue.
// The right side and the residual of the solve are grouped the same way
// (the vector kernels below).
#include <string.h>

#include <type_traits>

#include "tk_mfma.h"

namespace tk {
namespace {

constexpr int kGt = 64;        // tile edge over d' (pass 2) and q-row block (pass 3)
constexpr int kGkc = 32;       // samples (quadrant pass 2, vectors) or groups (pass 3) per chunk
constexpr int kGld = kGt + 1;  // padded LDS row
constexpr int kScanPer = 16 * kBlock;  // count-table entries per scan workgroup

// Exclusive prefix of v over the workgroup; *total gets the workgroup's sum.
__device__ inline int block_exscan(int v, int* total) {
  __shared__ int wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    off += i < w ? wsum[i] : 0;
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__device__ inline int32_t group_key(const int32_t* key, int64_t t, int64_t groups) {
  const int32_t k = key[t];
  return (k < 0 || k >= groups) ? 0 : k;  // flagged by the gather pass (weight 0)
}

// ------------------------------------------------------------------ pass 1: sort
// rank[t]: samples before t in its block with the same key; cnt[key nb + b]:
// the block's count of that key (written by the key's last sample in the block).
__global__ __launch_bounds__(kBlock) void grp_count_kernel(const int32_t* __restrict__ key,
                                                           int64_t s, int64_t groups, int64_t nb,
                                                           int32_t* __restrict__ rank,
                                                           int32_t* __restrict__ cnt) {
  __shared__ int32_t keys[kBlock];
  const int64_t b = blockIdx.x;
  const int64_t t = b * kBlock + threadIdx.x;
  const int32_t k = t < s ? group_key(key, t, groups) : -1;
  keys[threadIdx.x] = k;
  __syncthreads();
  int before = 0, after = 0;
  for (int j = 0; j < kBlock; ++j) {
    const bool same = keys[j] == k;
    before += (same && j < static_cast<int>(threadIdx.x)) ? 1 : 0;
    after += (same && j > static_cast<int>(threadIdx.x)) ? 1 : 0;
  }
  if (t < s) {
    rank[t] = before;
    if (after == 0) cnt[static_cast<int64_t>(k) * nb + b] = before + 1;
  }
}

// part[w] = sum of entries [w kScanPer, (w + 1) kScanPer) of v
__global__ __launch_bounds__(kBlock) void grp_scan_reduce_kernel(const int32_t* __restrict__ v,
                                                                 int64_t n,
                                                                 int32_t* __restrict__ part) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanPer + threadIdx.x * 16;
  int sum = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) sum += base + i < n ? v[base + i] : 0;
  int total = 0;
  (void)block_exscan(sum, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// exclusive scan of part[0, np) in place (one workgroup, np <= 16 * kBlock)
__global__ __launch_bounds__(kBlock) void grp_scan_top_kernel(int32_t* __restrict__ part,
                                                              int64_t np) {
  const int64_t per = (np + kBlock - 1) / kBlock;
  const int64_t lo = threadIdx.x * per;
  int sum = 0;
  for (int64_t i = lo; i < lo + per && i < np; ++i) sum += part[i];
  int total = 0;
  int run = block_exscan(sum, &total);
  for (int64_t i = lo; i < lo + per && i < np; ++i) {
    const int x = part[i];
    part[i] = run;
    run += x;
  }
}

// exclusive scan of v in place, workgroup w adding the scanned part[w]
__global__ __launch_bounds__(kBlock) void grp_scan_apply_kernel(int32_t* __restrict__ v, int64_t n,
                                                                const int32_t* __restrict__ part) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanPer + threadIdx.x * 16;
  int x[16];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    x[i] = base + i < n ? v[base + i] : 0;
    sum += x[i];
  }
  int total = 0;
  int run = part[blockIdx.x] + block_exscan(sum, &total);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (base + i < n) v[base + i] = run;
    run += x[i];
  }
}

// perm[off(key, block) + rank] = t: samples in key order, original order within a key
__global__ __launch_bounds__(kBlock) void grp_scatter_kernel(const int32_t* __restrict__ key,
                                                             int64_t s, int64_t groups, int64_t nb,
                                                             const int32_t* __restrict__ rank,
                                                             const int32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ perm) {
  const int64_t b = blockIdx.x;
  const int64_t t = b * kBlock + threadIdx.x;
  if (t >= s) return;
  const int32_t k = group_key(key, t, groups);
  perm[cnt[static_cast<int64_t>(k) * nb + b] + rank[t]] = static_cast<int32_t>(t);
}

struct GrpArgs {
  const double* rows;   // sorted sample rows: [u][S'], the rows of modes < L of sample perm[u]
  const double* scs;    // sorted w_t times the squared entries of the modes after L
  const int32_t* cnt;   // scanned count table: group k is [cnt[k nb], cnt[(k + 1) nb])
  double* B;            // [group][lower tile][64][64]
  const double* E;      // whitened rows of mode L (groups x R_L)
  const double* P;      // (L_n^T L_n)^{-1} at geom.roff
  double lambda;
  double* M;            // d x d, lower triangle written
  int64_t nb, groups, dp, ptiles;
  int32_t L, RL, sp;    // sp = S' = sum_{n<L} R_n
  int32_t tcn, n0, n1;  // pair form: column tiles, pairs of modes 0 and 1
};

// ------------------------------------------------------------------ pass 2: B_k
// Sorted sample rows: element e = u S' + j holds entry j of the concatenated
// rows of modes < L of sample t = perm[u]; with tau_t = prod_{n>L} q^(n)_{i_n}[0]
// (the modes after L have rank 1), scs[u] = w_t tau_t^2 and xs[u] = (w x)_t tau_t.
__global__ __launch_bounds__(kBlock) void grp_rows_kernel(Geom g, const int32_t* __restrict__ idx,
                                                          int64_t s, const double* __restrict__ Q64,
                                                          const double* __restrict__ weff,
                                                          const double* __restrict__ xw,
                                                          const int32_t* __restrict__ perm, int L,
                                                          int sp, double* __restrict__ rows,
                                                          double* __restrict__ scs,
                                                          double* __restrict__ xs) {
  // s S' < 2^31 (the plan's limit): 32-bit index arithmetic
  const uint32_t e = blockIdx.x * static_cast<uint32_t>(kBlock) + threadIdx.x;
  if (static_cast<int64_t>(e) >= s * sp) return;
  const uint32_t u = e / static_cast<uint32_t>(sp);
  const int j = static_cast<int>(e - u * static_cast<uint32_t>(sp));
  const int64_t t = perm[u];
  int n = 0;
  while (n + 1 < L && g.soff[n + 1] <= j) ++n;
  int32_t i = idx[static_cast<int64_t>(n) * s + t];
  if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
  rows[e] = Q64[g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n] + (j - g.soff[n])];
  if (j == 0) {
    double tau = 1.0;
    for (int m = L + 1; m < g.order; ++m) {
      int32_t im = idx[static_cast<int64_t>(m) * s + t];
      if (im < 0 || im >= g.dims[m]) im = 0;
      tau *= Q64[g.qoff[m] + im];  // rank 1
    }
    scs[u] = weff[t] * (tau * tau);
    xs[u] = xw[t] * tau;
  }
}

// Workgroup (group k, lower tile (ta, tb) of d' x d'); wave w multiplies
// quadrant (w / 2, w % 2) of the 64 x 64 tile (the upper quadrant of a
// diagonal tile stays zero).  Per chunk of 32 samples the rows (32 S'
// contiguous doubles) go to LDS from registers loaded during the previous
// chunk's products; each lane forms its operands y_t[p] = prod_{n<L}
// row_t[soff_n + digit_n(p)] (times scs on the left) from LDS.  NR >= S' / 8.
template <int NR>
__global__ __launch_bounds__(kBlock) void grp_block_kernel(Geom g, GrpArgs a) {
  extern __shared__ double rowbuf[];  // [kGkc][S' + 1]
  __shared__ double ssc[kGkc];
  const int64_t tau = blockIdx.x % a.ptiles;
  const int64_t k = blockIdx.x / a.ptiles;
  int64_t ta, tb;
  tri_index(tau, ta, tb);
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int L = a.L, SP = a.sp, LD = a.sp + 1;
  const int qa = w >> 1, qb = w & 1;
  const bool active = !(ta == tb && qa < qb);
  // LDS offsets (within a sample's row) of the digits of this lane's operand rows
  int oa[2][kMaxOrder], ob[2][kMaxOrder];
  bool va[2], vb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = i * 16 + (lane & 15);
    const int64_t pa = ta * kGt + qa * 32 + row, pb = tb * kGt + qb * 32 + row;
    va[i] = pa < a.dp;
    vb[i] = pb < a.dp;
    int64_t xa = va[i] ? pa : 0, xb = vb[i] ? pb : 0;
#pragma unroll
    for (int n = kMaxOrder - 1; n >= 0; --n) {
      oa[i][n] = 0;
      ob[i][n] = 0;
      if (n < L) {
        const int R = g.ranks[n];
        oa[i][n] = g.soff[n] + static_cast<int>(xa % R);
        ob[i][n] = g.soff[n] + static_cast<int>(xb % R);
        xa /= R;
        xb /= R;
      }
    }
  }
  // staging: element e = tid + 256 i of a chunk -> LDS (e / S') LD + e % S'
  const int nel = kGkc * SP;
  int lofs[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int e = tid + kBlock * i;
    lofs[i] = e < nel ? (e / SP) * LD + e % SP : -1;
  }
  double pf[NR];
  double psc = 0.0;
  auto fetch = [&](int64_t c0) {
    const int64_t lim = ((g1 < c0 + kGkc ? g1 : c0 + kGkc) - c0) * SP;
    const double* src = a.rows + c0 * SP;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int e = tid + kBlock * i;
      pf[i] = e < lim ? src[e] : 0.0;
    }
    if (tid < kGkc) psc = c0 + tid < g1 ? a.scs[c0 + tid] : 0.0;
  };
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  if (g0 < g1) fetch(g0);
  for (int64_t c0 = g0; c0 < g1; c0 += kGkc) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (lofs[i] >= 0) rowbuf[lofs[i]] = pf[i];
    if (tid < kGkc) ssc[tid] = psc;
    __syncthreads();
    if (c0 + kGkc < g1) fetch(c0 + kGkc);
    if (active) {
#pragma unroll 2
      for (int ks = 0; ks < kGkc / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        const double* rk = rowbuf + kk * LD;
        double a0 = ssc[kk], a1 = a0, b0 = 1.0, b1 = 1.0;
#pragma unroll
        for (int n = 0; n < kMaxOrder; ++n) {
          if (n < L) {
            a0 *= rk[oa[0][n]];
            a1 *= rk[oa[1][n]];
            b0 *= rk[ob[0][n]];
            b1 *= rk[ob[1][n]];
          }
        }
        a0 = va[0] ? a0 : 0.0;
        a1 = va[1] ? a1 : 0.0;
        b0 = vb[0] ? b0 : 0.0;
        b1 = vb[1] ? b1 : 0.0;
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator v of lane l: row l / 16 + 4 v, column l % 16 of its 16 x 16 block
  double* out = a.B + (k * a.ptiles + tau) * (kGt * kGt);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = qa * 32 + i * 16 + (lane >> 4) + 4 * v;
        const int col = qb * 32 + j * 16 + (lane & 15);
        out[row * kGt + col] = acc[i][j][v];
      }
}

// Sample-split form for at most three modes before L (NL): workgroup (group
// k, lower 64 x 64 tile (ta, tb) of d' x d'); every wave computes the whole
// tile as 4 x 4 blocks of v_mfma_f64_16x16x4 over its own quarter of each
// CK-sample chunk (samples w CK / 4 .. (w + 1) CK / 4 - 1, k-steps past the
// group's end skipped), so each formed operand feeds four products and no
// wave idles on a diagonal tile (its blocks above the diagonal are skipped).
// FP64 MFMA and ordinary vector instructions do not overlap on one SIMD, so
// the operand formation is kept to its multiplies: the chunk sits in LDS
// transposed, entry j of sample u at j CKP + u, which makes every operand
// address of a k-step a per-lane base fixed for the launch plus a constant;
// row S' is all zeros and serves the rows p >= d' of a ragged tile.  The four
// partial tiles are added in wave order through LDS at the end.
constexpr int kRld = kGt + 8;  // reduction tile row stride (two rows per bank sweep)
int split_ck(int sp) { return sp <= 32 ? 64 : 32; }
// p / R and p % R for p < 2^20, R <= 64: (p + 1/2) / R stays at least 1/(2R)
// from an integer, far more than the rounding of the float product
__device__ inline void small_divmod(int p, int R, float rinv, int& q, int& r) {
  q = static_cast<int>((static_cast<float>(p) + 0.5f) * rinv);
  r = p - q * R;
}
// (m, m') with c = m (m + 1) / 2 + m', 0 <= m' <= m, for c < 2^20
__device__ inline void pair_of(int c, int& m, int& mp) {
  int i = static_cast<int>((sqrtf(8.0f * static_cast<float>(c) + 1.0f) - 1.0f) * 0.5f);
  if ((i + 1) * (i + 2) / 2 <= c) ++i;
  if (i * (i + 1) / 2 > c) --i;
  m = i;
  mp = c - i * (i + 1) / 2;
}

// PAIR (NL = 2): with y_t = a_t (x) b_t (rows of modes 0 and 1), B_k[(r, s)][(r', s')]
// = C_k[i0][i1] = sum_t w_t a_t[r] a_t[r'] b_t[s] b_t[s'] depends only on the
// unordered pairs i0 = {r, r'} and i1 = {s, s'}, so the pass forms the n0 x n1
// matrix C_k (no symmetry left) in tiles (tr, tc) = (tau / tcn, tau % tcn): the
// operands are products of two entries of one mode instead of one of each mode.
template <int NR, int NL, int CK, bool PAIR>
__global__ __launch_bounds__(kBlock, 2) void grp_block_split_kernel(Geom g, GrpArgs a,
                                                                    int64_t nunits) {
  static_assert(!PAIR || NL == 2, "the pair form takes two modes before L");
  constexpr int CKP = CK + 2;       // transposed chunk stride
  extern __shared__ double rowT[];  // [S' + 1][CKP], then the 64 x kRld reduction tile
  __shared__ double ssc[CK];
  // workgroup ids go round-robin over the 8 XCDs
  int64_t k, tau, ta, tb;
  if (PAIR) {
    // XCD x takes the groups k = x mod 8 (their sorted rows stay in its L2),
    // tile by tile: the full tiles first, then those of the ragged last row or
    // column tile, so that the light workgroups fill the end
    const int64_t x = blockIdx.x % 8, j = blockIdx.x / 8;
    const int64_t gx = (a.groups - x + 7) / 8;
    if (j >= gx * a.ptiles) return;
    const int64_t rk = j / gx;
    k = x + 8 * (j % gx);
    const int64_t tcn = a.tcn, trn = a.ptiles / a.tcn;
    const int64_t h = (trn - 1) * (tcn - 1);
    if (rk < h) {
      ta = rk / (tcn - 1);
      tb = rk % (tcn - 1);
    } else if (rk < h + trn - 1) {
      ta = rk - h;
      tb = tcn - 1;
    } else if (rk < h + trn - 1 + tcn - 1) {
      ta = trn - 1;
      tb = rk - h - (trn - 1);
    } else {
      ta = trn - 1;
      tb = tcn - 1;
    }
    tau = ta * tcn + tb;
  } else {
    // consecutive units (one group's tiles, which read the same sorted rows)
    // are kept on one XCD
    const int64_t per_xcd = static_cast<int64_t>(gridDim.x) / 8;
    const int64_t unit = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (unit >= nunits) return;
    tau = unit % a.ptiles;
    k = unit / a.ptiles;
    tri_index(tau, ta, tb);
  }
  const bool diag = !PAIR && ta == tb;
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int SP = a.sp;
  double* red = rowT + (SP + 1) * CKP;
  // this lane's sample within a k-step and its first k-step's sample
  const int u0 = w * (CK / 4) + (lane >> 4);
  // LDS indices (at sample u0) of the digits of this lane's operand rows
  int ia[4][NL], ib[4][NL];
  // pair form: 16-row blocks of the tile that hold pairs
  int nbi = 4, nbj = 4;
  if (PAIR) {
    const int li = a.n0 - static_cast<int>(ta) * kGt, lj = a.n1 - static_cast<int>(tb) * kGt;
    nbi = li >= kGt ? 4 : (li + 15) / 16;
    nbj = lj >= kGt ? 4 : (lj + 15) / 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int i0 = static_cast<int>(ta) * kGt + i * 16 + (lane & 15);
      const int i1 = static_cast<int>(tb) * kGt + i * 16 + (lane & 15);
      int r = 0, rp = 0, s2 = 0, sp2 = 0;
      if (i0 < a.n0) pair_of(i0, r, rp);
      if (i1 < a.n1) pair_of(i1, s2, sp2);
      // the zero row past the last pair
      ia[i][0] = (i0 < a.n0 ? g.soff[0] + r : SP) * CKP + u0;
      ia[i][NL - 1] = (i0 < a.n0 ? g.soff[0] + rp : SP) * CKP + u0;
      ib[i][0] = (i1 < a.n1 ? g.soff[1] + s2 : SP) * CKP + u0;
      ib[i][NL - 1] = (i1 < a.n1 ? g.soff[1] + sp2 : SP) * CKP + u0;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (PAIR) break;
    const int pa = static_cast<int>(ta) * kGt + i * 16 + (lane & 15);
    const int pb = static_cast<int>(tb) * kGt + i * 16 + (lane & 15);
    const bool va = pa < a.dp, vb = pb < a.dp;
    int xa = va ? pa : 0, xb = vb ? pb : 0;
#pragma unroll
    for (int n = NL - 1; n >= 0; --n) {
      const int R = g.ranks[n];
      const float rinv = 1.0f / static_cast<float>(R);
      int qa, ra, qb, rb;
      small_divmod(xa, R, rinv, qa, ra);
      small_divmod(xb, R, rinv, qb, rb);
      // the zero row for p >= d' (in the first mode: the product is then 0)
      ia[i][n] = ((n == 0 && !va) ? SP : g.soff[n] + ra) * CKP + u0;
      ib[i][n] = ((n == 0 && !vb) ? SP : g.soff[n] + rb) * CKP + u0;
      xa = qa;
      xb = qb;
    }
  }
  // staging: element e = tid + 256 i of a chunk (sample e / S', entry e % S')
  const int nel = CK * SP;
  int lofs[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int e = tid + kBlock * i;
    lofs[i] = e < nel ? (e % SP) * CKP + e / SP : -1;
  }
  for (int u = tid; u < CK; u += kBlock) rowT[SP * CKP + u] = 0.0;
  double pf[NR];
  double psc = 0.0;
  auto fetch = [&](int64_t c0) {
    const int64_t lim = ((g1 < c0 + CK ? g1 : c0 + CK) - c0) * SP;
    const double* src = a.rows + c0 * SP;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int e = tid + kBlock * i;
      pf[i] = e < lim ? src[e] : 0.0;
    }
    if (tid < CK) psc = c0 + tid < g1 ? a.scs[c0 + tid] : 0.0;
  };
  doublex4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  if (g0 < g1) fetch(g0);
  for (int64_t c0 = g0; c0 < g1; c0 += CK) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (lofs[i] >= 0) rowT[lofs[i]] = pf[i];
    if (tid < CK) ssc[tid] = psc;
    __syncthreads();
    if (c0 + CK < g1) fetch(c0 + CK);
    const int64_t left = g1 - c0 - w * (CK / 4);  // samples of this wave's quarter
#pragma unroll
    for (int h = 0; h < CK / 16; ++h) {
      if (4 * h < left) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double x = ssc[u0 + 4 * h], y = 1.0;
#pragma unroll
          for (int n = 0; n < NL; ++n) {
            x *= rowT[ia[i][n] + 4 * h];
            y *= rowT[ib[i][n] + 4 * h];
          }
          av[i] = x;
          bv[i] = y;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (PAIR ? (i < nbi && j < nbj) : (!diag || i >= j))
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ((acc_3 + acc_2) + acc_1) + acc_0 through one LDS tile; accumulator v of
  // lane l: row l / 16 + 4 v, column l % 16 of its 16 x 16 block
  // (pair form: only the blocks that hold pairs; the expand pass reads no other)
  for (int src = 3; src >= 0; --src) {
    if (w == src) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (PAIR && (i >= nbi || j >= nbj)) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int e = (i * 16 + (lane >> 4) + 4 * v) * kRld + j * 16 + (lane & 15);
            red[e] = src == 3 ? acc[i][j][v] : red[e] + acc[i][j][v];
          }
        }
    }
    __syncthreads();
  }
  double* out = a.B + (k * a.ptiles + tau) * (kGt * kGt);
  const int nrow = 16 * nbi, ncol = 16 * nbj;
  for (int e = tid; e < kGt * kGt; e += kBlock) {
    const int r = e / kGt, c = e % kGt;
    if (!PAIR || (r < nrow && c < ncol)) out[e] = red[r * kRld + c];
  }
}

// x from another lane of the same 16-lane row (DPP control CTRL); the sum over
// the 16 lanes of a row, in every lane, in a fixed order.
template <int CTRL>
__device__ inline double grp_dpp(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned int>(lo)));
}
__device__ inline double row16_sum(double x) {
  x += grp_dpp<0x128>(x);  // row_ror:8
  x += grp_dpp<0x124>(x);  // row_ror:4
  x += grp_dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += grp_dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  return x;
}

// ------------------------------------------------------------------ right side and residual
// The same grouping for the vectors of the solve:
//   sum_t q_t (xw_t - weff_t q_t.h) = sum_k (sum_{t: i_L = k} c_t y_t) (x) e_k,
//   c_t = xs_t - scs_t (y_t . u_k),  u_k[p] = sum_m h[p R_L + m] e_k[m]
// (without h: c_t = xs_t, the right side).

// Chunk staging of the vector kernels: the CK S' doubles of a chunk of sorted
// rows, NP per thread in registers (the rest, for longer rows, loaded
// directly), so that the next chunk's loads are in flight while the current
// one is used.
template <int CK, int NP>
struct ChunkStage {
  double pf[NP];
  __device__ void fetch(const double* rows, int64_t c0, int64_t g1, int sp) {
    const int64_t lim = ((g1 < c0 + CK ? g1 : c0 + CK) - c0) * sp;
    const double* src = rows + c0 * sp;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = threadIdx.x + kBlock * i;
      pf[i] = e < lim ? src[e] : 0.0;
    }
  }
  __device__ void store(double* rowbuf, const double* rows, int64_t c0, int64_t g1, int sp) {
    const int ld = sp + 1, nel = CK * sp;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = threadIdx.x + kBlock * i;
      if (e < nel) rowbuf[(e / sp) * ld + e % sp] = pf[i];
    }
    const int64_t lim = ((g1 < c0 + CK ? g1 : c0 + CK) - c0) * sp;
    for (int e = threadIdx.x + NP * kBlock; e < nel; e += kBlock)
      rowbuf[(e / sp) * ld + e % sp] = e < lim ? rows[c0 * sp + e] : 0.0;
  }
};
using RowStage = ChunkStage<kGkc, 4>;

// U[k][p] = u_k[p]
__global__ __launch_bounds__(kBlock) void grp_hvec_kernel(GrpArgs a, const double* __restrict__ h,
                                                          double* __restrict__ U) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= a.groups * a.dp) return;
  const int64_t k = e / a.dp, p = e % a.dp;
  const double* ek = a.E + k * a.RL;
  const double* hp = h + p * a.RL;
  double sum = 0.0;
  for (int m = 0; m < a.RL; ++m) sum = fma(hp[m], ek[m], sum);
  U[e] = sum;
}

// V[k][p] = sum_{t in group k} c_t y_t[p], one workgroup per group, the group's
// samples in their sorted order in chunks of 32 staged in LDS.  A thread keeps
// the sums of p = tid + 256 i (i < kResPer); the dots y_t . u_k are taken by 8
// threads per sample over p = z, z + 8, ... and added in a fixed tree.
constexpr int kResPer = 4;  // d' <= 1024
template <int NL>
__global__ __launch_bounds__(kBlock) void grp_resid_kernel(Geom g, GrpArgs a,
                                                           const double* __restrict__ xs,
                                                           const double* __restrict__ U,
                                                           double* __restrict__ V) {
  extern __shared__ double smem[];  // rows [kGkc][S' + 1], u_k [d'], digit offsets [d'][NL]
  __shared__ double cfac[kGkc];
  const int SP = a.sp, LD = a.sp + 1;
  const int64_t dp = a.dp;
  double* rowbuf = smem;
  double* uk = smem + kGkc * LD;
  int* dig = reinterpret_cast<int*>(uk + dp);
  const int64_t k = blockIdx.x;
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x;
  for (int64_t p = tid; p < dp; p += kBlock) {
    if (U) uk[p] = U[k * dp + p];
    int64_t x = p;
#pragma unroll
    for (int n = NL - 1; n >= 0; --n) {
      const int R = g.ranks[n];
      dig[p * NL + n] = g.soff[n] + static_cast<int>(x % R);
      x /= R;
    }
  }
  double v[kResPer];
  int od[kResPer][NL];  // this thread's digit offsets
#pragma unroll
  for (int i = 0; i < kResPer; ++i) {
    v[i] = 0.0;
    int64_t x = tid + kBlock * i < dp ? tid + kBlock * i : 0;
#pragma unroll
    for (int n = NL - 1; n >= 0; --n) {
      const int R = g.ranks[n];
      od[i][n] = g.soff[n] + static_cast<int>(x % R);
      x /= R;
    }
  }
  const int jd = tid >> 3, zd = tid & 7;  // dot roles: sample jd, p slice zd
  RowStage stg;
  if (g0 < g1) stg.fetch(a.rows, g0, g1, SP);
  for (int64_t c0 = g0; c0 < g1; c0 += kGkc) {
    __syncthreads();  // previous chunk done (and the tables above written)
    stg.store(rowbuf, a.rows, c0, g1, SP);
    __syncthreads();
    if (c0 + kGkc < g1) stg.fetch(a.rows, c0 + kGkc, g1, SP);
    // c_j for the chunk's samples
    double dot = 0.0;
    if (U) {
      const double* rj = rowbuf + jd * LD;
      for (int64_t p = zd; p < dp; p += 8) {
        double y = 1.0;
#pragma unroll
        for (int n = 0; n < NL; ++n) y *= rj[dig[p * NL + n]];
        dot = fma(y, uk[p], dot);
      }
      dot += __shfl_xor(dot, 4, 64);
      dot += __shfl_xor(dot, 2, 64);
      dot += __shfl_xor(dot, 1, 64);
    }
    if (zd == 0) {
      const int64_t u = c0 + jd;
      cfac[jd] = u < g1 ? (U ? fma(-a.scs[u], dot, xs[u]) : xs[u]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kResPer; ++i) {
      const int64_t p = tid + kBlock * i;
      if (p < dp) {
        double acc = v[i];
#pragma unroll 8
        for (int j = 0; j < kGkc; ++j) {
          const double* rj = rowbuf + j * LD;
          double y = cfac[j];
#pragma unroll
          for (int n = 0; n < NL; ++n) y *= rj[od[i][n]];
          acc += y;
        }
        v[i] = acc;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kResPer; ++i) {
    const int64_t p = tid + kBlock * i;
    if (p < dp) V[k * dp + p] = v[i];
  }
}

// The same sums on FP64 MFMA, for d'' = prod_{n<L-1} R_n <= 64 and R_{L-1} <= 64.
// With y_t = o_t (x) b_t (o_t over the modes before L - 1, b_t the row of mode
// L - 1) and U2_k = u_k as a d'' x R_{L-1} matrix,
//   y_t . u_k = o_t^T U2_k b_t,  sum_t c_t y_t = vec(sum_t c_t o_t b_t^T),
// so per chunk of 32 samples Z = O U2 (32 x R_{L-1}) and V2 += O^T diag(c) B
// (d'' x R_{L-1}) are 16 x 16 block products.  Wave w takes the Z blocks and
// the V2 blocks congruent to w mod 4; each block's sums run in a fixed order.
constexpr int kRmMax = 64;
template <int NL>
__global__ __launch_bounds__(kBlock) void grp_resid_mfma_kernel(Geom g, GrpArgs a,
                                                                const double* __restrict__ xs,
                                                                const double* __restrict__ U,
                                                                double* __restrict__ V) {
  extern __shared__ double smem[];  // rows [kGkc][S' + 1], u_k [d'' R1]
  __shared__ double cfac[kGkc];
  __shared__ double zpart[kRmMax / 16][kGkc];
  __shared__ int od[kRmMax][NL > 1 ? NL - 1 : 1];  // row offsets of o's digits
  const int SP = a.sp, LD = a.sp + 1;
  const int R1 = g.ranks[NL - 1];
  const int nd = static_cast<int>(a.dp / R1);  // d''
  const int nc1 = (R1 + 15) / 16, nr0 = (nd + 15) / 16;
  const int sb = g.soff[NL - 1];
  double* rowbuf = smem;
  double* uk = smem + kGkc * LD;
  const int64_t k = blockIdx.x;
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (U)
    for (int e = tid; e < nd * R1; e += kBlock) uk[e] = U[k * a.dp + e];
  for (int p0 = tid; p0 < nd; p0 += kBlock) {
    int x = p0;
#pragma unroll
    for (int n = NL - 2; n >= 0; --n) {
      const int R = g.ranks[n];
      od[p0][n] = g.soff[n] + x % R;
      x /= R;
    }
  }
  // o_j[p0] from the staged rows (1 when no mode precedes L - 1)
  auto o_of = [&](int j, int p0) {
    double x = 1.0;
    const double* rj = rowbuf + j * LD;
#pragma unroll
    for (int n = 0; n < NL - 1; ++n) x *= rj[od[p0][n]];
    return x;
  };
  const int nbv = nr0 * nc1;      // V2 blocks
  doublex4 accv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) accv[i] = doublex4{0.0, 0.0, 0.0, 0.0};
  RowStage stg;
  if (g0 < g1) stg.fetch(a.rows, g0, g1, SP);
  for (int64_t c0 = g0; c0 < g1; c0 += kGkc) {
    __syncthreads();  // the previous chunk is done (and the tables above are written)
    stg.store(rowbuf, a.rows, c0, g1, SP);
    __syncthreads();
    if (c0 + kGkc < g1) stg.fetch(a.rows, c0 + kGkc, g1, SP);
    if (U) {
      // Z blocks (sample half, column block): dots of o_j^T U2 with b_j
      for (int zb = w; zb < 2 * nc1; zb += 4) {
        const int sh = zb & 1, cbk = zb >> 1;
        doublex4 z = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < (nd + 3) / 4; ++ks) {
          const int p0 = ks * 4 + (lane >> 4);
          const int j = sh * 16 + (lane & 15);
          const int p1 = cbk * 16 + (lane & 15);
          const double av = p0 < nd ? o_of(j, p0) : 0.0;
          const double bv = (p0 < nd && p1 < R1) ? uk[p0 * R1 + p1] : 0.0;
          z = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, z, 0, 0, 0);
        }
        // accumulator v: sample sh 16 + lane / 16 + 4 v, column cbk 16 + lane % 16
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = sh * 16 + (lane >> 4) + 4 * v;
          const int p1 = cbk * 16 + (lane & 15);
          double t = p1 < R1 ? z[v] * rowbuf[j * LD + sb + p1] : 0.0;
          t = row16_sum(t);
          if ((lane & 15) == 0) zpart[cbk][j] = t;
        }
      }
      __syncthreads();
    }
    if (tid < kGkc) {
      const int64_t u = c0 + tid;
      double dot = 0.0;
      if (U)
        for (int c = 0; c < nc1; ++c) dot += zpart[c][tid];
      cfac[tid] = u < g1 ? (U ? fma(-a.scs[u], dot, xs[u]) : xs[u]) : 0.0;
    }
    __syncthreads();
    // V2 blocks (row block of o, column block of b) over the chunk's 32 samples
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = w + 4 * i;
      if (b < nbv) {
        const int rb = b / nc1, cb = b % nc1;
#pragma unroll 2
        for (int ks = 0; ks < kGkc / 4; ++ks) {
          const int j = ks * 4 + (lane >> 4);
          const int p0 = rb * 16 + (lane & 15);
          const int p1 = cb * 16 + (lane & 15);
          const double av = p0 < nd ? cfac[j] * o_of(j, p0) : 0.0;
          const double bv = p1 < R1 ? rowbuf[j * LD + sb + p1] : 0.0;
          accv[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accv[i], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = w + 4 * i;
    if (b < nbv) {
      const int rb = b / nc1, cb = b % nc1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p0 = rb * 16 + (lane >> 4) + 4 * v;
        const int p1 = cb * 16 + (lane & 15);
        if (p0 < nd && p1 < R1) V[k * a.dp + p0 * R1 + p1] = accv[i][v];
      }
    }
  }
}

// The same sums with every wave on its own 32 samples of each 128-sample
// chunk, for V2 of at most four 16 x 16 blocks: each wave takes the Z blocks
// and the factors c of its samples and accumulates every V2 block over them,
// so a chunk needs only the barriers around its staging and its factors (the
// 32-sample form above keeps one or two waves busy per chunk at d'' = R1 =
// 16).  The four waves' partial blocks are added in wave order through LDS at
// the end, so every sum keeps a fixed order.
constexpr int kRwc = 128;  // samples per chunk
template <int NL>
__global__ __launch_bounds__(kBlock) void grp_resid_wave_kernel(Geom g, GrpArgs a,
                                                                const double* __restrict__ xs,
                                                                const double* __restrict__ U,
                                                                double* __restrict__ V) {
  extern __shared__ double smem[];  // rows [kRwc][S' + 1] (then the reduction), u_k [d'' R1]
  __shared__ double cfac[kRwc];
  __shared__ double zpart[kRmMax / 16][kRwc];
  __shared__ int od[kRmMax][NL > 1 ? NL - 1 : 1];  // row offsets of o's digits
  const int SP = a.sp, LD = a.sp + 1;
  const int R1 = g.ranks[NL - 1];
  const int nd = static_cast<int>(a.dp / R1);  // d''
  const int nc1 = (R1 + 15) / 16, nr0 = (nd + 15) / 16;
  const int nbv = nr0 * nc1;  // V2 blocks, at most 4
  const int sb = g.soff[NL - 1];
  const int rsz = kRwc * LD > nbv * 256 ? kRwc * LD : nbv * 256;
  double* rowbuf = smem;
  double* uk = smem + rsz;
  const int64_t k = blockIdx.x;
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ws0 = w * 32;  // this wave's first sample in a chunk
  if (U)
    for (int e = tid; e < nd * R1; e += kBlock) uk[e] = U[k * a.dp + e];
  for (int p0 = tid; p0 < nd; p0 += kBlock) {
    int x = p0;
#pragma unroll
    for (int n = NL - 2; n >= 0; --n) {
      const int R = g.ranks[n];
      od[p0][n] = g.soff[n] + x % R;
      x /= R;
    }
  }
  // o_j[p0] from the staged rows (1 when no mode precedes L - 1)
  auto o_of = [&](int j, int p0) {
    double x = 1.0;
    const double* rj = rowbuf + j * LD;
#pragma unroll
    for (int n = 0; n < NL - 1; ++n) x *= rj[od[p0][n]];
    return x;
  };
  doublex4 accv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) accv[i] = doublex4{0.0, 0.0, 0.0, 0.0};
  ChunkStage<kRwc, 16> stg;
  if (g0 < g1) stg.fetch(a.rows, g0, g1, SP);
  for (int64_t c0 = g0; c0 < g1; c0 += kRwc) {
    __syncthreads();  // the previous chunk is done (and the tables above are written)
    stg.store(rowbuf, a.rows, c0, g1, SP);
    __syncthreads();
    if (c0 + kRwc < g1) stg.fetch(a.rows, c0 + kRwc, g1, SP);
    const int64_t nleft = g1 - c0 - ws0;  // samples of this wave in the chunk
    if (U && nleft > 0) {
      // Z blocks (16-sample half of this wave, column block): dots of o_j^T U2 with b_j
      for (int zb = 0; zb < 2 * nc1; ++zb) {
        const int sh = zb & 1, cbk = zb >> 1;
        if (sh * 16 >= nleft) continue;
        doublex4 z = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < (nd + 3) / 4; ++ks) {
          const int p0 = ks * 4 + (lane >> 4);
          const int j = ws0 + sh * 16 + (lane & 15);
          const int p1 = cbk * 16 + (lane & 15);
          const double av = p0 < nd ? o_of(j, p0) : 0.0;
          const double bv = (p0 < nd && p1 < R1) ? uk[p0 * R1 + p1] : 0.0;
          z = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, z, 0, 0, 0);
        }
        // accumulator v: sample ws0 + sh 16 + lane / 16 + 4 v, column cbk 16 + lane % 16
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = ws0 + sh * 16 + (lane >> 4) + 4 * v;
          const int p1 = cbk * 16 + (lane & 15);
          double t = p1 < R1 ? z[v] * rowbuf[j * LD + sb + p1] : 0.0;
          t = row16_sum(t);
          if ((lane & 15) == 0) zpart[cbk][j] = t;
        }
      }
    }
    __syncthreads();
    if (lane < 32) {
      const int j = ws0 + lane;
      const int64_t u = c0 + j;
      double dot = 0.0;
      if (U)
        for (int c = 0; c < nc1; ++c) dot += zpart[c][j];
      cfac[j] = u < g1 ? (U ? fma(-a.scs[u], dot, xs[u]) : xs[u]) : 0.0;
    }
    __syncthreads();
    // V2 blocks (row block of o, column block of b) over this wave's 32 samples
    if (nleft > 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nbv) {
          const int rb = i / nc1, cb = i % nc1;
#pragma unroll 2
          for (int ks = 0; ks < 8; ++ks) {
            if (4 * ks >= nleft) break;
            const int j = ws0 + ks * 4 + (lane >> 4);
            const int p0 = rb * 16 + (lane & 15);
            const int p1 = cb * 16 + (lane & 15);
            const double av = p0 < nd ? cfac[j] * o_of(j, p0) : 0.0;
            const double bv = p1 < R1 ? rowbuf[j * LD + sb + p1] : 0.0;
            accv[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accv[i], 0, 0, 0);
          }
        }
      }
    }
  }
  // ((wave 3 + wave 2) + wave 1) + wave 0 through LDS; accumulator v of lane
  // l: row l / 16 + 4 v, column l % 16 of its block
  double* red = smem;
  __syncthreads();
  for (int src = 3; src >= 0; --src) {
    if (w == src) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nbv) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int e = i * 256 + ((lane >> 4) + 4 * v) * 16 + (lane & 15);
            red[e] = src == 3 ? accv[i][v] : red[e] + accv[i][v];
          }
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nbv * 256; e += kBlock) {
    const int i = e >> 8, rem = e & 255;
    const int p0 = (i / nc1) * 16 + (rem >> 4), p1 = (i % nc1) * 16 + (rem & 15);
    if (p0 < nd && p1 < R1) V[k * a.dp + p0 * R1 + p1] = red[e];
  }
}

// out[p R_L + m] = sum_k V[k][p] e_k[m]: workgroup per 16 outputs, 16 threads
// per output summing groups z, z + 16, ... then a fixed shuffle tree
__global__ __launch_bounds__(kBlock) void grp_vec_expand_kernel(GrpArgs a,
                                                                const double* __restrict__ V,
                                                                double* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 16 + (threadIdx.x >> 4);
  const int z = threadIdx.x & 15;
  double sum = 0.0;
  if (e < a.dp * a.RL) {
    const int64_t p = e / a.RL;
    const int m = static_cast<int>(e % a.RL);
    for (int64_t k = z; k < a.groups; k += 16) sum = fma(V[k * a.dp + p], a.E[k * a.RL + m], sum);
  }
  sum += __shfl_xor(sum, 8, 64);
  sum += __shfl_xor(sum, 4, 64);
  sum += __shfl_xor(sum, 2, 64);
  sum += __shfl_xor(sum, 1, 64);
  if (e < a.dp * a.RL && z == 0) out[e] = sum;
}

// ------------------------------------------------------------------ pass 3: M
// Workgroup (row a of lower tile tau, block cb of 64 columns c = m (m + 1) / 2 + m',
// m' <= m): out[b][c] = sum_k B_k[tau][a][b] e_k[m] e_k[m'] for b in [0, 64), the
// pairs (p, p') = (64 ta + a, 64 tb + b).  The sum is symmetric in (m, m'), so only
// m' <= m is formed and, for p' < p, stored at both (p R_L + m, p' R_L + m') and
// (p R_L + m', p' R_L + m).  Wave w takes quadrant (w / 2, w % 2) of
// the 64 x 64 output on v_mfma_f64_4x4x4_4b (lane layout as in pass 2): per
// k-step of 4 groups, 8 row operands (rows b = 4 r .. 4 r + 3 of the
// quadrant, the same in all four blocks: B_k entries read straight from LDS)
// and 2 column operands (block q: columns 16 cc + 4 q .. + 3, the products
// e_k[m] e_k[m'] formed from LDS) feed 16 instructions; on a diagonal tile the
// rows above a are skipped.  Per chunk of 32 groups the B_k entries and the
// rows e_k (transposed, with a zero row for the padded columns) go to LDS from
// registers loaded during the previous chunk's products.  Workgroup ids are
// spread so that the column blocks of one row, which read the same B_k
// entries, run on one XCD (ids go round-robin over the 8 XCDs), and each XCD
// takes its rows in order.  NE >= R_L / 8.
// PAIR: the B_k are the pair form's C_k; row a of tile (tr, tc) is the pair i0 =
// {r >= r'} of mode 0 and the 64 operand rows b the pairs i1 = {s >= s'} of mode 1,
// all needed (no triangle), and each sum, symmetric in s <-> s' and m <-> m', goes
// to the up to four places (r, s1, m1; r', s2, m2) of M's lower triangle.
template <int NE, bool PAIR>
__global__ __launch_bounds__(kBlock) void grp_expand_kernel(Geom g, GrpArgs a, int ncb) {
  constexpr int kEld = kGkc + 2;  // transposed e_k stride
  __shared__ double as[kGkc][kGld];
  __shared__ double esT[(kMaxRank + 1) * kEld];
  // ids go round-robin over the 8 XCDs: XCD x takes the rows q = x mod 8 in
  // order, each with its ncb column blocks in a row
  const int64_t j = blockIdx.x / 8;
  const int cb = static_cast<int>(j % ncb);
  const int64_t qrow = (j / ncb) * 8 + blockIdx.x % 8;
  if (qrow >= a.ptiles * kGt) return;
  int64_t ta, tb;
  int arow;
  if (PAIR) {  // column-tile major: the ragged last column tile's rows come last
    const int64_t trn = a.ptiles / a.tcn;
    tb = qrow / (trn * kGt);
    const int64_t rem = qrow % (trn * kGt);
    ta = rem / kGt;
    arow = static_cast<int>(rem % kGt);
  } else {
    tri_index(qrow / kGt, ta, tb);
    arow = static_cast<int>(qrow % kGt);
  }
  const int64_t tau = PAIR ? ta * a.tcn + tb : qrow / kGt;
  const int64_t p = ta * kGt + arow;  // PAIR: the pair index i0
  if (p >= (PAIR ? a.n0 : a.dp)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = (lane >> 2) & 3, l4 = lane & 3, lk = lane >> 4;
  const int RL = a.RL;
  const int nc = RL * (RL + 1) / 2;  // column pairs m' <= m
  const int qa = w >> 1, qc = w & 1;
  const bool diag = !PAIR && ta == tb;
  // last row b needed: on a diagonal tile b <= arow; in the pair form the pairs
  const int blim = PAIR ? min(kGt - 1, a.n1 - 1 - static_cast<int>(tb) * kGt)
                        : diag ? arow : kGt - 1;
  // quadrant rows b >= 32 qa
  const bool active = qa * 32 <= blim && cb * 64 + qc * 32 < nc;
  // LDS indices (at k-step 0) of this lane's row and column operands
  int ia[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) ia[r] = lk * kGld + qa * 32 + 4 * r + l4;
  int im[2], imp[2];
  const float rlinv = 1.0f / static_cast<float>(RL);
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const int c = cb * 64 + qc * 32 + cc * 16 + 4 * q + l4;
    int m = RL, mp = 0;  // the zero row past the last pair
    if (c < nc) pair_of(c, m, mp);
    im[cc] = m * kEld + lk;
    imp[cc] = mp * kEld + lk;
  }
  for (int u = tid; u < kGkc; u += kBlock) esT[RL * kEld + u] = 0.0;
  // staging roles: B entries (group tid / 8, entries 8 (tid % 8) .. + 8) and
  // row elements tid + 256 i of the chunk's 32 R_L contiguous e_k entries
  const int skk = tid >> 3, se = (tid & 7) * 8;
  const double* Bsrc = a.B + tau * (kGt * kGt) + static_cast<int64_t>(arow) * kGt + se;
  const int64_t bstride = a.ptiles * (kGt * kGt);
  int eofs[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = tid + kBlock * i;
    int kk, m;
    small_divmod(e, RL, rlinv, kk, m);
    eofs[i] = e < kGkc * RL ? m * kEld + kk : -1;
  }
  double pa[8], pe[NE];
  auto fetch = [&](int64_t k0) {
    const bool kv = k0 + skk < a.groups;
    const double* src = Bsrc + (k0 + skk) * bstride;
#pragma unroll
    for (int e = 0; e < 8; ++e) pa[e] = kv ? src[e] : 0.0;
    const int64_t lim = ((a.groups < k0 + kGkc ? a.groups : k0 + kGkc) - k0) * RL;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + kBlock * i;
      pe[i] = e < lim ? a.E[k0 * RL + e] : 0.0;
    }
  };
  double acc[8][2];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[r][0] = acc[r][1] = 0.0;
  fetch(0);
  for (int64_t k0 = 0; k0 < a.groups; k0 += kGkc) {
#pragma unroll
    for (int e = 0; e < 8; ++e) as[skk][se + e] = pa[e];
#pragma unroll
    for (int i = 0; i < NE; ++i)
      if (eofs[i] >= 0) esT[eofs[i]] = pe[i];
    __syncthreads();
    if (k0 + kGkc < a.groups) fetch(k0 + kGkc);
    // PART: some rows of the quadrant lie above a diagonal tile's row a;
    // ONE: the quadrant's second 16 columns lie past the last pair
    auto ksteps = [&](auto part, auto one) __attribute__((always_inline)) {
      constexpr bool PART = decltype(part)::value;
      constexpr bool ONE = decltype(one)::value;
#pragma unroll
      for (int ks = 0; ks < kGkc / 4; ++ks) {
        const double f0 = esT[im[0] + 4 * ks] * esT[imp[0] + 4 * ks];
        const double f1 = ONE ? 0.0 : esT[im[1] + 4 * ks] * esT[imp[1] + 4 * ks];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          if (PART && qa * 32 + 4 * r > blim) continue;
          const double av = (&as[0][0])[ia[r] + 4 * ks * kGld];
          acc[r][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, f0, acc[r][0], 0, 0, 0);
          if (!ONE) acc[r][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, f1, acc[r][1], 0, 0, 0);
        }
      }
    };
    if (active) {
      const bool part = qa * 32 + 28 > blim;
      if (cb * 64 + qc * 32 + 16 < nc) {
        if (part)
          ksteps(std::true_type{}, std::false_type{});
        else
          ksteps(std::false_type{}, std::false_type{});
      } else {
        if (part)
          ksteps(std::true_type{}, std::true_type{});
        else
          ksteps(std::false_type{}, std::true_type{});
      }
    }
    __syncthreads();
  }
  if (!active) return;
  // epilogue: the pair's ridge term lambda prod_{n != L} P_n[digit_n(p)][digit_n(p')]
  // (modes after L: their 1 x 1 P_n) times P_L[m][m'], then the lower-triangle store;
  // accumulator lane l: row l / 16, column l % 4 of block (l / 4) % 4
  const int64_t d = g.d;
  const double* PL = a.P + g.roff[a.L];
  if (PAIR) {
    const int R0 = g.ranks[0], R1 = g.ranks[1];
    int r0, r0p;
    pair_of(static_cast<int>(p), r0, r0p);
    double lam = a.lambda;  // the modes after L: 1 x 1 P_n
    for (int n = a.L + 1; n < g.order; ++n) lam *= a.P[g.roff[n]];
    lam *= a.P[g.roff[0] + r0 * R0 + r0p];
    const double* P1 = a.P + g.roff[1];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i1 = static_cast<int>(tb) * kGt + qa * 32 + 4 * r + lk;
      if (i1 >= a.n1) continue;
      int s1, s1p;
      pair_of(i1, s1, s1p);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int c = cb * 64 + qc * 32 + cc * 16 + 4 * q + l4;
        if (c >= nc) continue;
        int m, mp;
        pair_of(c, m, mp);
        for (int o1 = 0; o1 < (s1 == s1p ? 1 : 2); ++o1) {
          const int sa = o1 ? s1p : s1, sb = o1 ? s1 : s1p;
          for (int o2 = 0; o2 < (m == mp ? 1 : 2); ++o2) {
            const int ma = o2 ? mp : m, mb = o2 ? m : mp;
            const int64_t row = static_cast<int64_t>(r0 * R1 + sa) * RL + ma;
            const int64_t col = static_cast<int64_t>(r0p * R1 + sb) * RL + mb;
            if (row < col) continue;
            a.M[row * d + col] = fma(lam * P1[sa * R1 + sb], PL[ma * RL + mb], acc[r][cc]);
          }
        }
      }
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int b = qa * 32 + 4 * r + lk;
    const int64_t pp = tb * kGt + b;
    if (pp >= a.dp || pp > p) continue;
    double pr = a.lambda;
    {
      int x = static_cast<int>(p), y = static_cast<int>(pp);
      for (int n = g.order - 1; n >= 0; --n) {
        if (n == a.L) continue;
        const int R = g.ranks[n];
        const float rinv = 1.0f / static_cast<float>(R);
        int qx, rx, qy, ry;
        small_divmod(x, R, rinv, qx, rx);
        small_divmod(y, R, rinv, qy, ry);
        pr *= a.P[g.roff[n] + rx * R + ry];
        x = qx;
        y = qy;
      }
    }
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const int c = cb * 64 + qc * 32 + cc * 16 + 4 * q + l4;
      if (c >= nc) continue;
      int m, mp;
      pair_of(c, m, mp);
      a.M[(p * RL + m) * d + pp * RL + mp] = fma(pr, PL[m * RL + mp], acc[r][cc]);
      if (pp < p && mp < m)
        a.M[(p * RL + mp) * d + pp * RL + m] = fma(pr, PL[mp * RL + m], acc[r][cc]);
    }
  }
}

// Carved pieces of the grouped Gram's scratch.
struct GrpWS {
  int32_t* rank;
  int32_t* perm;
  int32_t* cnt;
  int32_t* part;
  double* rows;
  double* scs;
  double* xs;
  double* U;
  double* V;
  double* B;
};

void carve_grouped(Carver& c, const GroupedPlan& gp, GrpWS& w) {
  w.rank = c.take<int32_t>(gp.s);
  w.perm = c.take<int32_t>(gp.s);
  w.cnt = c.take<int32_t>(gp.ncnt);
  w.part = c.take<int32_t>(gp.nparts);
  w.rows = c.take<double>(static_cast<size_t>(gp.s) * gp.sp);
  w.scs = c.take<double>(gp.s);
  w.xs = c.take<double>(gp.s);
  w.U = c.take<double>(static_cast<size_t>(gp.groups) * gp.dp);
  w.V = c.take<double>(static_cast<size_t>(gp.groups) * gp.dp);
  w.B = c.take<double>(static_cast<size_t>(gp.groups) * gp.ptiles * kGt * kGt);
}

// Register sizes of the two MFMA passes' staging.
int block_nr(int sp) { return sp <= 16 ? 2 : sp <= 32 ? 4 : sp <= 64 ? 8 : 17; }
int expand_ne(int rl) { return rl <= 8 ? 1 : rl <= 16 ? 2 : rl <= 32 ? 4 : 8; }

template <int NR>
void launch_block(const Geom& gr, const GrpArgs& a, unsigned grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(grp_block_kernel<NR>, dim3(grid), dim3(kBlock), lds, st, gr, a);
}
template <int NR, int NL, int CK, bool PAIR = false>
void launch_block_split(const Geom& gr, const GrpArgs& a, hipStream_t st) {
  const size_t lds =
      (static_cast<size_t>(a.sp + 1) * (CK + 2) + static_cast<size_t>(kGt) * kRld) * sizeof(double);
  if (lds > 65536)
    ensure_dyn_lds(reinterpret_cast<const void*>(grp_block_split_kernel<NR, NL, CK, PAIR>),
                   static_cast<int>(lds));
  const int64_t nunits = a.groups * a.ptiles;
  // the pair form's grid: 8 XCDs x (groups k = x mod 8) x tiles
  const int64_t nwg = PAIR ? 8 * cdiv(a.groups, 8) * a.ptiles : cdiv(nunits, 8) * 8;
  hipLaunchKernelGGL((grp_block_split_kernel<NR, NL, CK, PAIR>),
                     dim3(static_cast<unsigned>(nwg)), dim3(kBlock), lds, st, gr, a, nunits);
}
template <int NR, int CK>
void launch_block_split_nl(const Geom& gr, const GrpArgs& a, hipStream_t st) {
  switch (a.L) {
    case 1: launch_block_split<NR, 1, CK>(gr, a, st); break;
    case 2:
      if (a.tcn > 0)
        launch_block_split<NR, 2, CK, true>(gr, a, st);
      else
        launch_block_split<NR, 2, CK>(gr, a, st);
      break;
    default: launch_block_split<NR, 3, CK>(gr, a, st); break;
  }
}
template <int NE>
void launch_expand(const Geom& gr, const GrpArgs& a, int ncb, bool pair, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(cdiv(a.ptiles * kGt, 8) * 8 * ncb));
  if (pair)
    hipLaunchKernelGGL((grp_expand_kernel<NE, true>), grid, dim3(kBlock), 0, st, gr, a, ncb);
  else
    hipLaunchKernelGGL((grp_expand_kernel<NE, false>), grid, dim3(kBlock), 0, st, gr, a, ncb);
}

}  // namespace

GroupedPlan plan_grouped(const Geom& gr, int64_t s, tk_dtype prec) {
  GroupedPlan gp;
  memset(&gp, 0, sizeof(gp));
  if (prec != TK_F64 || s < 1 || s >= (int64_t(1) << 31)) return gp;
  const int L = gr.last;
  const int RL = gr.ranks[L];
  if (RL < 2 || gr.d < 256) return gp;
  gp.L = L;
  gp.RL = RL;
  gp.s = s;
  gp.dp = gr.d / RL;
  gp.groups = gr.dims[L];
  gp.nb = cdiv(s, kBlock);
  gp.ncnt = gp.groups * gp.nb + 1;
  gp.nparts = cdiv(gp.ncnt, kScanPer);
  const int64_t pt = cdiv(gp.dp, kGt);
  gp.ptiles = pt * (pt + 1) / 2;
  gp.sp = gr.soff[L];
  if (gp.ncnt > (int64_t(1) << 24) || gp.groups * gp.ptiles >= (int64_t(1) << 31) ||
      s * gp.sp >= (int64_t(1) << 31) || gp.sp > 17 * kBlock / kGkc || gp.dp >= (int64_t(1) << 20))
    return gp;
  // multiply-adds of the two forms (tiles padded to 64): grouped only when
  // clearly fewer, and B_k within 4 GiB
  const double dd = static_cast<double>(gr.d);
  const double plain = static_cast<double>(s) * dd * dd * 0.5;
  const double tile = static_cast<double>(kGt * kGt) * static_cast<double>(gp.ptiles);
  const double grouped = tile * (static_cast<double>(s) + static_cast<double>(gp.groups) * RL * RL);
  const double bbytes = tile * static_cast<double>(gp.groups) * 8.0;
  if (grouped * 3.0 > plain || bbytes > 4.0 * 1024 * 1024 * 1024) return gp;
  if (L == 2) {  // the pair form, where it takes no more tiles
    const int n0 = gr.ranks[0] * (gr.ranks[0] + 1) / 2, n1 = gr.ranks[1] * (gr.ranks[1] + 1) / 2;
    const int64_t t0 = cdiv(n0, kGt), t1 = cdiv(n1, kGt);
    if (t0 * t1 <= gp.ptiles) {
      gp.pair = 1;
      gp.n0 = n0;
      gp.n1 = n1;
      gp.tcn = static_cast<int32_t>(t1);
      gp.ptiles = t0 * t1;
    }
  }
  gp.on = 1;
  return gp;
}

size_t grouped_bytes(const GroupedPlan& gp) {
  Carver c(nullptr);
  GrpWS w;
  carve_grouped(c, gp, w);
  return c.used;
}

void launch_grouped_gram(const Geom& gr, const GroupedPlan& gp, const int32_t* idx,
                         const double* Q64, const double* weff, const double* xw, const double* P,
                         double lambda, void* ws, double* M, hipStream_t st) {
  Carver c(ws);
  GrpWS w;
  carve_grouped(c, gp, w);
  const int32_t* key = idx + static_cast<int64_t>(gp.L) * gp.s;
  launch_fill_i32(gp.ncnt, 0, w.cnt, st);
  hipLaunchKernelGGL(grp_count_kernel, dim3(static_cast<unsigned>(gp.nb)), dim3(kBlock), 0, st,
                     key, gp.s, gp.groups, gp.nb, w.rank, w.cnt);
  hipLaunchKernelGGL(grp_scan_reduce_kernel, dim3(static_cast<unsigned>(gp.nparts)), dim3(kBlock),
                     0, st, w.cnt, gp.ncnt, w.part);
  hipLaunchKernelGGL(grp_scan_top_kernel, dim3(1), dim3(kBlock), 0, st, w.part, gp.nparts);
  hipLaunchKernelGGL(grp_scan_apply_kernel, dim3(static_cast<unsigned>(gp.nparts)), dim3(kBlock),
                     0, st, w.cnt, gp.ncnt, w.part);
  hipLaunchKernelGGL(grp_scatter_kernel, dim3(static_cast<unsigned>(gp.nb)), dim3(kBlock), 0, st,
                     key, gp.s, gp.groups, gp.nb, w.rank, w.cnt, w.perm);
  const int64_t nel = gp.s * gp.sp;
  hipLaunchKernelGGL(grp_rows_kernel, dim3(static_cast<unsigned>(cdiv(nel, kBlock))), dim3(kBlock),
                     0, st, gr, idx, gp.s, Q64, weff, xw, w.perm, gp.L, gp.sp, w.rows, w.scs,
                     w.xs);
  GrpArgs a;
  a.rows = w.rows;
  a.scs = w.scs;
  a.cnt = w.cnt;
  a.B = w.B;
  a.E = Q64 + gr.qoff[gp.L];
  a.P = P;
  a.lambda = lambda;
  a.M = M;
  a.nb = gp.nb;
  a.groups = gp.groups;
  a.dp = gp.dp;
  a.ptiles = gp.ptiles;
  a.L = gp.L;
  a.RL = gp.RL;
  a.sp = gp.sp;
  a.tcn = gp.pair ? gp.tcn : 0;
  a.n0 = gp.n0;
  a.n1 = gp.n1;
  const unsigned grid = static_cast<unsigned>(gp.groups * gp.ptiles);
  const size_t lds = static_cast<size_t>(kGkc) * (gp.sp + 1) * sizeof(double);
  if (gp.L <= 3) {  // every wave the whole tile over a quarter of each chunk
    // staging registers: CK S' / 256 doubles per thread
    if (split_ck(gp.sp) == 64) {
      if (gp.sp <= 16)
        launch_block_split_nl<4, 64>(gr, a, st);
      else
        launch_block_split_nl<8, 64>(gr, a, st);
    } else {
      if (gp.sp <= 64)
        launch_block_split_nl<8, 32>(gr, a, st);
      else
        launch_block_split_nl<17, 32>(gr, a, st);
    }
  } else {
    switch (block_nr(gp.sp)) {
      case 2: launch_block<2>(gr, a, grid, lds, st); break;
      case 4: launch_block<4>(gr, a, grid, lds, st); break;
      case 8: launch_block<8>(gr, a, grid, lds, st); break;
      default: launch_block<17>(gr, a, grid, lds, st); break;
    }
  }
  const int ncb = static_cast<int>(cdiv(static_cast<int64_t>(gp.RL) * (gp.RL + 1) / 2, kGt));
  switch (expand_ne(gp.RL)) {
    case 1: launch_expand<1>(gr, a, ncb, gp.pair != 0, st); break;
    case 2: launch_expand<2>(gr, a, ncb, gp.pair != 0, st); break;
    case 4: launch_expand<4>(gr, a, ncb, gp.pair != 0, st); break;
    default: launch_expand<8>(gr, a, ncb, gp.pair != 0, st); break;
  }
}

bool grouped_resid_ok(const GroupedPlan& gp) {
  return gp.on && gp.L <= 3 && gp.dp <= int64_t(kResPer) * kBlock;
}

void launch_grouped_resid(const Geom& gr, const GroupedPlan& gp, const double* Q64, void* ws,
                          const double* h, double* out, hipStream_t st) {
  Carver c(ws);
  GrpWS w;
  carve_grouped(c, gp, w);
  GrpArgs a;
  memset(&a, 0, sizeof(a));
  a.rows = w.rows;
  a.scs = w.scs;
  a.cnt = w.cnt;
  a.E = Q64 + gr.qoff[gp.L];
  a.nb = gp.nb;
  a.groups = gp.groups;
  a.dp = gp.dp;
  a.L = gp.L;
  a.RL = gp.RL;
  a.sp = gp.sp;
  if (h)
    hipLaunchKernelGGL(grp_hvec_kernel, dim3(static_cast<unsigned>(cdiv(gp.groups * gp.dp, kBlock))),
                       dim3(kBlock), 0, st, a, h, w.U);
  const size_t lds = static_cast<size_t>(kGkc) * (gp.sp + 1) * sizeof(double) +
                     static_cast<size_t>(gp.dp) * sizeof(double) +
                     static_cast<size_t>(gp.dp) * gp.L * sizeof(int);
  const dim3 grid(static_cast<unsigned>(gp.groups));
  const double* U = h ? w.U : nullptr;
  const int R1 = gr.ranks[gp.L - 1];
  const int nd = static_cast<int>(gp.dp / R1);
  if (R1 <= kRmMax && nd <= kRmMax && ((nd + 15) / 16) * ((R1 + 15) / 16) <= 4) {
    const size_t rsz = static_cast<size_t>(kRwc) * (gp.sp + 1) > static_cast<size_t>(
                                                                      ((nd + 15) / 16) * ((R1 + 15) / 16) * 256)
                           ? static_cast<size_t>(kRwc) * (gp.sp + 1)
                           : static_cast<size_t>(((nd + 15) / 16) * ((R1 + 15) / 16) * 256);
    const size_t lds_w = (rsz + static_cast<size_t>(gp.dp)) * sizeof(double);
    switch (gp.L) {
      case 1:
        if (lds_w > 65536)
          ensure_dyn_lds(reinterpret_cast<const void*>(grp_resid_wave_kernel<1>), static_cast<int>(lds_w));
        hipLaunchKernelGGL(grp_resid_wave_kernel<1>, grid, dim3(kBlock), lds_w, st, gr, a, w.xs, U,
                           w.V);
        break;
      case 2:
        if (lds_w > 65536)
          ensure_dyn_lds(reinterpret_cast<const void*>(grp_resid_wave_kernel<2>), static_cast<int>(lds_w));
        hipLaunchKernelGGL(grp_resid_wave_kernel<2>, grid, dim3(kBlock), lds_w, st, gr, a, w.xs, U,
                           w.V);
        break;
      default:
        if (lds_w > 65536)
          ensure_dyn_lds(reinterpret_cast<const void*>(grp_resid_wave_kernel<3>), static_cast<int>(lds_w));
        hipLaunchKernelGGL(grp_resid_wave_kernel<3>, grid, dim3(kBlock), lds_w, st, gr, a, w.xs, U,
                           w.V);
        break;
    }
  } else if (R1 <= kRmMax && nd <= kRmMax) {
    const size_t lds_m = static_cast<size_t>(kGkc) * (gp.sp + 1) * sizeof(double) +
                         static_cast<size_t>(gp.dp) * sizeof(double);
    switch (gp.L) {
      case 1:
        hipLaunchKernelGGL(grp_resid_mfma_kernel<1>, grid, dim3(kBlock), lds_m, st, gr, a, w.xs, U,
                           w.V);
        break;
      case 2:
        hipLaunchKernelGGL(grp_resid_mfma_kernel<2>, grid, dim3(kBlock), lds_m, st, gr, a, w.xs, U,
                           w.V);
        break;
      default:
        hipLaunchKernelGGL(grp_resid_mfma_kernel<3>, grid, dim3(kBlock), lds_m, st, gr, a, w.xs, U,
                           w.V);
        break;
    }
  } else switch (gp.L) {
    case 1:
      hipLaunchKernelGGL(grp_resid_kernel<1>, grid, dim3(kBlock), lds, st, gr, a, w.xs, U, w.V);
      break;
    case 2:
      hipLaunchKernelGGL(grp_resid_kernel<2>, grid, dim3(kBlock), lds, st, gr, a, w.xs, U, w.V);
      break;
    default:
      hipLaunchKernelGGL(grp_resid_kernel<3>, grid, dim3(kBlock), lds, st, gr, a, w.xs, U, w.V);
      break;
  }
  hipLaunchKernelGGL(grp_vec_expand_kernel, dim3(static_cast<unsigned>(cdiv(gp.dp * gp.RL, 16))),
                     dim3(kBlock), 0, st, a, w.V, out);
}

}  // namespace tk
