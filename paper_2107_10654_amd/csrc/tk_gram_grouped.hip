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
//     tile of d' x d'), y_t formed in LDS per chunk of 32 samples of the
//     group (in their original order, so every sum has a fixed order);
//  3. M[p R_L + m][p' R_L + m'] = sum_k B_k[p][p'] e_k[m] e_k[m']
//     + lambda prod_n P_n[..][..] on the lower triangle: a GEMM over the
//     groups on the same MFMA, with the ridge term's Kronecker product in
//     its epilogue.
#include <string.h>

#include "tk_mfma.h"

namespace tk {
namespace {

constexpr int kGt = 64;        // tile edge over d' (pass 2) and q-row block (pass 3)
constexpr int kGkc = 32;       // samples (pass 2) or groups (pass 3) per LDS chunk
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
};

// ------------------------------------------------------------------ pass 2: B_k
// Sorted sample rows: element e = u S' + j holds entry j of the concatenated
// rows of modes < L of sample t = perm[u]; scs[u] = w_t prod_{n>L} q^(n)_{i_n}[0]^2.
__global__ __launch_bounds__(kBlock) void grp_rows_kernel(Geom g, const int32_t* __restrict__ idx,
                                                          int64_t s, const double* __restrict__ Q64,
                                                          const double* __restrict__ weff,
                                                          const int32_t* __restrict__ perm, int L,
                                                          int sp, double* __restrict__ rows,
                                                          double* __restrict__ scs) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= s * sp) return;
  const int64_t u = e / sp;
  const int j = static_cast<int>(e - u * sp);
  const int64_t t = perm[u];
  int n = 0;
  while (n + 1 < L && g.soff[n + 1] <= j) ++n;
  int32_t i = idx[static_cast<int64_t>(n) * s + t];
  if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
  rows[e] = Q64[g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n] + (j - g.soff[n])];
  if (j == 0) {
    double sc = weff[t];
    for (int m = L + 1; m < g.order; ++m) {
      int32_t im = idx[static_cast<int64_t>(m) * s + t];
      if (im < 0 || im >= g.dims[m]) im = 0;
      const double q = Q64[g.qoff[m] + im];  // rank 1
      sc *= q * q;
    }
    scs[u] = sc;
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

// ------------------------------------------------------------------ pass 3: M
// Workgroup (row a of lower tile tau, block cb of 64 columns c = m R_L + m'):
// out[b][c] = sum_k B_k[tau][a][b] e_k[m] e_k[m'] for b in [0, 64), the pairs
// (p, p') = (64 ta + a, 64 tb + b).  Wave w takes quadrant (w / 2, w % 2) of
// the 64 x 64 output.  Per chunk of 32 groups the B_k entries and the rows e_k
// go to LDS from registers loaded during the previous chunk's products; each
// lane forms its e_k[m] e_k[m'] operands from LDS.  Workgroup ids are spread
// so that the column blocks of one row, which read the same B_k entries, run
// on one XCD (ids go round-robin over the 8 XCDs).  NE >= R_L / 8.
template <int NE>
__global__ __launch_bounds__(kBlock) void grp_expand_kernel(Geom g, GrpArgs a, int64_t nunits,
                                                            int ncb) {
  __shared__ double as[kGkc][kGld];
  __shared__ double es[kGkc * kMaxRank];
  const int64_t per_xcd = static_cast<int64_t>(gridDim.x) / 8;
  const int64_t unit = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (unit >= nunits) return;
  const int cb = static_cast<int>(unit % ncb);
  const int64_t qrow = unit / ncb;
  const int64_t tau = qrow / kGt;
  const int arow = static_cast<int>(qrow % kGt);
  int64_t ta, tb;
  tri_index(tau, ta, tb);
  const int64_t p = ta * kGt + arow;
  if (p >= a.dp) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int RL = a.RL;
  const int rr = RL * RL;
  const int qa = w >> 1, qc = w & 1;
  // quadrant rows b >= 32 qa; on a diagonal tile only b <= arow is stored
  const bool active = !(ta == tb && qa * 32 > arow) && cb * 64 + qc * 32 < rr;
  // this lane's two operand columns c -> (m, m')
  int fm[2], fmp[2];
  bool fv[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int c = cb * 64 + qc * 32 + j * 16 + (lane & 15);
    fv[j] = c < rr;
    fm[j] = fv[j] ? c / RL : 0;
    fmp[j] = fv[j] ? c % RL : 0;
  }
  // staging roles: B entries (group tid / 8, entries 8 (tid % 8) .. + 8) and
  // row elements tid + 256 i of the chunk's 32 R_L contiguous e_k entries
  const int skk = tid >> 3, se = (tid & 7) * 8;
  const double* Bsrc = a.B + tau * (kGt * kGt) + static_cast<int64_t>(arow) * kGt + se;
  const int64_t bstride = a.ptiles * (kGt * kGt);
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
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int64_t k0 = 0; k0 < a.groups; k0 += kGkc) {
#pragma unroll
    for (int e = 0; e < 8; ++e) as[skk][se + e] = pa[e];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + kBlock * i;
      if (e < kGkc * RL) es[e] = pe[i];
    }
    __syncthreads();
    if (k0 + kGkc < a.groups) fetch(k0 + kGkc);
    if (active) {
#pragma unroll 2
      for (int ks = 0; ks < kGkc / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        const double a0 = as[kk][qa * 32 + (lane & 15)];
        const double a1 = as[kk][qa * 32 + 16 + (lane & 15)];
        const double* ek = es + kk * RL;
        const double f0 = fv[0] ? ek[fm[0]] * ek[fmp[0]] : 0.0;
        const double f1 = fv[1] ? ek[fm[1]] * ek[fmp[1]] : 0.0;
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, f0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, f1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, f0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, f1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (!active) return;
  // epilogue: the pair's ridge term lambda prod_{n != L} P_n[digit_n(p)][digit_n(p')]
  // (modes after L: their 1 x 1 P_n) times P_L[m][m'], then the lower-triangle store
  const int64_t d = g.d;
  const double* PL = a.P + g.roff[a.L];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = qa * 32 + i * 16 + (lane >> 4) + 4 * v;
      const int64_t pp = tb * kGt + b;
      if (pp >= a.dp || pp > p) continue;
      double pr = a.lambda;
      {
        int64_t x = p, y = pp;
        for (int n = g.order - 1; n >= 0; --n) {
          if (n == a.L) continue;
          const int R = g.ranks[n];
          pr *= a.P[g.roff[n] + (x % R) * R + (y % R)];
          x /= R;
          y /= R;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = cb * 64 + qc * 32 + j * 16 + (lane & 15);
        if (c >= rr) continue;
        const int m = c / RL, mp = c % RL;
        if (pp == p && mp > m) continue;
        a.M[(p * RL + m) * d + pp * RL + mp] = fma(pr, PL[m * RL + mp], acc[i][j][v]);
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
  double* B;
};

void carve_grouped(Carver& c, const GroupedPlan& gp, GrpWS& w) {
  w.rank = c.take<int32_t>(gp.s);
  w.perm = c.take<int32_t>(gp.s);
  w.cnt = c.take<int32_t>(gp.ncnt);
  w.part = c.take<int32_t>(gp.nparts);
  w.rows = c.take<double>(static_cast<size_t>(gp.s) * gp.sp);
  w.scs = c.take<double>(gp.s);
  w.B = c.take<double>(static_cast<size_t>(gp.groups) * gp.ptiles * kGt * kGt);
}

// Register sizes of the two MFMA passes' staging.
int block_nr(int sp) { return sp <= 16 ? 2 : sp <= 32 ? 4 : sp <= 64 ? 8 : 17; }
int expand_ne(int rl) { return rl <= 8 ? 1 : rl <= 16 ? 2 : rl <= 32 ? 4 : 8; }

template <int NR>
void launch_block(const Geom& gr, const GrpArgs& a, unsigned grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(grp_block_kernel<NR>, dim3(grid), dim3(kBlock), lds, st, gr, a);
}
template <int NE>
void launch_expand(const Geom& gr, const GrpArgs& a, int64_t nunits, int ncb, hipStream_t st) {
  hipLaunchKernelGGL(grp_expand_kernel<NE>, dim3(static_cast<unsigned>(cdiv(nunits, 8) * 8)),
                     dim3(kBlock), 0, st, gr, a, nunits, ncb);
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
      s * gp.sp >= (int64_t(1) << 31) || gp.sp > 17 * kBlock / kGkc)
    return gp;
  // multiply-adds of the two forms (tiles padded to 64): grouped only when
  // clearly fewer, and B_k within 4 GiB
  const double dd = static_cast<double>(gr.d);
  const double plain = static_cast<double>(s) * dd * dd * 0.5;
  const double tile = static_cast<double>(kGt * kGt) * static_cast<double>(gp.ptiles);
  const double grouped = tile * (static_cast<double>(s) + static_cast<double>(gp.groups) * RL * RL);
  const double bbytes = tile * static_cast<double>(gp.groups) * 8.0;
  if (grouped * 3.0 > plain || bbytes > 4.0 * 1024 * 1024 * 1024) return gp;
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
                         const double* Q64, const double* weff, const double* P, double lambda,
                         void* ws, double* M, hipStream_t st) {
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
                     0, st, gr, idx, gp.s, Q64, weff, w.perm, gp.L, gp.sp, w.rows, w.scs);
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
  const unsigned grid = static_cast<unsigned>(gp.groups * gp.ptiles);
  const size_t lds = static_cast<size_t>(kGkc) * (gp.sp + 1) * sizeof(double);
  switch (block_nr(gp.sp)) {
    case 2: launch_block<2>(gr, a, grid, lds, st); break;
    case 4: launch_block<4>(gr, a, grid, lds, st); break;
    case 8: launch_block<8>(gr, a, grid, lds, st); break;
    default: launch_block<17>(gr, a, grid, lds, st); break;
  }
  const int ncb = static_cast<int>(cdiv(static_cast<int64_t>(gp.RL) * gp.RL, kGt));
  const int64_t nunits = gp.ptiles * kGt * ncb;
  switch (expand_ne(gp.RL)) {
    case 1: launch_expand<1>(gr, a, nunits, ncb, st); break;
    case 2: launch_expand<2>(gr, a, nunits, ncb, st); break;
    case 4: launch_expand<4>(gr, a, nunits, ncb, st); break;
    default: launch_expand<8>(gr, a, nunits, ncb, st); break;
  }
}

}  // namespace tk
