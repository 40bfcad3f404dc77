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
  const int32_t* idx;   // [order][s]
  const double* Q64;    // whitened rows at geom.qoff
  const double* weff;   // per sample
  const int32_t* perm;  // samples by key
  const int32_t* cnt;   // scanned count table: group k is perm[cnt[k nb], cnt[(k + 1) nb])
  double* B;            // [group][lower tile][64][64]
  const double* P;      // (L_n^T L_n)^{-1} at geom.roff
  double lambda;
  double* M;            // d x d, lower triangle written
  int64_t s, nb, groups, dp, ptiles;
  int32_t L, RL;
};

// ------------------------------------------------------------------ pass 2: B_k
// Workgroup (group k, lower tile (ta, tb) of d' x d').  Thread (wave w, lane l)
// forms rows pa = 64 ta + l (times w_t) and pb = 64 tb + l of y_t for samples
// w, w + 4, ... of each chunk; wave w then multiplies quadrant (w / 2, w % 2)
// of the tile (the upper quadrant of a diagonal tile is left zero).
__global__ __launch_bounds__(kBlock) void grp_block_kernel(Geom g, GrpArgs a) {
  __shared__ double ya[kGkc][kGld];
  __shared__ double yb[kGkc][kGld];
  __shared__ int64_t sbase[kGkc][kMaxOrder];
  __shared__ double ssc[kGkc];
  const int64_t tau = blockIdx.x % a.ptiles;
  const int64_t k = blockIdx.x / a.ptiles;
  int64_t ta, tb;
  tri_index(tau, ta, tb);
  const int64_t g0 = a.cnt[k * a.nb], g1 = a.cnt[(k + 1) * a.nb];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int L = a.L;
  const int64_t pa = ta * kGt + lane, pb = tb * kGt + lane;
  const bool va = pa < a.dp, vb = pb < a.dp;
  int da[kMaxOrder], db[kMaxOrder];
  {
    int64_t xa = va ? pa : 0, xb = vb ? pb : 0;
#pragma unroll
    for (int n = kMaxOrder - 1; n >= 0; --n) {
      da[n] = 0;
      db[n] = 0;
      if (n < L) {
        const int R = g.ranks[n];
        da[n] = static_cast<int>(xa % R);
        db[n] = static_cast<int>(xb % R);
        xa /= R;
        xb /= R;
      }
    }
  }
  const int qa = w >> 1, qb = w & 1;
  const bool active = !(ta == tb && qa < qb);
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = g0; c0 < g1; c0 += kGkc) {
    if (tid < kGkc) {  // the chunk's samples: row offsets of modes < L, w_t times modes > L
      const int64_t u = c0 + tid;
      double sc = 0.0;
      if (u < g1) {
        const int64_t t = a.perm[u];
        sc = a.weff[t];
        for (int n = 0; n < g.order; ++n) {
          int32_t i = a.idx[static_cast<int64_t>(n) * a.s + t];
          if (i < 0 || i >= g.dims[n]) i = 0;
          const int64_t off = g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n];
          if (n < L) sbase[tid][n] = off;
          if (n > L) sc *= a.Q64[off] * a.Q64[off];
        }
      } else {
        for (int n = 0; n < L; ++n) sbase[tid][n] = g.qoff[n];
      }
      ssc[tid] = sc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kGkc / 4; ++i) {
      const int j = w + 4 * i;
      double xa = ssc[j], xb = 1.0;
#pragma unroll
      for (int n = 0; n < kMaxOrder; ++n) {
        if (n < L) {
          xa *= a.Q64[sbase[j][n] + da[n]];
          xb *= a.Q64[sbase[j][n] + db[n]];
        }
      }
      ya[j][lane] = va ? xa : 0.0;
      yb[j][lane] = vb ? xb : 0.0;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int ks = 0; ks < kGkc / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        const double a0 = ya[kk][qa * 32 + (lane & 15)];
        const double a1 = ya[kk][qa * 32 + 16 + (lane & 15)];
        const double b0 = yb[kk][qb * 32 + (lane & 15)];
        const double b1 = yb[kk][qb * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
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
// the 64 x 64 output.  Workgroup ids are spread so that the column blocks of
// one row, which read the same B entries, run on one XCD (ids go round-robin
// over the 8 XCDs).
__global__ __launch_bounds__(kBlock) void grp_expand_kernel(Geom g, GrpArgs a, int64_t nunits,
                                                            int ncb) {
  __shared__ double as[kGkc][kGld];
  __shared__ double fs[kGkc][kGld];
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
  // staging roles: group kk = tid / 8, entries 8 (tid % 8) .. + 8
  const int skk = tid >> 3, se = (tid & 7) * 8;
  const double* Bsrc = a.B + tau * (kGt * kGt) + static_cast<int64_t>(arow) * kGt + se;
  const int64_t bstride = a.ptiles * (kGt * kGt);
  const double* E = a.Q64 + g.qoff[a.L];
  int fm[8], fmp[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = cb * 64 + se + e;
    fm[e] = c < rr ? c / RL : -1;
    fmp[e] = c < rr ? c % RL : 0;
  }
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < a.groups; k0 += kGkc) {
    const int64_t k = k0 + skk;
    if (k < a.groups) {
      const double* src = Bsrc + k * bstride;
      const double* ek = E + k * RL;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        as[skk][se + e] = src[e];
        fs[skk][se + e] = fm[e] >= 0 ? ek[fm[e]] * ek[fmp[e]] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        as[skk][se + e] = 0.0;
        fs[skk][se + e] = 0.0;
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int ks = 0; ks < kGkc / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        const double a0 = as[kk][qa * 32 + (lane & 15)];
        const double a1 = as[kk][qa * 32 + 16 + (lane & 15)];
        const double f0 = fs[kk][qc * 32 + (lane & 15)];
        const double f1 = fs[kk][qc * 32 + 16 + (lane & 15)];
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
  double* B;
};

void carve_grouped(Carver& c, const GroupedPlan& gp, GrpWS& w) {
  w.rank = c.take<int32_t>(gp.s);
  w.perm = c.take<int32_t>(gp.s);
  w.cnt = c.take<int32_t>(gp.ncnt);
  w.part = c.take<int32_t>(gp.nparts);
  w.B = c.take<double>(static_cast<size_t>(gp.groups) * gp.ptiles * kGt * kGt);
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
  if (gp.ncnt > (int64_t(1) << 24) || gp.groups * gp.ptiles >= (int64_t(1) << 31)) return gp;
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
  GrpArgs a;
  a.idx = idx;
  a.Q64 = Q64;
  a.weff = weff;
  a.perm = w.perm;
  a.cnt = w.cnt;
  a.B = w.B;
  a.P = P;
  a.lambda = lambda;
  a.M = M;
  a.s = gp.s;
  a.nb = gp.nb;
  a.groups = gp.groups;
  a.dp = gp.dp;
  a.ptiles = gp.ptiles;
  a.L = gp.L;
  a.RL = gp.RL;
  hipLaunchKernelGGL(grp_block_kernel, dim3(static_cast<unsigned>(gp.groups * gp.ptiles)),
                     dim3(kBlock), 0, st, gr, a);
  const int ncb = static_cast<int>(cdiv(static_cast<int64_t>(gp.RL) * gp.RL, kGt));
  const int64_t nunits = gp.ptiles * kGt * ncb;
  hipLaunchKernelGGL(grp_expand_kernel, dim3(static_cast<unsigned>(cdiv(nunits, 8) * 8)),
                     dim3(kBlock), 0, st, gr, a, nunits, ncb);
}

}  // namespace tk
