// Sketched normal equations of the sampled core update.
//
// Proof of Thm 4.2: the sketched Gram (SK)^T (SK) is a sum of s outer
// products of design rows, and each row of K is formed from factor rows
// (the implicit query structure of Alg. 3), never stored.  With the
// whitened rows q (q_t = (x)_n q^(n)_{i_n}, see tk_leverage.hip) the
// kernels here compute
//   Gram = sum_t weff_t q_t q_t^T        (gram_kernel, MFMA)
//   out  = sum_t c_t q_t                 (rows_t_vec_kernel, FP64)
//   c_t  = a_t - b_t (q_t . h)           (rows_dot_kernel, FP64)
//
// A pre-gather pass writes each sample's factor rows contiguously, transposed
// per chunk of 32 samples, so the hot kernels stream coalesced chunks into a
// padded [row position][sample] LDS layout with shifts only (no division, no
// bank conflicts) and prefetch the next chunk while computing the current.
// Kronecker rows are formed in LDS with one multiply per element: with L the
// last mode of rank >= 2, a design index r splits into an outer index
// o = r / R_L and r % R_L, so y_t[r] = O_t[o] * q^(L)_{i_L}[r % R_L] with
// O_t[o] = sqrt(weff_t) prod_{n != L} q^(n)_{i_n}[digit_n(o)] staged per chunk
// (modes after L have rank 1 and contribute their single entry).
#include <string.h>

#include <mutex>

#include "tk_mfma.h"

namespace tk {
namespace {

// ------------------------------------------------------------------ pre-gather
// Element (t, j) of the chunk-transposed layout: chunk c = t / 32, row
// position j, at c 32 sum_r + 32 j + t % 32.

__global__ __launch_bounds__(kBlock) void pregather_kernel(Geom g, const int32_t* __restrict__ idx,
                                                           const double* __restrict__ weff,
                                                           int64_t s,
                                                           const double* __restrict__ Q64,
                                                           double* __restrict__ rows64,
                                                           float* __restrict__ rows32) {
  // one thread per sample t: its indices and weight are read once, then its
  // concatenated row goes to positions j of chunk t / 32 (consecutive threads
  // write consecutive t of a position: coalesced)
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= row_chunks(s) * kRowChunk) return;
  const int SR = g.sum_r;
  const int64_t base = (t >> 5) * SR * kRowChunk + (t & (kRowChunk - 1));
  float* o32 = rows32 + base;
  double* o64 = rows64 ? rows64 + base : nullptr;
  if (t >= s) {  // padding samples of the last chunk
    for (int j = 0; j < SR; ++j) {
      o32[j * kRowChunk] = 0.0f;
      if (o64) o64[j * kRowChunk] = 0.0;
    }
    return;
  }
  const double sw = sqrt(weff[t]);  // sqrt(w_t) folded into the mode-0 entries of rows32
  for (int n = 0; n < g.order; ++n) {
    int32_t i = idx[static_cast<int64_t>(n) * s + t];
    if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
    const int R = g.ranks[n];
    const double* q = Q64 + g.qoff[n] + static_cast<int64_t>(i) * R;
    const int j0 = g.soff[n];
    for (int r = 0; r < R; ++r) {
      const double v = q[r];
      o32[(j0 + r) * kRowChunk] = static_cast<float>(n == 0 ? v * sw : v);
      if (o64) o64[(j0 + r) * kRowChunk] = v;
    }
  }
}

// Row offsets of the outer factors of outer index o: for every mode n != L,
// the row position soff_n + digit_n(o) (digit 0 for modes after L).
__device__ inline void outer_offsets(const Geom& g, int64_t o, unsigned char* offs) {
  const int L = g.last;
  int k = 0;
  int64_t rem = o;
  unsigned char tmp[kMaxOrder];
  for (int n = L - 1; n >= 0; --n) {
    tmp[n] = static_cast<unsigned char>(g.soff[n] + rem % g.ranks[n]);
    rem /= g.ranks[n];
  }
  for (int n = 0; n < L; ++n) offs[k++] = tmp[n];
  for (int n = L + 1; n < g.order; ++n) offs[k++] = static_cast<unsigned char>(g.soff[n]);
}

// ------------------------------------------------------------------ Gram, FP64 (64 x 64 tiles)
template <class V>
struct GramSmem {
  static constexpr int T = V::TILE, BK = V::BK;
  static constexpr int NO = T / 2 + 1;  // outer indices a tile can touch (R_L >= 2)
  static constexpr int RT = BK + 1;
  typename V::Src rT[kMaxSumR * RT];    // staged rows, [row position][sample]
  typename V::Src sw[BK];
  typename V::Src OA[NO][BK];
  typename V::Src OB[NO][BK];
  unsigned char offs[2][NO][kMaxOrder];
  short rowo[2][T];
  short rowl[2][T];
  alignas(16) typename V::Op YA[T * V::LDK];
  alignas(16) typename V::Op YB[T * V::LDK];
};

template <class V>
__global__ __launch_bounds__(kBlock) void gram_kernel(Geom g,
                                                      const typename V::Src* __restrict__ rows,
                                                      const double* __restrict__ weff,
                                                      int prescaled, int64_t s, int64_t chunk,
                                                      typename V::Out* __restrict__ part) {
  using Src = typename V::Src;
  using Op = typename V::Op;
  using Acc = typename V::Acc;
  constexpr int T = V::TILE, BK = V::BK, LDK = V::LDK, RT = GramSmem<V>::RT;
  constexpr int NO = GramSmem<V>::NO;
  constexpr int PF = (BK * kMaxSumR + kBlock - 1) / kBlock;
  __shared__ GramSmem<V> sm;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = g.order;
  const int RL = g.ranks[g.last];
  const int SR = g.sum_r;
  const int sl = g.soff[g.last];
  const int64_t d = g.d;

  int64_t ti, tj;
  tri_index(blockIdx.x, ti, tj);
  const bool diag = (ti == tj);
  const int64_t r0 = ti * T, c0 = tj * T;
  // split blockIdx.y covers whole chunks [ca, cb)
  const int64_t ca = static_cast<int64_t>(blockIdx.y) * (chunk / BK);
  int64_t cb = ca + chunk / BK;
  if (cb > row_chunks(s)) cb = row_chunks(s);

  int64_t ob[2];
  int no[2];
  for (int side = 0; side < 2; ++side) {
    const int64_t base = side == 0 ? r0 : c0;
    const int64_t last = ((base + T < d) ? base + T : d) - 1;
    ob[side] = base / RL;
    no[side] = static_cast<int>(last / RL - ob[side] + 1);
  }
  for (int e = tid; e < 2 * NO; e += kBlock) {
    const int side = e / NO, oi = e - side * NO;
    outer_offsets(g, ob[side] + oi, sm.offs[side][oi]);
  }
  for (int e = tid; e < 2 * T; e += kBlock) {
    const int side = e / T, i = e - side * T;
    const int64_t r = (side == 0 ? r0 : c0) + i;
    const int64_t rr = r < d ? r : d - 1;
    sm.rowo[side][i] = static_cast<short>(rr / RL - ob[side]);
    sm.rowl[side][i] = static_cast<short>(rr % RL);
  }

  Src pf[PF];
  const int nval = BK * SR;
  auto fetch = [&](int64_t c) {
    const Src* src = rows + c * nval;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kBlock;
      pf[k] = (e < nval) ? src[e] : Src(0);
    }
  };
  auto commit = [&](int64_t c) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kBlock;
      if (e < nval) sm.rT[(e >> 5) * RT + (e & 31)] = pf[k];
    }
    for (int t = tid; t < BK; t += kBlock) {
      const int64_t tt = c * BK + t;
      sm.sw[t] = tt < s ? (prescaled ? Src(1) : static_cast<Src>(sqrt(weff[tt]))) : Src(0);
    }
  };

  constexpr int WT = T / 2, NB = WT / V::MT;
  const int wr = wave >> 1, wc = wave & 1;
  Acc acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < V::NACC; ++v) acc[a][b][v] = 0;

  if (ca < cb) {
    fetch(ca);
    commit(ca);
  }
  __syncthreads();
  for (int64_t c = ca; c < cb; ++c) {
    const bool more = c + 1 < cb;
    if (more) fetch(c + 1);
    {
      const int nsides = diag ? 1 : 2;
      for (int side = 0; side < nsides; ++side) {
        Src(*O)[BK] = side == 0 ? sm.OA : sm.OB;
        for (int e = tid; e < no[side] * BK; e += kBlock) {
          const int oi = e >> 5, t = e & 31;
          Src v = sm.sw[t];
          for (int k = 0; k < N - 1; ++k) v *= sm.rT[sm.offs[side][oi][k] * RT + t];
          O[oi][t] = v;
        }
      }
    }
    __syncthreads();
    {
      const int nsides = diag ? 1 : 2;
      for (int side = 0; side < nsides; ++side) {
        Src(*O)[BK] = side == 0 ? sm.OA : sm.OB;
        Op* Y = side == 0 ? sm.YA : sm.YB;
        const int64_t base = side == 0 ? r0 : c0;
        for (int e = tid; e < T * BK; e += kBlock) {
          const int i = e >> 5, t = e & 31;
          const bool ok = base + i < d;
          Y[i * LDK + t] =
              ok ? V::cvt(O[sm.rowo[side][i]][t] * sm.rT[(sl + sm.rowl[side][i]) * RT + t]) : Op(0);
        }
      }
    }
    __syncthreads();
    const Op* YB = diag ? sm.YA : sm.YB;
#pragma unroll
    for (int kk = 0; kk < BK; kk += V::KT) {
      const int kofs = kk + (lane / V::MT) * V::EPL;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = V::mma(&sm.YA[(wr * WT + a * V::MT + lane % V::MT) * LDK + kofs],
                             &YB[(wc * WT + b * V::MT + lane % V::MT) * LDK + kofs], acc[a][b]);
    }
    if (more) commit(c + 1);
    __syncthreads();
  }

  typename V::Out* out = part + static_cast<int64_t>(blockIdx.y) * d * d;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < V::NACC; ++v) {
        const int64_t r = r0 + wr * WT + a * V::MT + V::acc_row(lane, v);
        const int64_t cc = c0 + wc * WT + b * V::MT + V::acc_col(lane, v);
        if (r < d && cc < d) out[r * d + cc] = static_cast<typename V::Out>(acc[a][b][v]);
      }
}

// ------------------------------------------------------------------ assemble (FP64 splits)
template <class In>
__global__ __launch_bounds__(kBlock) void assemble_kernel(Geom g, const In* __restrict__ part,
                                                          int ksplit, const double* __restrict__ P,
                                                          double lambda, double* __restrict__ M) {
  const int64_t d = g.d;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (e > i) return;  // lower triangle only
  const int64_t j = e;
  double v = 0.0;
  for (int k = 0; k < ksplit; ++k) v += static_cast<double>(part[static_cast<int64_t>(k) * d * d + i * d + j]);
  // lambda prod_n P_n[i_n][j_n] (32-bit digit arithmetic: d < 2^31)
  double p = 1.0;
  uint32_t a = static_cast<uint32_t>(i), b = static_cast<uint32_t>(j);
  for (int n = g.order - 1; n >= 0; --n) {
    const uint32_t R = static_cast<uint32_t>(g.ranks[n]);
    p *= P[g.roff[n] + (a % R) * R + (b % R)];
    a /= R;
    b /= R;
  }
  M[i * d + j] = fma(lambda, p, v);
}

// ------------------------------------------------------------------ gather
template <class T>
__global__ __launch_bounds__(kBlock) void gather_kernel(Geom g, const T* __restrict__ X,
                                                        const uint32_t* __restrict__ mask,
                                                        const int32_t* __restrict__ idx,
                                                        const double* __restrict__ weight,
                                                        int64_t s, double* __restrict__ weff,
                                                        double* __restrict__ xw,
                                                        unsigned int* missing, int32_t* status,
                                                        int ridge_ok) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  bool miss = false, bad = false;
  if (t < s) {
    int64_t flat = 0;
    int nridge = 0;  // modes whose index lies in the ridge range [I_n, I_n + R_n)
    for (int n = 0; n < g.order; ++n) {
      const int32_t i = idx[static_cast<int64_t>(n) * s + t];
      if (ridge_ok && i >= g.dims[n] && i < g.dims[n] + g.ranks[n])
        ++nridge;
      else if (i < 0 || i >= g.dims[n])
        bad = true;
      flat += static_cast<int64_t>(i) * g.strides[n];
    }
    if (nridge != 0 && nridge != g.order) bad = true;  // a ridge draw has all digits in range
    double w = weight[t];
    double x = 0.0;
    if (bad) {
      w = 0.0;
    } else if (nridge) {
      x = 0.0;  // ridge row: response 0, never masked
    } else {
      x = static_cast<double>(X[flat]);
      if (mask && !((mask[flat >> 5] >> (flat & 31)) & 1u)) {
        miss = true;
        w = 0.0;
      }
    }
    weff[t] = w;
    xw[t] = w * x;
  }
  const unsigned long long bm = __ballot(miss);
  if ((threadIdx.x & 63) == 0 && bm) atomicAdd(missing, static_cast<unsigned int>(__popcll(bm)));
  if (bad) atomicMax(status, static_cast<int32_t>(TK_E_ARG));
}

// ------------------------------------------------------------------ rows^T c and rows . h
// FP64, chunk-transposed sample rows.  A workgroup owns RW design rows
// (RW = min(1024, 64 R_L): at most 65 outer indices) and a split of the
// sample chunks; thread tid owns rows r0 + tid + 256 k (k < 4).
constexpr int kVK = kRowChunk;  // samples per stage
constexpr int kVO = 65;         // outer indices per workgroup
constexpr int kVRT = kVK + 1;   // LDS row stride (doubles)
constexpr int kVPF = (kVK * kMaxSumR + kBlock - 1) / kBlock;

// The staged sample rows (sum_r x kVRT doubles) live in dynamic LDS sized by
// the problem's sum_r at launch, so that small rank sums leave room for more
// workgroups per CU.
struct VecSmem {
  double sc[kVK];
  double O[kVO][kVK + 1];  // padded: MFMA fragments read 16 rows at one column
  unsigned char offs[kVO][kMaxOrder];
  double red[4][kVK];
};

struct VecGeo {
  int64_t r0;
  int rw;
  int no;
  int my_o[4], my_l[4];
  bool my_ok[4];
};

__host__ __device__ inline int vec_rows_per_wg(const Geom& g) {
  const int RL = g.ranks[g.last];
  const int rw = 64 * RL;
  return rw < 1024 ? rw : 1024;
}

__device__ inline VecGeo vec_setup(const Geom& g, VecSmem& sm) {
  VecGeo vg;
  const int RL = g.ranks[g.last];
  const int64_t d = g.d;
  const int RW = vec_rows_per_wg(g);
  vg.r0 = static_cast<int64_t>(blockIdx.x) * RW;
  vg.rw = static_cast<int>((d - vg.r0) < RW ? (d - vg.r0) : RW);
  const int64_t obase = vg.r0 / RL;
  vg.no = static_cast<int>((vg.r0 + vg.rw - 1) / RL - obase + 1);
  for (int oi = threadIdx.x; oi < vg.no; oi += kBlock) outer_offsets(g, obase + oi, sm.offs[oi]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
    vg.my_ok[k] = i < vg.rw;
    const int64_t r = vg.r0 + (vg.my_ok[k] ? i : 0);
    vg.my_o[k] = static_cast<int>(r / RL - obase);
    vg.my_l[k] = static_cast<int>(r % RL);
  }
  return vg;
}

// NPF prefetch registers per thread: kVK sum_r <= NPF kBlock
constexpr int kVPFSmall = (kVK * 64 + kBlock - 1) / kBlock;  // sum_r <= 64

template <int NPF>
__device__ inline void vec_fetch(const Geom& g, const double* rows, int64_t c, double* pf) {
  const int nval = kVK * g.sum_r;
  const double* src = rows + c * nval;
#pragma unroll
  for (int k = 0; k < NPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    pf[k] = (e < nval) ? src[e] : 0.0;
  }
}

template <int NPF>
__device__ inline void vec_commit(const Geom& g, VecSmem& sm, double* rT, const double* pf,
                                  const double* coef, int64_t c, int64_t s) {
  const int nval = kVK * g.sum_r;
#pragma unroll
  for (int k = 0; k < NPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    if (e < nval) rT[(e >> 5) * kVRT + (e & 31)] = pf[k];
  }
  for (int t = threadIdx.x; t < kVK; t += kBlock) {
    const int64_t tt = c * kVK + t;
    sm.sc[t] = tt < s ? (coef ? coef[tt] : 1.0) : 0.0;
  }
}

// O[oi][t] = coef_t prod_{n != L} q^(n)[digit]
__device__ inline void vec_outer(const Geom& g, VecSmem& sm, const double* rT, const VecGeo& vg) {
  const int N = g.order;
  for (int e = threadIdx.x; e < vg.no * kVK; e += kBlock) {
    const int oi = e >> 5, t = e & 31;
    double v = sm.sc[t];
    for (int k = 0; k < N - 1; ++k) v *= rT[sm.offs[oi][k] * kVRT + t];
    sm.O[oi][t] = v;
  }
}

// part[split][r] = sum_{t in split} c_t q_t[r], with r = (obase + o) R_L + l:
// the block out[o][l] = sum_t O[o][t] q_L[l][t] is a small FP64 GEMM over the
// samples, run on v_mfma_f64_16x16x4 in 16 x 16 blocks shared by the 4 waves.
__device__ inline double mfma_f64_operand(const double* base, int stride, int row, int nrows,
                                          int col) {
  // row-clamped read, zero outside: the fragment of a partial 16-row block
  const double v = base[(row < nrows ? row : nrows - 1) * stride + col];
  return row < nrows ? v : 0.0;
}

template <int NPF>
__global__ __launch_bounds__(kBlock) void rows_t_vec_kernel(Geom g, const double* __restrict__ rows,
                                                            const double* __restrict__ c,
                                                            int64_t s, int64_t cps,
                                                            double* __restrict__ part,
                                                            const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  extern __shared__ double rT[];  // sum_r x kVRT
  const VecGeo vg = vec_setup(g, sm);
  const int sl = g.soff[g.last];
  const int RL = g.ranks[g.last];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nob = (vg.no + 15) / 16, nlb = (RL + 15) / 16;
  const int nblk = nob * nlb;  // <= 20 blocks of 16 x 16, wave w takes w, w + 4, ...
  const int64_t ca = static_cast<int64_t>(blockIdx.y) * cps;
  int64_t cb = ca + cps;
  if (cb > row_chunks(s)) cb = row_chunks(s);
  doublex4 acc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = doublex4{0, 0, 0, 0};
  double pf[NPF];
  if (ca < cb) {
    vec_fetch<NPF>(g, rows, ca, pf);
    vec_commit<NPF>(g, sm, rT, pf, c, ca, s);
  }
  __syncthreads();
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool more = ch + 1 < cb;
    if (more) vec_fetch<NPF>(g, rows, ch + 1, pf);
    vec_outer(g, sm, rT, vg);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int blk = wave + 4 * q;
      if (blk < nblk) {
        const int ob = blk / nlb, lb = blk % nlb;
#pragma unroll
        for (int kk = 0; kk < kVK; kk += 4) {
          const int t = kk + lane / 16;
          const double av = mfma_f64_operand(&sm.O[0][0], kVK + 1, ob * 16 + lane % 16, vg.no, t);
          const double bv =
              mfma_f64_operand(rT + sl * kVRT, kVRT, lb * 16 + lane % 16, RL, t);
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (more) vec_commit<NPF>(g, sm, rT, pf, c, ch + 1, s);
    __syncthreads();
  }
  // accumulator register v of lane l: o = ob 16 + l / 16 + 4 v, l_ = lb 16 + l % 16
  const int64_t obase = vg.r0 / RL;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int blk = wave + 4 * q;
    if (blk < nblk) {
      const int ob = blk / nlb, lb = blk % nlb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = ob * 16 + lane / 16 + 4 * v, l = lb * 16 + lane % 16;
        const int64_t r = (obase + o) * RL + l;
        if (o < vg.no && l < RL && r >= vg.r0 && r < vg.r0 + vg.rw)
          part[static_cast<int64_t>(blockIdx.y) * g.d + r] = acc[q][v];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void sum_parts_kernel(const double* __restrict__ part,
                                                           int64_t nparts, int64_t n,
                                                           double* __restrict__ out,
                                                           const int32_t* done) {
  if (done && *done) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int64_t k = 0;
  for (; k + 4 <= nparts; k += 4) {  // four independent loads in flight per step
    v0 += part[k * n + i];
    v1 += part[(k + 1) * n + i];
    v2 += part[(k + 2) * n + i];
    v3 += part[(k + 3) * n + i];
  }
  for (; k < nparts; ++k) v0 += part[k * n + i];
  out[i] = (v0 + v1) + (v2 + v3);
}

// part[rchunk][t] = sum_{r in rchunk} h[r] q_t[r] = sum_o O[o][t] U[o][t] with
// U[o][t] = sum_l h[(obase + o) R_L + l] q_L[l][t]: U is a small FP64 GEMM on
// v_mfma_f64_16x16x4 (16 x 16 blocks (o, t) shared by the 4 waves, K = R_L); each
// lane then multiplies its accumulators by O and the partial sums over o are
// reduced across lanes and waves.
template <int NPF>
__global__ __launch_bounds__(kBlock) void rows_dot_kernel(Geom g, const double* __restrict__ rows,
                                                          const double* __restrict__ h,
                                                          int64_t s, int64_t cps,
                                                          double* __restrict__ part,
                                                          const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  extern __shared__ double rT[];  // sum_r x kVRT
  const VecGeo vg = vec_setup(g, sm);
  const int sl = g.soff[g.last];
  const int RL = g.ranks[g.last];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t obase = vg.r0 / RL;
  // h[(obase + o) R_L + l] inside this workgroup's rows, 0 outside (read through L1)
  auto h_at = [&](int o, int l) -> double {
    const int64_t r = (obase + o) * RL + l;
    const bool ok = o < vg.no && l < RL && r >= vg.r0 && r < vg.r0 + vg.rw;
    const double v = h[ok ? r : vg.r0];
    return ok ? v : 0.0;
  };
  const int nob = (vg.no + 15) / 16;
  const int nblk = nob * (kVK / 16);  // (o block, t block) pairs, <= 10
  const int64_t ca = static_cast<int64_t>(blockIdx.y) * cps;
  int64_t cb = ca + cps;
  if (cb > row_chunks(s)) cb = row_chunks(s);
  double pf[NPF];
  if (ca < cb) {
    vec_fetch<NPF>(g, rows, ca, pf);
    vec_commit<NPF>(g, sm, rT, pf, nullptr, ca, s);
  }
  __syncthreads();
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool more = ch + 1 < cb;
    if (more) vec_fetch<NPF>(g, rows, ch + 1, pf);
    vec_outer(g, sm, rT, vg);
    __syncthreads();
    double ct[2] = {0.0, 0.0};  // this lane's partial c for t = tb 16 + lane % 16, tb = 0, 1
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int blk = wave + 4 * q;
      if (blk < nblk) {
        const int ob = blk >> 1, tb = blk & 1;
        doublex4 u = doublex4{0, 0, 0, 0};
        for (int kl = 0; kl < RL; kl += 4) {
          const int l = kl + lane / 16;
          const double av = h_at(ob * 16 + lane % 16, l);
          const double bq = rT[(sl + (l < RL ? l : RL - 1)) * kVRT + tb * 16 + lane % 16];
          const double bv = l < RL ? bq : 0.0;
          u = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, u, 0, 0, 0);
        }
        // register v: o = ob 16 + lane / 16 + 4 v, t = tb 16 + lane % 16
        double p = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = ob * 16 + lane / 16 + 4 * v;
          const int oc = o < vg.no ? o : vg.no - 1;
          const double ov = sm.O[oc][tb * 16 + lane % 16];
          p = fma(o < vg.no ? ov : 0.0, u[v], p);
        }
        ct[tb] += p;
      }
    }
    // sum the four lanes that share t (lane % 16), then the waves through LDS
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      double v = ct[tb];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      ct[tb] = v;
    }
    if (lane < 16) {
      sm.red[wave][lane] = ct[0];
      sm.red[wave][16 + lane] = ct[1];
    }
    __syncthreads();
    if (threadIdx.x < kVK) {
      const int64_t tt = ch * kVK + threadIdx.x;
      if (tt < s)
        part[static_cast<int64_t>(blockIdx.x) * s + tt] =
            sm.red[0][threadIdx.x] + sm.red[1][threadIdx.x] + sm.red[2][threadIdx.x] +
            sm.red[3][threadIdx.x];
    }
    if (more) vec_commit<NPF>(g, sm, rT, pf, nullptr, ch + 1, s);
    __syncthreads();
  }
}

// c_t = a_t - b_t * sum_rc part[rc][t]
__global__ __launch_bounds__(kBlock) void dot_finish_kernel(const double* __restrict__ part,
                                                            int64_t nrc, int64_t s,
                                                            const double* __restrict__ a,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ c,
                                                            const int32_t* done) {
  if (done && *done) return;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= s) return;
  double u = 0.0;
  for (int64_t k = 0; k < nrc; ++k) u += part[k * s + t];
  c[t] = (a ? a[t] : 0.0) - b[t] * u;
}

// ---- small Kronecker dimension: d <= kSmD and sum_r <= kSmSumR.
// part[wg][r] = sum_{t in wg} c_t k_t[r], c_t = a_t - b_t (k_t . h) (the a term
// absent when a is null, the dot when h is null), read straight from the
// sample indices and the whitened factor tables Q64 in one pass.  Per chunk of
// 256 samples: the chunk's indices are staged in LDS, then all threads load
// the chunk's factor rows (sample k, row position j) with several loads in
// flight; one thread per sample forms c_t (k_t . h through the last mode's
// inner products, h in LDS, the other modes' offsets from a per-base table);
// then one thread per Kronecker index r (and sample group when d < 256)
// accumulates c_t prod_n q^(n)_t[r_n].  Groups are added in a fixed order.
constexpr int kSmD = 256, kSmSumR = 20, kSmChunk = 256;

struct SmallLds {  // byte offsets of the dynamic LDS regions
  int rows, coef, hs, red, idx, offb, posq, posr;
  int bytes;
};

__host__ __device__ inline SmallLds small_lds(int sum_r) {
  SmallLds L;
  const int ld = sum_r | 1;
  L.rows = 0;
  L.coef = L.rows + 8 * kSmChunk * ld;
  L.hs = L.coef + 8 * kSmChunk;
  L.red = L.hs + 8 * kSmD;
  L.posq = L.red + 8 * kBlock;                 // int64 per row position: qoff[n] - r... base
  L.idx = L.posq + 8 * kSmSumR;                // int32 [kMaxOrder][kSmChunk]
  L.posr = L.idx + 4 * kMaxOrder * kSmChunk;   // int32 per row position: mode n | R_n << 8 | r << 16
  L.offb = L.posr + 4 * kSmSumR;               // uint8 [kSmD][kMaxOrder]
  L.bytes = L.offb + kSmD * kMaxOrder;
  return L;
}

template <int N>  // tensor order: every loop over modes has a static bound
__global__ __launch_bounds__(kBlock) void resid_small_kernel(
    Geom g, const int32_t* __restrict__ idx, const double* __restrict__ Q64,
    const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ h,
    int64_t s, int64_t cpw, double* __restrict__ part, const int32_t* done) {
  if (done && *done) return;
  extern __shared__ __align__(16) char sm_small[];
  const int d = static_cast<int>(g.d), SR = g.sum_r;
  const int RL = g.ranks[N - 1], sl = g.soff[N - 1];
  const int ld = SR | 1;
  const SmallLds L = small_lds(SR);
  double* rowsL = reinterpret_cast<double*>(sm_small + L.rows);
  double* coefL = reinterpret_cast<double*>(sm_small + L.coef);
  double* hs = reinterpret_cast<double*>(sm_small + L.hs);
  double* red = reinterpret_cast<double*>(sm_small + L.red);
  int64_t* posq = reinterpret_cast<int64_t*>(sm_small + L.posq);
  int32_t* idxL = reinterpret_cast<int32_t*>(sm_small + L.idx);
  int32_t* posr = reinterpret_cast<int32_t*>(sm_small + L.posr);
  uint8_t* offb = reinterpret_cast<uint8_t*>(sm_small + L.offb);
  const int tid = threadIdx.x;
  // ---- per-workgroup tables
  if (h)
    for (int e = tid; e < d; e += kBlock) hs[e] = h[e];
  if (tid < SR) {
    int n = 0;
#pragma unroll
    for (int m = 1; m < N; ++m)
      if (g.soff[m] <= tid) n = m;
    int64_t qo = 0;
    int R = 1, so = 0;
#pragma unroll
    for (int m = 0; m < N; ++m)
      if (m == n) {
        qo = g.qoff[m];
        R = g.ranks[m];
        so = g.soff[m];
      }
    posq[tid] = qo + (tid - so);
    posr[tid] = n | (R << 8);
  }
  const int nb = d / RL;  // bases of the last mode: offsets of modes 0 .. N-2
  for (int base = tid; base < nb; base += kBlock) {
    int q = base;
#pragma unroll
    for (int n = N - 2; n >= 0; --n) {
      const int R = g.ranks[n];
      offb[base * kMaxOrder + n] = static_cast<uint8_t>(g.soff[n] + q % R);
      q /= R;
    }
  }
  // phase-2 role: Kronecker index rr of sample group grp
  const int ngrp = kBlock / d;
  const int rr = tid % d, grp = tid / d;
  int offs[N];
  {
    int q = rr;
#pragma unroll
    for (int n = N - 1; n >= 0; --n) {
      const int R = g.ranks[n];
      offs[n] = g.soff[n] + q % R;
      q /= R;
    }
  }
  double acc = 0.0;
  const int64_t nch = (s + kSmChunk - 1) / kSmChunk;
  const int64_t ca = static_cast<int64_t>(blockIdx.x) * cpw;
  const int64_t cb = ca + cpw < nch ? ca + cpw : nch;
  // this thread's sample of a chunk: indices and coefficients, loaded one chunk ahead
  int32_t iv[N];
  double av = 0.0, bv = 0.0;
  auto fetch = [&](int64_t ch) {
    const int64_t t = ch * kSmChunk + tid;
    const int64_t tc = t < s ? t : s - 1;
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const int32_t i = idx[n * s + tc];  // clamped into range (invalid ones carry weight 0)
      const int32_t imax = static_cast<int32_t>(g.dims[n] - 1);
      iv[n] = i < 0 ? 0 : (i > imax ? imax : i);
    }
    av = a ? a[tc] : 0.0;
    bv = (b && h) ? b[tc] : 0.0;
  };
  fetch(ca);
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool valid = ch * kSmChunk + tid < s;
    __syncthreads();  // the previous chunk's LDS reads are done; tables are ready
#pragma unroll
    for (int n = 0; n < N; ++n) idxL[n * kSmChunk + tid] = iv[n];
    const double a_t = av, b_t = bv;
    __syncthreads();
    if (ch + 1 < cb) fetch(ch + 1);
    // the chunk's factor rows: item e = (sample e / SR, position e % SR), all
    // loads issued together (positions past SR repeat the last one, unstored)
    {
      double v[kSmSumR];
      int dst[kSmSumR];
#pragma unroll
      for (int m = 0; m < kSmSumR; ++m) {
        const int mc = m < SR ? m : SR - 1;
        const int e = tid + kBlock * mc;
        const int k = e / SR, j = e - k * SR;
        const int pr = posr[j];
        v[m] = Q64[posq[j] + static_cast<int64_t>(idxL[(pr & 0xff) * kSmChunk + k]) * (pr >> 8)];
        dst[m] = k * ld + j;
      }
#pragma unroll
      for (int m = 0; m < kSmSumR; ++m)
        if (m < SR) rowsL[dst[m]] = v[m];
    }
    __syncthreads();
    double c = a_t;
    if (h) {
      const double* me = rowsL + tid * ld;
      double u = 0.0;
#pragma unroll 2
      for (int base = 0; base < nb; ++base) {
        double pr = 1.0;
#pragma unroll
        for (int n = 0; n < N - 1; ++n) pr *= me[offb[base * kMaxOrder + n]];
        double in0 = 0.0, in1 = 0.0;
        int k = 0;
        for (; k + 2 <= RL; k += 2) {
          in0 = fma(me[sl + k], hs[base * RL + k], in0);
          in1 = fma(me[sl + k + 1], hs[base * RL + k + 1], in1);
        }
        if (k < RL) in0 = fma(me[sl + k], hs[base * RL + k], in0);
        u = fma(pr, in0 + in1, u);
      }
      c = fma(-b_t, u, c);
    }
    coefL[tid] = valid ? c : 0.0;
    __syncthreads();
    if (grp < ngrp) {
#pragma unroll 4
      for (int k = grp; k < kSmChunk; k += ngrp) {
        const double* row = rowsL + k * ld;
        double v = coefL[k];
#pragma unroll
        for (int n = 0; n < N; ++n) v *= row[offs[n]];
        acc += v;
      }
    }
  }
  __syncthreads();
  red[tid] = acc;
  __syncthreads();
  if (tid < d) {
    double v = 0.0;
    for (int k = 0; k < ngrp; ++k) v += red[k * d + tid];
    part[static_cast<int64_t>(blockIdx.x) * d + tid] = v;
  }
}

// The same partial sums when every rank is at most RM (a power of two) and
// RM^N <= 64, with the Kronecker row kept in registers: in the zero-padded
// index space p = sum_n digit_n RM^(N-1-n), a sample is shared by SPL = RM
// lanes, lane j owning the entries whose mode-0 digit is j,
// i.e. RM^(N-1) static indices p'.  The lanes of a sample load its factor rows
// (zero-padded to RM), form their part of k_t . h (h in LDS) and add it across
// the group by xor shuffles, then accumulate c_t k_t over their entries.  The
// workgroup adds its lanes' accumulators once at the end (xor tree over the
// lanes of equal j, then the waves in order).
template <int N, int RM>
struct PadSpace {
  static constexpr int PD = RM * PadSpace<N - 1, RM>::PD;
};
template <int RM>
struct PadSpace<0, RM> {
  static constexpr int PD = 1;
};

constexpr int kRegThreads = 256;

template <int N, int RM, bool EXACT>  // EXACT: every rank equals RM (no padding)
__global__ __launch_bounds__(kRegThreads) void resid_reg_kernel(
    Geom g, const int32_t* __restrict__ idx, const double* __restrict__ Q64,
    const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ h,
    int64_t s, double* __restrict__ part, const int32_t* done) {
  constexpr int PD = PadSpace<N, RM>::PD;
  constexpr int SPL = RM;              // lanes per sample: one per mode-0 digit
  constexpr int PL = PD / SPL;         // entries per lane
  constexpr int HLD = PL + 1;          // padded stride of lane j's slice of h
  if (done && *done) return;
  __shared__ double hs[SPL * HLD];
  __shared__ double red[kRegThreads / 64][PD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane % SPL;
  int R[N];
  int64_t qo[N];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    R[n] = g.ranks[n];
    qo[n] = g.qoff[n];
  }
  // padded index -> unpadded Kronecker index (or -1 past a mode's rank)
  auto unpad = [&](int p) {
    int q = p, r = 0, mul = 1;
    bool ok = true;
#pragma unroll
    for (int n = N - 1; n >= 0; --n) {
      const int dg = q % RM;
      q /= RM;
      ok = ok && dg < R[n];
      r += dg * mul;
      mul *= R[n];
    }
    return ok ? r : -1;
  };
  for (int p = tid; p < PD; p += kRegThreads) {
    const int r = unpad(p);
    hs[(p / PL) * HLD + p % PL] = (h && r >= 0) ? h[r] : 0.0;
  }
  __syncthreads();
  double acc[PL];
#pragma unroll
  for (int e = 0; e < PL; ++e) acc[e] = 0.0;
  const int64_t slots = static_cast<int64_t>(gridDim.x) * (kRegThreads / SPL);
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * (kRegThreads / SPL) + tid / SPL;
  // software pipeline: indices and coefficients two samples ahead, factor
  // rows one sample ahead (past the end: the last sample, never used)
  struct Ix {
    int32_t i[N];
    double a, b;
  };
  struct Rows {
    double q0;
    double q[N > 1 ? N - 1 : 1][RM];
  };
  int32_t Imax[N];  // indices are clamped into range (invalid ones carry weight 0)
#pragma unroll
  for (int n = 0; n < N; ++n) Imax[n] = static_cast<int32_t>(g.dims[n] - 1);
  auto fetch_ix = [&](int64_t t) {
    Ix x;
    const int64_t tc = t < s ? t : s - 1;
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const int32_t i = idx[n * s + tc];
      x.i[n] = i < 0 ? 0 : (i > Imax[n] ? Imax[n] : i);
    }
    x.a = a ? a[tc] : 0.0;
    x.b = (b && h) ? b[tc] : 0.0;
    return x;
  };
  auto fetch_rows = [&](const Ix& x) {
    Rows w;
    if (EXACT) {
      // rows of RM doubles at RM-aligned offsets: 16-byte loads for RM >= 2
      w.q0 = Q64[qo[0] + static_cast<int64_t>(x.i[0]) * RM + j];
#pragma unroll
      for (int n = 1; n < N; ++n) {
        const double* row = Q64 + qo[n] + static_cast<int64_t>(x.i[n]) * RM;
        if (RM >= 2) {
          typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
          for (int r = 0; r < RM; r += 2) {
            const d2 v = *reinterpret_cast<const d2*>(row + r);
            w.q[n - 1][r] = v.x;
            w.q[n - 1][r + 1] = v.y;
          }
        } else {
          w.q[n - 1][0] = row[0];
        }
      }
      return w;
    }
    {
      const double v = Q64[qo[0] + static_cast<int64_t>(x.i[0]) * R[0] + (j < R[0] ? j : R[0] - 1)];
      w.q0 = j < R[0] ? v : 0.0;
    }
#pragma unroll
    for (int n = 1; n < N; ++n) {
      const double* row = Q64 + qo[n] + static_cast<int64_t>(x.i[n]) * R[n];
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const double v = row[r < R[n] ? r : R[n] - 1];
        w.q[n - 1][r] = r < R[n] ? v : 0.0;
      }
    }
    return w;
  };
  Ix xa = fetch_ix(t0), xb = fetch_ix(t0 + slots);
  Rows wa = fetch_rows(xa);
  for (int64_t t = t0; t < s; t += slots) {
    const Ix xc = fetch_ix(t + 2 * slots);
    const Rows wb = fetch_rows(xb);
    // entry p' of this lane: q0 * prod_{n >= 1} q_n[digit_n(p')]
    auto tail = [&](int pp) {
      double k = 1.0;
      int rest = pp;
#pragma unroll
      for (int n = N - 1; n >= 1; --n) {
        k *= wa.q[n - 1][rest % RM];
        rest /= RM;
      }
      return k;
    };
    double c = xa.a;
    if (h) {
      double u = 0.0;
#pragma unroll
      for (int pp = 0; pp < PL; ++pp) u = fma(tail(pp), hs[j * HLD + pp], u);
      u *= wa.q0;
#pragma unroll
      for (int off = 1; off < SPL; off <<= 1) u += __shfl_xor(u, off, 64);
      c = fma(-xa.b, u, c);
    }
    const double cq = c * wa.q0;
#pragma unroll
    for (int pp = 0; pp < PL; ++pp) acc[pp] = fma(cq, tail(pp), acc[pp]);
    xa = xb;
    xb = xc;
    wa = wb;
  }
  // lanes of equal j, then the waves
#pragma unroll
  for (int pp = 0; pp < PL; ++pp) {
    double v = acc[pp];
#pragma unroll
    for (int off = SPL; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    acc[pp] = v;
  }
  if (lane < SPL) {
#pragma unroll
    for (int pp = 0; pp < PL; ++pp) red[wave][lane * PL + pp] = acc[pp];
  }
  __syncthreads();
  for (int p = tid; p < PD; p += kRegThreads) {
    const int r = unpad(p);
    if (r >= 0) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kRegThreads / 64; ++w) v += red[w][p];
      part[static_cast<int64_t>(blockIdx.x) * g.d + r] = v;
    }
  }
}

// out[i] = sum_k part[k][i] for many parts: 64 outputs per workgroup of 16
// waves, wave w adds a contiguous sixteenth of the parts eight at a time, the
// waves' sums are added in wave order.
constexpr int kSpWaves = 16;

__global__ __launch_bounds__(64 * kSpWaves) void sum_parts_wide_kernel(
    const double* __restrict__ part, int64_t nparts, int64_t n, double* __restrict__ out,
    const int32_t* done) {
  if (done && *done) return;
  __shared__ double red[kSpWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const int64_t ic = i < n ? i : n - 1;
  const int64_t ka = (nparts * wave) / kSpWaves, kb = (nparts * (wave + 1)) / kSpWaves;
  double v = 0.0;
  int64_t k = ka;
  for (; k + 8 <= kb; k += 8) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = part[(k + u) * n + ic];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; k < kb; ++k) v += part[k * n + ic];
  red[wave][lane] = v;
  __syncthreads();
  if (wave == 0 && i < n) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kSpWaves; ++w) sum += red[w][lane];
    out[i] = sum;
  }
}

// ------------------------------------------------------------------ fused residual, larger d
// out_w = sum_t c_t q_t over workgroup w's sample chunks, c_t = a_t - b_t (q_t . h)
// (a null: a_t = 0; h null: c_t = a_t), in one pass over the FP64 sample rows.
// With design index r = o R_L + l, q_t[r] = O_t[o] q^(L)_t[l] and
//   q_t . h = sum_o O_t[o] U[o][t],  U[o][t] = sum_l h[o R_L + l] q^(L)_t[l],
//   sum_t c_t q_t[o R_L + l] = sum_t (c_t O_t[o]) q^(L)_t[l],
// both products of a (16 outer indices) x (samples or last-mode entries) block
// on v_mfma_f64_16x16x4.  Per chunk of 32 samples wave w takes the blocks of
// 16 outer indices w, w + 4, ...: U and its lanes' share of the dot products,
// which are added over the lanes and then the waves in wave order; then c_t
// and the accumulation of Z[o][l] in registers.  h sits in LDS; the outer
// factors O_t[o] are products of staged row entries, formed where used.
constexpr int kRbMaxO = 512;  // outer indices (4 waves x 8 blocks of 16)
constexpr int kRbMaxD = 4096;
constexpr int kRbMaxRL = 32;

// entry m of a packed offset word: the LDS row of outer factor m
__device__ inline int rb_row(uint64_t pk, int m) { return static_cast<int>((pk >> (8 * m)) & 0xff); }

// two workgroups per CU where the registers allow it without spilling
template <int NOBW, int NLB>
__global__ __launch_bounds__(kBlock, NOBW * NLB >= 8 ? 1 : 2) void resid_big_kernel(
    Geom g, const double* __restrict__ rows, const double* __restrict__ a,
    const double* __restrict__ b, const double* __restrict__ h, int64_t s, int64_t cpw,
    double* __restrict__ part, const int32_t* done) {
  if (done && *done) return;
  constexpr int KS = kVK / 4;         // k-steps over the chunk's samples
  constexpr int KL = kRbMaxRL / 4;    // k-steps over the last mode (at most)
  __shared__ __align__(8) unsigned char offs[kRbMaxO][kMaxOrder];
  __shared__ double abs_[2][2][kVK];  // per buffer: a_t, b_t
  __shared__ double red[4][kVK];
  // h (d doubles), then two buffers of staged rows (sum_r x kVRT each): chunk
  // k + 1 is staged while chunk k's second half runs
  extern __shared__ double rb_smem[];
  const int64_t d = g.d;
  double* Hs = rb_smem;
  double* rT0 = rb_smem + d;
  double* rT1 = rT0 + g.sum_r * kVRT;
  const int RL = g.ranks[g.last], sl = g.soff[g.last], nm1 = g.order - 1;
  const int O = static_cast<int>(d / RL);
  const int nob = (O + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nch = row_chunks(s);
  const int64_t ca = static_cast<int64_t>(blockIdx.x) * cpw;
  const int64_t cb = ca + cpw < nch ? ca + cpw : nch;
  for (int o = threadIdx.x; o < O; o += kBlock) {
    unsigned char* po = offs[o];
    outer_offsets(g, o, po);
    for (int m = nm1; m < kMaxOrder; ++m) po[m] = 0;
  }
  if (h)
    for (int64_t i = threadIdx.x; i < d; i += kBlock) Hs[i] = h[i];
  doublex4 Z[NOBW][NLB];
#pragma unroll
  for (int j = 0; j < NOBW; ++j)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb) Z[j][lb] = doublex4{0, 0, 0, 0};
  double pf[kVPFSmall];
  auto commit = [&](int64_t c, int buf) __attribute__((always_inline)) {
    double* rs = buf ? rT1 : rT0;
    const int nval = kVK * g.sum_r;
#pragma unroll
    for (int k = 0; k < kVPFSmall; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < nval) rs[(e >> 5) * kVRT + (e & 31)] = pf[k];
    }
    if (threadIdx.x < kVK) {
      const int64_t tt = c * kVK + threadIdx.x;
      abs_[buf][0][threadIdx.x] = (tt < s && a) ? a[tt] : 0.0;
      abs_[buf][1][threadIdx.x] = (tt < s && b) ? b[tt] : 0.0;
    }
  };
  if (ca < cb) {
    vec_fetch<kVPFSmall>(g, rows, ca, pf);
    commit(ca, 0);
  }
  __syncthreads();
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool more = ch + 1 < cb;
    const int buf = static_cast<int>((ch - ca) & 1);
    const double* rT = buf ? rT1 : rT0;
    const double(*ab)[kVK] = abs_[buf];
    if (more) vec_fetch<kVPFSmall>(g, rows, ch + 1, pf);
    if (h) {
      // q^(L) operands of U, B[l][t] (lane: l = 4 k + lane / 16, t = tb 16 + lane % 16),
      // loaded together (rows clamped into the last mode, zero past R_L)
      double qa[2][KL];
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int k = 0; k < KL; ++k) {
          qa[tb][k] = 0.0;
          if (4 * k < RL) {  // k-steps past R_L are skipped below
            const int l = 4 * k + lane / 16;
            const double v = rT[(sl + (l < RL ? l : RL - 1)) * kVRT + tb * 16 + lane % 16];
            qa[tb][k] = l < RL ? v : 0.0;
          }
        }
      // this lane's share of q_t . h for t = tb 16 + lane % 16
      double pt[2] = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < NOBW; ++j) {
        const int ob = wave + 4 * j;
        if (ob < nob) {
          const int oa = ob * 16 + lane % 16;
          double hv[KL];
#pragma unroll
          for (int k = 0; k < KL; ++k) {
            hv[k] = 0.0;
            if (4 * k < RL) {
              const int l = 4 * k + lane / 16;
              const bool ok = oa < O && l < RL;
              const double v = Hs[ok ? oa * RL + l : 0];
              hv[k] = ok ? v : 0.0;
            }
          }
          // outer factors at the accumulator positions o = ob 16 + lane / 16 + 4 v
          uint64_t pk[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int o = ob * 16 + lane / 16 + 4 * v;
            pk[v] = *reinterpret_cast<const uint64_t*>(offs[o < O ? o : 0]);
          }
#pragma unroll
          for (int tb = 0; tb < 2; ++tb) {
            doublex4 u = doublex4{0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < KL; ++k)
              if (4 * k < RL) u = __builtin_amdgcn_mfma_f64_16x16x4f64(hv[k], qa[tb][k], u, 0, 0, 0);
            const int t = tb * 16 + lane % 16;
            // two modes per pass so that their loads issue together
            double ov[4] = {1.0, 1.0, 1.0, 1.0};
            int m = 0;
            for (; m + 2 <= nm1; m += 2) {
              double f0[4], f1[4];
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                f0[v] = rT[rb_row(pk[v], m) * kVRT + t];
                f1[v] = rT[rb_row(pk[v], m + 1) * kVRT + t];
              }
#pragma unroll
              for (int v = 0; v < 4; ++v) ov[v] = (ov[v] * f0[v]) * f1[v];
            }
            if (m < nm1) {
#pragma unroll
              for (int v = 0; v < 4; ++v) ov[v] *= rT[rb_row(pk[v], m) * kVRT + t];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int o = ob * 16 + lane / 16 + 4 * v;
              pt[tb] = fma(o < O ? ov[v] : 0.0, u[v], pt[tb]);
            }
          }
        }
      }
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        double v = pt[tb];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < 16) red[wave][tb * 16 + lane] = v;
      }
    }
    __syncthreads();
    // this lane's operand samples t = 4 ks + lane / 16: c_t, and q^(L) as
    // B[t][l] (l = lb 16 + lane % 16)
    double cks[KS], qb[NLB][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int t = 4 * ks + lane / 16;
      cks[ks] = h ? ab[0][t] - ab[1][t] * (((red[0][t] + red[1][t]) + red[2][t]) + red[3][t])
                  : ab[0][t];
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb) {
        const int l = lb * 16 + lane % 16;
        const double v = rT[(sl + (l < RL ? l : RL - 1)) * kVRT + t];
        qb[lb][ks] = l < RL ? v : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < NOBW; ++j) {
      const int ob = wave + 4 * j;
      if (ob < nob) {
        const int o = ob * 16 + lane % 16;
        const bool ook = o < O;
        const uint64_t pk = *reinterpret_cast<const uint64_t*>(offs[ook ? o : 0]);
        double ov[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) ov[ks] = 1.0;
        int m = 0;
        for (; m + 2 <= nm1; m += 2) {
          const double* row0 = rT + rb_row(pk, m) * kVRT + lane / 16;
          const double* row1 = rT + rb_row(pk, m + 1) * kVRT + lane / 16;
          double f0[KS], f1[KS];
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            f0[ks] = row0[4 * ks];
            f1[ks] = row1[4 * ks];
          }
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) ov[ks] = (ov[ks] * f0[ks]) * f1[ks];
        }
        if (m < nm1) {
          const double* row = rT + rb_row(pk, m) * kVRT + lane / 16;
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) ov[ks] *= row[4 * ks];
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const double av = ook ? ov[ks] * cks[ks] : 0.0;
#pragma unroll
          for (int lb = 0; lb < NLB; ++lb)
            Z[j][lb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, qb[lb][ks], Z[j][lb], 0, 0, 0);
        }
      }
    }
    if (more) commit(ch + 1, buf ^ 1);  // the other buffer: last read two chunks ago
    __syncthreads();
  }
  // Z register v: o = ob 16 + lane / 16 + 4 v, l = lb 16 + lane % 16
  double* out = part + static_cast<int64_t>(blockIdx.x) * d;
#pragma unroll
  for (int j = 0; j < NOBW; ++j) {
    const int ob = wave + 4 * j;
    if (ob < nob) {
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = ob * 16 + lane / 16 + 4 * v, l = lb * 16 + lane % 16;
          if (o < O && l < RL) out[static_cast<int64_t>(o) * RL + l] = Z[j][lb][v];
        }
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host side
GramPlan plan_gram(const Geom& g, int64_t s, tk_dtype prec, int ksplit_override) {
  GramPlan pl;
  memset(&pl, 0, sizeof(pl));
  pl.prec = prec;
  pl.streamk = prec != TK_F64;
  pl.bk = kRowChunk;
  const int64_t nch = row_chunks(s);
  if (pl.streamk) {
    pl.sk.count = 1;
    pl.sk.p[0] = sk_prob(g, s, nullptr);
    SkConfig cfg = sk_default_config(g.d);
    if (ksplit_override > 0) cfg.wg_per_cu = ksplit_override;
    sk_finalize(pl.sk, prec, cfg);
    pl.tile = cfg.tile;
    pl.ntiles = pl.sk.tiles;
    pl.ksplit = 1;
    pl.chunk = nch * kRowChunk;
    return pl;
  }
  pl.tile = VarF64::TILE;
  const int64_t nt = cdiv(g.d, pl.tile);
  pl.ntiles = nt * (nt + 1) / 2;
  int64_t ks = ksplit_override > 0 ? ksplit_override : cdiv(1024, pl.ntiles);
  const int64_t max_ks = cdiv(nch, 2);
  if (ks > max_ks) ks = max_ks;
  if (ks > 64) ks = 64;
  if (ks < 1) ks = 1;
  while (ks > 1 && ks * g.d * g.d * 8 > (int64_t(4) << 30)) --ks;
  const int64_t cps = cdiv(nch, ks);  // chunks per split
  pl.chunk = cps * kRowChunk;
  pl.ksplit = static_cast<int>(cdiv(nch, cps));
  if (pl.ksplit < 1) pl.ksplit = 1;
  return pl;
}

size_t gram_partial_bytes(const Geom& g, const GramPlan& pl) {
  if (pl.grp.on) return grouped_bytes(pl.grp);
  if (pl.streamk) return ((sk_slot_bytes(pl.sk) + 255) & ~size_t(255)) + sk_index_bytes(pl.sk);
  return static_cast<size_t>(pl.ksplit) * static_cast<size_t>(g.d) * static_cast<size_t>(g.d) * 8;
}

void launch_pregather(const Geom& g, const int32_t* idx, const double* weff, int64_t s,
                      const double* Q64, double* rows64, float* rows32, hipStream_t st) {
  const int64_t n = row_chunks(s) * kRowChunk * g.sum_r;
  if (n <= 0) return;
  hipLaunchKernelGGL(pregather_kernel,
                     dim3(static_cast<unsigned>(cdiv(row_chunks(s) * kRowChunk, kBlock))),
                     dim3(kBlock), 0, st, g, idx, weff, s, Q64, rows64, rows32);
}

void launch_gram(const Geom& g, const GramPlan& pl, const double* rows64, const float* rows32,
                 const double* weff, int64_t s, void* partials, hipStream_t st) {
  if (pl.prec == TK_F64) {
    dim3 grid(static_cast<unsigned>(pl.ntiles), static_cast<unsigned>(pl.ksplit));
    hipLaunchKernelGGL(gram_kernel<VarF64>, grid, dim3(kBlock), 0, st, g, rows64, weff, 0, s,
                       pl.chunk, static_cast<double*>(partials));
    return;
  }
  SkBatch b = pl.sk;
  b.p[0].rows = rows32;
  char* base = static_cast<char*>(partials);
  const size_t off = (sk_slot_bytes(b) + 255) & ~size_t(255);
  launch_gram_sk(b, reinterpret_cast<float*>(base), reinterpret_cast<int64_t*>(base + off), st);
}

void launch_assemble(const Geom& g, const GramPlan& pl, const void* partials, const double* P,
                     double lambda, double* M, hipStream_t st) {
  if (pl.streamk) {
    const char* base = static_cast<const char*>(partials);
    const size_t off = (sk_slot_bytes(pl.sk) + 255) & ~size_t(255);
    launch_assemble_sk(pl.sk, 0, g, reinterpret_cast<const float*>(base),
                       reinterpret_cast<const int64_t*>(base + off), P, lambda, M, st);
    return;
  }
  dim3 grid(static_cast<unsigned>(cdiv(g.d, kBlock)), static_cast<unsigned>(g.d));
  hipLaunchKernelGGL(assemble_kernel<double>, grid, dim3(kBlock), 0, st, g,
                     static_cast<const double*>(partials), pl.ksplit, P, lambda, M);
}

void launch_gather(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                   const int32_t* idx, const double* weight, int64_t s, double* weff, double* xw,
                   unsigned int* missing, int32_t* status, hipStream_t st, int ridge) {
  if (s <= 0) return;
  dim3 grid(static_cast<unsigned>(cdiv(s, kBlock)));
  if (dt == TK_F64)
    hipLaunchKernelGGL(gather_kernel<double>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const double*>(X), mask, idx, weight, s, weff, xw, missing,
                       status, ridge);
  else
    hipLaunchKernelGGL(gather_kernel<float>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const float*>(X), mask, idx, weight, s, weff, xw, missing,
                       status, ridge);
}

namespace {
struct VecPlan {
  int64_t nr;      // row chunks
  int64_t nsplit;  // sample splits
  int64_t cps;     // sample chunks per split
};

VecPlan plan_vec(const Geom& g, int64_t s) {
  VecPlan vp;
  vp.nr = cdiv(g.d, vec_rows_per_wg(g));
  const int64_t nch = row_chunks(s);
  int64_t ns = cdiv(1024, vp.nr);
  const int64_t maxs = cdiv(nch, 4);
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  vp.cps = cdiv(nch, ns);
  vp.nsplit = cdiv(nch, vp.cps);
  return vp;
}

struct SmallPlan {
  int64_t nwg;  // workgroups
  int64_t cpw;  // 256-sample chunks per workgroup
};

SmallPlan plan_small(int64_t s) {
  SmallPlan sp;
  const int64_t nch = cdiv(s, kSmChunk);
  const int64_t want = nch < 1024 ? nch : 1024;
  sp.cpw = cdiv(nch, want < 1 ? 1 : want);
  sp.nwg = cdiv(nch, sp.cpw);
  return sp;
}
// (N, RM) of the register-resident kernel for this geometry, RM = 0 if none
int reg_rm(const Geom& g) {
  int rmax = 1;
  for (int n = 0; n < g.order; ++n) rmax = g.ranks[n] > rmax ? g.ranks[n] : rmax;
  int rm = 1;
  while (rm < rmax) rm *= 2;
  if (rm > 8) return 0;
  int64_t pd = 1;
  for (int n = 0; n < g.order; ++n) pd *= rm;
  return (pd <= 64 && g.order <= 6) ? rm : 0;
}

int64_t reg_grid(int64_t s) {
  // about eight samples per 64-lane slot group at most 1024 workgroups
  const int64_t want = cdiv(s, 512);
  return want < 1 ? 1 : (want > 1024 ? 1024 : want);
}

}  // namespace

namespace {
std::mutex g_query_mu;  // guards every cache below

// Runs one HIP query; on failure clears the error only if none was pending
// before it (an earlier error stays visible to the entry point and the caller).
template <class F>
hipError_t quiet_query(F&& f) {
  const hipError_t prior = hipPeekAtLastError();
  const hipError_t e = f();
  if (e != hipSuccess && prior == hipSuccess) (void)hipGetLastError();
  return e;
}

int current_device() {
  int dev = 0;
  if (quiet_query([&] { return hipGetDevice(&dev); }) != hipSuccess) dev = 0;
  return dev;
}

constexpr int kQueryDevices = 64;
int g_cus[kQueryDevices];

int cu_count_locked(int dev) {
  if (dev >= 0 && dev < kQueryDevices && g_cus[dev] > 0) return g_cus[dev];
  int n = 0;
  if (quiet_query([&] {
        return hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
      }) != hipSuccess ||
      n < 1)
    n = 256;  // MI355X
  if (dev >= 0 && dev < kQueryDevices) g_cus[dev] = n;
  return n;
}

struct GridKey {
  int dev;
  const void* kernel;
  size_t lds;
  int threads;
  int val;
};
GridKey g_grids[128];
int g_ngrids = 0;

struct LdsKey {
  int dev;
  const void* kernel;
  int bytes;
};
LdsKey g_lds[64];
int g_nlds = 0;
}  // namespace

int device_cu_count() {
  std::lock_guard<std::mutex> lock(g_query_mu);
  return cu_count_locked(current_device());
}

int resident_grid(const void* kernel, int threads, size_t dyn_lds) {
  std::lock_guard<std::mutex> lock(g_query_mu);
  const int dev = current_device();
  for (int k = 0; k < g_ngrids; ++k)
    if (g_grids[k].dev == dev && g_grids[k].kernel == kernel && g_grids[k].lds == dyn_lds &&
        g_grids[k].threads == threads)
      return g_grids[k].val;
  int per_cu = 0;
  if (quiet_query([&] {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dyn_lds);
      }) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int v = per_cu * cu_count_locked(dev);
  if (g_ngrids < 128) g_grids[g_ngrids++] = GridKey{dev, kernel, dyn_lds, threads, v};
  return v;
}

void ensure_dyn_lds(const void* kernel, int bytes) {
  std::lock_guard<std::mutex> lock(g_query_mu);
  const int dev = current_device();
  for (int k = 0; k < g_nlds; ++k)
    if (g_lds[k].dev == dev && g_lds[k].kernel == kernel) {
      if (g_lds[k].bytes >= bytes) return;
      if (quiet_query([&] {
            return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
          }) == hipSuccess)
        g_lds[k].bytes = bytes;
      return;
    }
  if (quiet_query([&] {
        return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
      }) == hipSuccess &&
      g_nlds < 64)
    g_lds[g_nlds++] = LdsKey{dev, kernel, bytes};
}

bool resid_small_ok(const Geom& g) { return g.d <= kSmD && g.sum_r <= kSmSumR; }

bool resid_big_ok(const Geom& g) {
  const int RL = g.ranks[g.last];
  return !resid_small_ok(g) && g.d <= kRbMaxD && g.sum_r <= 64 && RL <= kRbMaxRL &&
         g.d / RL <= kRbMaxO;
}

namespace {
struct BigPlan {
  int64_t nwg;  // workgroups
  int64_t cpw;  // sample chunks per workgroup
};

BigPlan plan_big(int64_t s) {
  // about two workgroups per CU; each adds a d-vector of partials
  BigPlan bp;
  const int64_t nch = row_chunks(s);
  const int64_t want = nch < 512 ? nch : 512;
  bp.cpw = cdiv(nch, want < 1 ? 1 : want);
  bp.nwg = cdiv(nch, bp.cpw);
  return bp;
}
}  // namespace

int64_t vec_part_doubles(const Geom& g, int64_t s) {
  const VecPlan vp = plan_vec(g, s);
  int64_t n = vp.nsplit * g.d;
  if (resid_big_ok(g) && plan_big(s).nwg * g.d > n) n = plan_big(s).nwg * g.d;
  if (vp.nr * s > n) n = vp.nr * s;
  if (resid_small_ok(g) && plan_small(s).nwg * g.d > n) n = plan_small(s).nwg * g.d;
  if (resid_small_ok(g) && reg_grid(s) * g.d > n) n = reg_grid(s) * g.d;
  return n;
}

// Returns the grid used (one partial vector per workgroup): at most `grid`,
// and no more workgroups than are resident at once.
template <int N, int RM>
int64_t launch_reg(int64_t grid, hipStream_t st, const Geom& g, const int32_t* idx,
                   const double* Q64, const double* a, const double* b, const double* h,
                   int64_t s, double* part, const int32_t* done) {
  // exact ranks: every mode RM wide and every mode's rows 16-byte aligned
  bool exact = true;
  for (int n = 0; n < N; ++n)
    exact = exact && g.ranks[n] == RM && (RM < 2 || (g.qoff[n] % 2) == 0);
  exact = exact && (reinterpret_cast<uintptr_t>(Q64) % 16) == 0;
  const void* k = exact ? reinterpret_cast<const void*>(&resid_reg_kernel<N, RM, true>)
                        : reinterpret_cast<const void*>(&resid_reg_kernel<N, RM, false>);
  const int64_t res = resident_grid(k, kRegThreads, 0);
  if (grid > res) grid = res;
  const dim3 gd(static_cast<unsigned>(grid));
  if (exact)
    hipLaunchKernelGGL((resid_reg_kernel<N, RM, true>), gd, dim3(kRegThreads), 0, st, g, idx, Q64,
                       a, b, h, s, part, done);
  else
    hipLaunchKernelGGL((resid_reg_kernel<N, RM, false>), gd, dim3(kRegThreads), 0, st, g, idx,
                       Q64, a, b, h, s, part, done);
  return grid;
}

bool try_resid_reg(const Geom& g, const int32_t* idx, const double* Q64, const double* a,
                   const double* b, const double* h, int64_t s, double* part, const int32_t* done,
                   hipStream_t st, int64_t* nparts) {
  const int rm = reg_rm(g);
  if (rm == 0) return false;
  const int64_t gd = reg_grid(s);
  int64_t grid = 0;
  const int key = g.order * 16 + rm;
  switch (key) {
    case 1 * 16 + 1: grid = launch_reg<1, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 1 * 16 + 2: grid = launch_reg<1, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 1 * 16 + 4: grid = launch_reg<1, 4>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 1 * 16 + 8: grid = launch_reg<1, 8>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 2 * 16 + 1: grid = launch_reg<2, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 2 * 16 + 2: grid = launch_reg<2, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 2 * 16 + 4: grid = launch_reg<2, 4>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 2 * 16 + 8: grid = launch_reg<2, 8>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 3 * 16 + 1: grid = launch_reg<3, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 3 * 16 + 2: grid = launch_reg<3, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 3 * 16 + 4: grid = launch_reg<3, 4>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 4 * 16 + 1: grid = launch_reg<4, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 4 * 16 + 2: grid = launch_reg<4, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 5 * 16 + 1: grid = launch_reg<5, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 5 * 16 + 2: grid = launch_reg<5, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 6 * 16 + 1: grid = launch_reg<6, 1>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    case 6 * 16 + 2: grid = launch_reg<6, 2>(gd, st, g, idx, Q64, a, b, h, s, part, done); break;
    default: return false;
  }
  *nparts = grid;
  return true;
}

int64_t launch_resid_small_parts(const Geom& g, const int32_t* idx, const double* Q64,
                                 const double* a, const double* b, const double* h, int64_t s,
                                 double* part, const int32_t* done, hipStream_t st) {
  int64_t np = 0;
  if (try_resid_reg(g, idx, Q64, a, b, h, s, part, done, st, &np)) return np;
  const SmallPlan sp = plan_small(s);
  const size_t lds = static_cast<size_t>(small_lds(g.sum_r).bytes);
  const dim3 grid(static_cast<unsigned>(sp.nwg));
#define TK_RS_CASE(NN)                                                                           \
  case NN:                                                                                       \
    hipLaunchKernelGGL(resid_small_kernel<NN>, grid, dim3(kBlock), lds, st, g, idx, Q64, a, b, h, \
                       s, sp.cpw, part, done);                                                    \
    break;
  switch (g.order) {
    TK_RS_CASE(1)
    TK_RS_CASE(2)
    TK_RS_CASE(3)
    TK_RS_CASE(4)
    TK_RS_CASE(5)
    TK_RS_CASE(6)
    TK_RS_CASE(7)
    TK_RS_CASE(8)
  }
#undef TK_RS_CASE
  return sp.nwg;
}

void launch_resid_small(const Geom& g, const int32_t* idx, const double* Q64, const double* a,
                        const double* b, const double* h, int64_t s, double* part, double* out,
                        const int32_t* done, hipStream_t st) {
  const int64_t nwg = launch_resid_small_parts(g, idx, Q64, a, b, h, s, part, done, st);
  hipLaunchKernelGGL(sum_parts_wide_kernel, dim3(static_cast<unsigned>(cdiv(g.d, 64))),
                     dim3(64 * kSpWaves), 0, st, static_cast<const double*>(part), nwg, g.d, out,
                     done);
}

namespace {
template <int W, int NL>
void resid_big_launch(dim3 grid, size_t lds, hipStream_t st, const Geom& g, const double* rows64,
                      const double* a, const double* b, const double* h, int64_t s, int64_t cpw,
                      double* part, const int32_t* done) {
  if (lds > 64 * 1024)  // dynamic LDS above the default limit (gfx950: 160 KB per CU)
    ensure_dyn_lds(reinterpret_cast<const void*>(&resid_big_kernel<W, NL>), 96 * 1024);
  hipLaunchKernelGGL((resid_big_kernel<W, NL>), grid, dim3(kBlock), lds, st, g, rows64, a, b, h,
                     s, cpw, part, done);
}
}  // namespace

void launch_resid_big(const Geom& g, const double* rows64, const double* a, const double* b,
                      const double* h, int64_t s, double* part, double* out, const int32_t* done,
                      hipStream_t st) {
  const BigPlan bp = plan_big(s);
  const int RL = g.ranks[g.last];
  const int nob = static_cast<int>(cdiv(g.d / RL, 16));
  const int nobw = static_cast<int>(cdiv(nob, 4));
  const int nlb = static_cast<int>(cdiv(RL, 16));
  const size_t lds = sizeof(double) * static_cast<size_t>(g.d + 2 * g.sum_r * kVRT);
  const dim3 grid(static_cast<unsigned>(bp.nwg));
#define TK_RB_CASE(W, NL)                                                             \
  if (nobw <= W && nlb == NL) {                                                       \
    resid_big_launch<W, NL>(grid, lds, st, g, rows64, a, b, h, s, bp.cpw, part, done); \
  } else
  // (eight blocks of 16 outer indices per wave with R_L > 16 would exceed d = 4096)
  TK_RB_CASE(1, 1) TK_RB_CASE(2, 1) TK_RB_CASE(4, 1) TK_RB_CASE(8, 1)
  TK_RB_CASE(1, 2) TK_RB_CASE(2, 2) TK_RB_CASE(4, 2) {}
#undef TK_RB_CASE
  hipLaunchKernelGGL(sum_parts_wide_kernel, dim3(static_cast<unsigned>(cdiv(g.d, 64))),
                     dim3(64 * kSpWaves), 0, st, static_cast<const double*>(part), bp.nwg, g.d,
                     out, done);
}

void launch_rows_t_vec(const Geom& g, const double* rows64, const double* c, int64_t s,
                       double* part, double* out, const int32_t* done, hipStream_t st) {
  const VecPlan vp = plan_vec(g, s);
  const size_t lds = sizeof(double) * static_cast<size_t>(g.sum_r) * kVRT;
  const dim3 grid(static_cast<unsigned>(vp.nr), static_cast<unsigned>(vp.nsplit));
  if (g.sum_r <= 64)
    hipLaunchKernelGGL(rows_t_vec_kernel<kVPFSmall>, grid, dim3(kBlock), lds, st, g, rows64, c, s,
                       vp.cps, part, done);
  else
    hipLaunchKernelGGL(rows_t_vec_kernel<kVPF>, grid, dim3(kBlock), lds, st, g, rows64, c, s,
                       vp.cps, part, done);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, static_cast<const double*>(part), vp.nsplit, g.d, out,
                     done);
}

void launch_residual_coef(const Geom& g, const double* rows64, const double* xw,
                          const double* weff, const double* h, int64_t s, double* part, double* c,
                          const int32_t* done, hipStream_t st) {
  const VecPlan vp = plan_vec(g, s);
  const size_t lds = sizeof(double) * static_cast<size_t>(g.sum_r) * kVRT;
  const dim3 grid(static_cast<unsigned>(vp.nr), static_cast<unsigned>(vp.nsplit));
  if (g.sum_r <= 64)
    hipLaunchKernelGGL(rows_dot_kernel<kVPFSmall>, grid, dim3(kBlock), lds, st, g, rows64, h, s,
                       vp.cps, part, done);
  else
    hipLaunchKernelGGL(rows_dot_kernel<kVPF>, grid, dim3(kBlock), lds, st, g, rows64, h, s,
                       vp.cps, part, done);
  hipLaunchKernelGGL(dot_finish_kernel, dim3(static_cast<unsigned>(cdiv(s, kBlock))), dim3(kBlock),
                     0, st, static_cast<const double*>(part), vp.nr, s, xw, weff, c, done);
}

}  // namespace tk
