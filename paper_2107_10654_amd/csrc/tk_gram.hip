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
#include "tk_internal.h"

namespace tk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;

// ------------------------------------------------------------------ MFMA variants
// Operand fragment of lane l: row (l % MT), k-run starting at (l / MT) * EPL.
// Accumulator element v of lane l maps to (row, col) by acc_row / acc_col.
struct VarF64 {
  using Src = double;
  using Op = double;
  using Acc = doublex4;
  using Out = double;
  static constexpr int MT = 16, KT = 4, EPL = 1, NACC = 4;
  static constexpr int TILE = 64, BK = kRowChunk, LDK = BK + 1;
  __device__ static Acc mma(const Op* a, const Op* b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
  // FP64 16x16x4: accumulator register v of lane l holds row l / 16 + 4 v
  __device__ static int acc_row(int lane, int v) { return lane / 16 + 4 * v; }
  __device__ static int acc_col(int lane, int) { return lane % 16; }
  __device__ static Op cvt(Src x) { return x; }
};

struct VarF32 {
  using Src = float;
  using Op = float;
  using Acc = floatx16;
  using Out = float;
  static constexpr int MT = 32, KT = 2, EPL = 1, NACC = 16;
  static constexpr int TILE = 128, BK = kRowChunk, LDK = BK + 1;
  __device__ static Acc mma(const Op* a, const Op* b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int v) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }
  __device__ static int acc_col(int lane, int) { return lane % 32; }
  __device__ static Op cvt(Src x) { return x; }
};

struct VarBF16 {
  using Src = float;
  using Op = __bf16;
  using Acc = floatx16;
  using Out = float;
  static constexpr int MT = 32, KT = 16, EPL = 8, NACC = 16;
  static constexpr int TILE = 128, BK = kRowChunk, LDK = BK + 8;
  __device__ static Acc mma(const Op* a, const Op* b, Acc c) {
    const bf16x8 va = *reinterpret_cast<const bf16x8*>(a);
    const bf16x8 vb = *reinterpret_cast<const bf16x8*>(b);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(va, vb, c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int v) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }
  __device__ static int acc_col(int lane, int) { return lane % 32; }
  __device__ static Op cvt(Src x) { return static_cast<__bf16>(x); }
};


// lower-triangular tile index -> (ti, tj), ti >= tj
__device__ inline void tri_index(int64_t tau, int64_t& ti, int64_t& tj) {
  int64_t i = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(tau) + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= tau) ++i;
  while (i * (i + 1) / 2 > tau) --i;
  ti = i;
  tj = tau - i * (i + 1) / 2;
}

// ------------------------------------------------------------------ pre-gather
__global__ __launch_bounds__(kBlock) void pregather_kernel(Geom g, const int32_t* __restrict__ idx,
                                                           const double* __restrict__ weff,
                                                           int64_t s,
                                                           const double* __restrict__ Q64,
                                                           double* __restrict__ rows64,
                                                           float* __restrict__ rows32) {
  const int SR = g.sum_r;
  const int64_t total = row_chunks(s) * kRowChunk * SR;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const int tt = static_cast<int>(e & (kRowChunk - 1));
  const int64_t rest = e >> 5;
  const int64_t c = rest / SR;
  const int j = static_cast<int>(rest - c * SR);
  const int64_t t = c * kRowChunk + tt;
  double v = 0.0;
  float v32 = 0.0f;
  if (t < s) {
    int n = 0;
    while (n + 1 < g.order && j >= g.soff[n + 1]) ++n;
    int32_t i = idx[static_cast<int64_t>(n) * s + t];
    if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
    v = Q64[g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n] + (j - g.soff[n])];
    v32 = static_cast<float>(n == 0 ? v * sqrt(weff[t]) : v);
  }
  rows64[e] = v;
  rows32[e] = v32;
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

// ------------------------------------------------------------------ stream-K Gram (FP32 / BF16)
// T x T output tiles (T = 128), 4 waves (2 x 2), each wave (T/2) x (T/2) in MFMA
// 32 x 32 blocks; up to three workgroups share a CU so some form Kronecker rows
// while others run MFMA.  The (tile, chunk of 32 samples) units are laid out
// tile by tile; workgroup w walks units [w U / G, (w + 1) U / G) and writes one
// partial tile per tile it touches into slot w * maxseg + k.  The assembly
// kernel sums the slots of each tile in workgroup order (deterministic).
// LDS (dynamic, sized by sum_r): Y tiles | outer products | offsets | rows.
constexpr int kSkT = 128;
constexpr int kSkThreads = 256;
#ifndef TK_SK_WG_PER_CU
#define TK_SK_WG_PER_CU 3
#endif
constexpr int kSkWgPerCu = TK_SK_WG_PER_CU;
constexpr int kSkNO = kSkT / 2 + 1;  // outer indices per tile (R_L >= 2)
constexpr int kSkRT = kRowChunk + 4; // padded LDS row: conflict-free 32-byte reads

template <class V>
struct SkLayout {
  static constexpr int BK = V::BK;
  static constexpr size_t y_bytes = sizeof(typename V::Op) * kSkT * V::LDK;     // one side
  static constexpr size_t o_bytes = sizeof(typename V::Src) * kSkNO * BK;       // one side
  static constexpr size_t offs_bytes = 2 * kSkNO * kMaxOrder;
  static constexpr size_t fixed = 2 * y_bytes + 2 * o_bytes + offs_bytes;
  // rows: sum_r rows plus one zero row
  __host__ __device__ static size_t bytes(int sum_r) {
    return fixed + sizeof(typename V::Src) * static_cast<size_t>(sum_r + 1) * kSkRT;
  }
};

__host__ __device__ inline int64_t sk_unit_start(const SkPlan& sp, int64_t w) {
  return (w * sp.units) / sp.grid;
}

// PF4: 16-byte prefetch registers per thread; a chunk of rows holds
// kRowChunk * sum_r values, so PF4 * 4 * kSkThreads >= kRowChunk * sum_r.
constexpr int kSkPfSmall = 2;  // sum_r <= 64
constexpr int kSkPfLarge = (kRowChunk * kMaxSumR / 4 + kSkThreads - 1) / kSkThreads;
__host__ __device__ constexpr int sk_pf_slots(int sum_r) {
  return kRowChunk * sum_r <= 4 * kSkThreads * kSkPfSmall ? kSkPfSmall : kSkPfLarge;
}

template <class V, int PF4>
__global__ __launch_bounds__(kSkThreads, kSkWgPerCu) void gram_sk_kernel(
    Geom g, SkPlan sp, const typename V::Src* __restrict__ rows,
    typename V::Out* __restrict__ slots) {
  using Src = typename V::Src;
  using Op = typename V::Op;
  using Acc = typename V::Acc;
  using L = SkLayout<V>;
  constexpr int T = kSkT, BK = V::BK, LDK = V::LDK, RT = kSkRT, NO = kSkNO;
  constexpr int IW = V::EPL == 8 ? 8 : 4;         // samples per formation item
  constexpr int IPR = BK / IW;                    // items per row
  constexpr int ITEMS = T * IPR / kSkThreads;     // items per thread per side
  static_assert(BK == kRowChunk, "chunk size");
  extern __shared__ __align__(16) unsigned char sk_smem[];
  Op* YA = reinterpret_cast<Op*>(sk_smem);
  Op* YBs = reinterpret_cast<Op*>(sk_smem + L::y_bytes);
  Src* OA = reinterpret_cast<Src*>(sk_smem + 2 * L::y_bytes);
  Src* OB = reinterpret_cast<Src*>(sk_smem + 2 * L::y_bytes + L::o_bytes);
  unsigned char* offs = sk_smem + 2 * L::y_bytes + 2 * L::o_bytes;  // [2][NO][kMaxOrder]
  Src* rT = reinterpret_cast<Src*>(sk_smem + L::fixed);             // [sum_r + 1][RT]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = g.order;
  const int RL = g.ranks[g.last];
  const int SR = g.sum_r;
  const int sl = g.soff[g.last];
  const int64_t d = g.d;
  const int64_t w = blockIdx.x;
  const int64_t u0 = sk_unit_start(sp, w), u1 = sk_unit_start(sp, w + 1);
  if (u0 >= u1) return;
  for (int e = tid; e < RT; e += kSkThreads) rT[SR * RT + e] = Src(0);  // zero row

  constexpr int WR = T / 2, WC = T / 2, NBR = WR / V::MT, NBC = WC / V::MT;
  const int wr = wave >> 1, wc = wave & 1;
  Acc acc[NBR][NBC];

  const int nval4 = BK * SR / 4;
  f32x4 pf[PF4];
  auto fetch = [&](int64_t c) {
    const f32x4* src = reinterpret_cast<const f32x4*>(rows + c * BK * SR);
#pragma unroll
    for (int k = 0; k < PF4; ++k) {
      const int e = tid + k * kSkThreads;
      if (e < nval4) pf[k] = src[e];
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int k = 0; k < PF4; ++k) {
      const int e = tid + k * kSkThreads;
      if (e < nval4) {
        const int f = 4 * e;  // element index j * 32 + t
        *reinterpret_cast<f32x4*>(&rT[(f >> 5) * RT + (f & 31)]) = pf[k];
      }
    }
  };

  int64_t u = u0;
  int seg = 0;
  while (u < u1) {
    const int64_t tau = u / sp.nchunks;
    const int64_t c_begin = u - tau * sp.nchunks;
    const int64_t tile_end_unit = (tau + 1) * sp.nchunks;
    const int64_t c_end = (u1 < tile_end_unit ? u1 : tile_end_unit) - tau * sp.nchunks;
    int64_t ti, tj;
    tri_index(tau, ti, tj);
    const bool diag = (ti == tj);
    const int64_t r0 = ti * T, c0 = tj * T;
    int64_t ob[2];
    int no[2];
    for (int side = 0; side < 2; ++side) {
      const int64_t base = side == 0 ? r0 : c0;
      const int64_t last = ((base + T < d) ? base + T : d) - 1;
      ob[side] = base / RL;
      no[side] = static_cast<int>(last / RL - ob[side] + 1);
    }
    // this thread's formation items: LDS offsets into O and rT (zero row when
    // the design row is past d)
    int iofs_o[2][ITEMS], iofs_q[2][ITEMS];
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const int e = tid + k * kSkThreads;
        const int i = e / IPR, tg = (e % IPR) * IW;
        const int64_t r = (side == 0 ? r0 : c0) + i;
        const int64_t rr = r < d ? r : d - 1;
        iofs_o[side][k] = static_cast<int>(rr / RL - ob[side]) * BK + tg;
        iofs_q[side][k] = (r < d ? (sl + static_cast<int>(rr % RL)) : SR) * RT + tg;
      }
    __syncthreads();  // the previous tile's LDS use is complete
#pragma unroll 1
    for (int e = tid; e < 2 * NO; e += kSkThreads) {
      const int side = e / NO, oi = e - side * NO;
      outer_offsets(g, ob[side] + oi, offs + (side * NO + oi) * kMaxOrder);
    }
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
      for (int b = 0; b < NBC; ++b)
#pragma unroll
        for (int v = 0; v < V::NACC; ++v) acc[a][b][v] = 0;

    fetch(c_begin);
    commit();
    __syncthreads();
    for (int64_t c = c_begin; c < c_end; ++c) {
      const bool more = c + 1 < c_end;
      if (more) fetch(c + 1);
      // (b) outer products O[oi][t]
      {
        const int nsides = diag ? 1 : 2;
#pragma unroll 1
        for (int side = 0; side < nsides; ++side) {
          Src* O = side == 0 ? OA : OB;
          const unsigned char* so = offs + side * NO * kMaxOrder;
#pragma unroll 1
          for (int e = tid; e < no[side] * BK; e += kSkThreads) {
            const int oi = e >> 5, t = e & 31;
            const uint64_t pk = *reinterpret_cast<const uint64_t*>(so + oi * kMaxOrder);
            Src v = Src(1);
#pragma unroll
            for (int k = 0; k < kMaxOrder - 1; ++k)
              if (k < N - 1) v *= rT[static_cast<int>((pk >> (8 * k)) & 0xff) * RT + t];
            O[e] = v;
          }
        }
      }
      __syncthreads();
      // (c) Kronecker rows of both tiles
      {
        const int nsides = diag ? 1 : 2;
#pragma unroll 1
        for (int side = 0; side < nsides; ++side) {
          const Src* O = side == 0 ? OA : OB;
          Op* Y = side == 0 ? YA : YBs;
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) {
            const int e = tid + k * kSkThreads;
            const int i = e / IPR, tg = (e % IPR) * IW;
            const f32x4* op = reinterpret_cast<const f32x4*>(O + iofs_o[side][k]);
            const f32x4* qp = reinterpret_cast<const f32x4*>(rT + iofs_q[side][k]);
            if constexpr (V::EPL == 8) {
              const f32x4 o0 = op[0], o1 = op[1], q0 = qp[0], q1 = qp[1];
              bf16x8 v;
              v[0] = V::cvt(o0.x * q0.x);
              v[1] = V::cvt(o0.y * q0.y);
              v[2] = V::cvt(o0.z * q0.z);
              v[3] = V::cvt(o0.w * q0.w);
              v[4] = V::cvt(o1.x * q1.x);
              v[5] = V::cvt(o1.y * q1.y);
              v[6] = V::cvt(o1.z * q1.z);
              v[7] = V::cvt(o1.w * q1.w);
              *reinterpret_cast<bf16x8*>(&Y[i * LDK + tg]) = v;
            } else {
              const f32x4 o = op[0], q = qp[0];
              Op* y = &Y[i * LDK + tg];
              y[0] = V::cvt(o.x * q.x);
              y[1] = V::cvt(o.y * q.y);
              y[2] = V::cvt(o.z * q.z);
              y[3] = V::cvt(o.w * q.w);
            }
          }
        }
      }
      __syncthreads();
      // (d) MFMA; then stage the prefetched chunk
      const Op* YB = diag ? YA : YBs;
#pragma unroll
      for (int kk = 0; kk < BK; kk += V::KT) {
        const int kofs = kk + (lane / V::MT) * V::EPL;
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
          for (int b = 0; b < NBC; ++b)
            acc[a][b] = V::mma(&YA[(wr * WR + a * V::MT + lane % V::MT) * LDK + kofs],
                               &YB[(wc * WC + b * V::MT + lane % V::MT) * LDK + kofs], acc[a][b]);
      }
      if (more) commit();
      __syncthreads();
    }
    typename V::Out* out = slots + (w * sp.maxseg + seg) * static_cast<int64_t>(T * T);
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
      for (int b = 0; b < NBC; ++b)
#pragma unroll
        for (int v = 0; v < V::NACC; ++v) {
          const int r = wr * WR + a * V::MT + V::acc_row(lane, v);
          const int cc = wc * WC + b * V::MT + V::acc_col(lane, v);
          out[r * T + cc] = static_cast<typename V::Out>(acc[a][b][v]);
        }
    ++seg;
    u = tau * sp.nchunks + c_end;
  }
}

// M[i][j] (i >= j) = sum of the tile's slots + lambda prod_n P_n[i_n][j_n]
template <class In>
__global__ __launch_bounds__(kBlock) void assemble_sk_kernel(Geom g, SkPlan sp,
                                                             const In* __restrict__ slots,
                                                             const double* __restrict__ P,
                                                             double lambda,
                                                             double* __restrict__ M) {
  const int64_t d = g.d;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j > i) return;
  const int64_t ti = i / kSkT, tj = j / kSkT;
  const int64_t tau = ti * (ti + 1) / 2 + tj;
  const int64_t ua = tau * sp.nchunks, ub = ua + sp.nchunks;  // the tile's units [ua, ub)
  int64_t w = (ua * sp.grid) / sp.units;
  while (w > 0 && sk_unit_start(sp, w) > ua) --w;
  while (sk_unit_start(sp, w + 1) <= ua) ++w;
  const int64_t off = (i - ti * kSkT) * kSkT + (j - tj * kSkT);
  double v = 0.0;
  for (; w < sp.grid && sk_unit_start(sp, w) < ub; ++w) {
    if (sk_unit_start(sp, w + 1) <= sk_unit_start(sp, w)) continue;  // empty range
    const int64_t first_tile = sk_unit_start(sp, w) / sp.nchunks;
    const int64_t k = tau - first_tile;
    v += static_cast<double>(slots[(w * sp.maxseg + k) * static_cast<int64_t>(kSkT * kSkT) + off]);
  }
  double p = 1.0;
  int64_t a = i, b = j;
  for (int n = g.order - 1; n >= 0; --n) {
    const int R = g.ranks[n];
    p *= P[g.roff[n] + (a % R) * R + (b % R)];
    a /= R;
    b /= R;
  }
  M[i * d + j] = fma(lambda, p, v);
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
  double p = 1.0;
  int64_t a = i, b = j;
  for (int n = g.order - 1; n >= 0; --n) {
    const int R = g.ranks[n];
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
                                                        unsigned int* missing, int32_t* status) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  bool miss = false, bad = false;
  if (t < s) {
    int64_t flat = 0;
    for (int n = 0; n < g.order; ++n) {
      const int32_t i = idx[static_cast<int64_t>(n) * s + t];
      if (i < 0 || i >= g.dims[n]) bad = true;
      flat += static_cast<int64_t>(i) * g.strides[n];
    }
    double w = weight[t];
    double x = 0.0;
    if (bad) {
      w = 0.0;
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

struct VecSmem {
  double rT[kMaxSumR * kVRT];
  double sc[kVK];
  double O[kVO][kVK];
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

__device__ inline void vec_fetch(const Geom& g, const double* rows, int64_t c, double* pf) {
  const int nval = kVK * g.sum_r;
  const double* src = rows + c * nval;
#pragma unroll
  for (int k = 0; k < kVPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    pf[k] = (e < nval) ? src[e] : 0.0;
  }
}

__device__ inline void vec_commit(const Geom& g, VecSmem& sm, const double* pf,
                                  const double* coef, int64_t c, int64_t s) {
  const int nval = kVK * g.sum_r;
#pragma unroll
  for (int k = 0; k < kVPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    if (e < nval) sm.rT[(e >> 5) * kVRT + (e & 31)] = pf[k];
  }
  for (int t = threadIdx.x; t < kVK; t += kBlock) {
    const int64_t tt = c * kVK + t;
    sm.sc[t] = tt < s ? (coef ? coef[tt] : 1.0) : 0.0;
  }
}

// O[oi][t] = coef_t prod_{n != L} q^(n)[digit]
__device__ inline void vec_outer(const Geom& g, VecSmem& sm, const VecGeo& vg) {
  const int N = g.order;
  for (int e = threadIdx.x; e < vg.no * kVK; e += kBlock) {
    const int oi = e >> 5, t = e & 31;
    double v = sm.sc[t];
    for (int k = 0; k < N - 1; ++k) v *= sm.rT[sm.offs[oi][k] * kVRT + t];
    sm.O[oi][t] = v;
  }
}

// part[split][r] = sum_{t in split} c_t q_t[r]
__global__ __launch_bounds__(kBlock) void rows_t_vec_kernel(Geom g, const double* __restrict__ rows,
                                                            const double* __restrict__ c,
                                                            int64_t s, int64_t cps,
                                                            double* __restrict__ part,
                                                            const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const VecGeo vg = vec_setup(g, sm);
  const int sl = g.soff[g.last];
  const int64_t ca = static_cast<int64_t>(blockIdx.y) * cps;
  int64_t cb = ca + cps;
  if (cb > row_chunks(s)) cb = row_chunks(s);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double pf[kVPF];
  if (ca < cb) {
    vec_fetch(g, rows, ca, pf);
    vec_commit(g, sm, pf, c, ca, s);
  }
  __syncthreads();
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool more = ch + 1 < cb;
    if (more) vec_fetch(g, rows, ch + 1, pf);
    vec_outer(g, sm, vg);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!vg.my_ok[k]) continue;
      const double* Ok = sm.O[vg.my_o[k]];
      const double* ql = sm.rT + (sl + vg.my_l[k]) * kVRT;
      double a = acc[k];
#pragma unroll 8
      for (int t = 0; t < kVK; ++t) a = fma(Ok[t], ql[t], a);
      acc[k] = a;
    }
    __syncthreads();
    if (more) vec_commit(g, sm, pf, c, ch + 1, s);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (vg.my_ok[k])
      part[static_cast<int64_t>(blockIdx.y) * g.d + vg.r0 + threadIdx.x + k * kBlock] = acc[k];
}

__global__ __launch_bounds__(kBlock) void sum_parts_kernel(const double* __restrict__ part,
                                                           int64_t nparts, int64_t n,
                                                           double* __restrict__ out,
                                                           const int32_t* done) {
  if (done && *done) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int64_t k = 0; k < nparts; ++k) v += part[k * n + i];
  out[i] = v;
}

// part[rchunk][t] = sum_{r in rchunk} h[r] q_t[r]
__global__ __launch_bounds__(kBlock) void rows_dot_kernel(Geom g, const double* __restrict__ rows,
                                                          const double* __restrict__ h,
                                                          int64_t s, int64_t cps,
                                                          double* __restrict__ part,
                                                          const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const VecGeo vg = vec_setup(g, sm);
  const int sl = g.soff[g.last];
  double hr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) hr[k] = vg.my_ok[k] ? h[vg.r0 + threadIdx.x + k * kBlock] : 0.0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ca = static_cast<int64_t>(blockIdx.y) * cps;
  int64_t cb = ca + cps;
  if (cb > row_chunks(s)) cb = row_chunks(s);
  double pf[kVPF];
  if (ca < cb) {
    vec_fetch(g, rows, ca, pf);
    vec_commit(g, sm, pf, nullptr, ca, s);
  }
  __syncthreads();
  for (int64_t ch = ca; ch < cb; ++ch) {
    const bool more = ch + 1 < cb;
    if (more) vec_fetch(g, rows, ch + 1, pf);
    vec_outer(g, sm, vg);
    __syncthreads();
    double v[kVK];
#pragma unroll
    for (int t = 0; t < kVK; ++t) v[t] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!vg.my_ok[k]) continue;
      const double* Ok = sm.O[vg.my_o[k]];
      const double* ql = sm.rT + (sl + vg.my_l[k]) * kVRT;
#pragma unroll
      for (int t = 0; t < kVK; ++t) v[t] = fma(hr[k] * Ok[t], ql[t], v[t]);
    }
    // butterfly reduction over the wave: after the steps with masks 32..2 lane l
    // holds sample (b5 b4 b3 b2 b1) of its lane index, summed over 32 lanes
#pragma unroll
    for (int wdt = kVK / 2, m = 32; wdt >= 1; wdt >>= 1, m >>= 1) {
      const bool up = (lane & m) != 0;
#pragma unroll
      for (int j = 0; j < wdt; ++j) {
        const double send = up ? v[j] : v[j + wdt];
        const double keep = up ? v[j + wdt] : v[j];
        v[j] = keep + __shfl_xor(send, m, 64);
      }
    }
    v[0] += __shfl_xor(v[0], 1, 64);
    const int tl = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
                   ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
    if ((lane & 1) == 0) sm.red[wave][tl] = v[0];
    __syncthreads();
    if (threadIdx.x < kVK) {
      const int64_t tt = ch * kVK + threadIdx.x;
      if (tt < s)
        part[static_cast<int64_t>(blockIdx.x) * s + tt] =
            sm.red[0][threadIdx.x] + sm.red[1][threadIdx.x] + sm.red[2][threadIdx.x] +
            sm.red[3][threadIdx.x];
    }
    if (more) vec_commit(g, sm, pf, nullptr, ch + 1, s);
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

}  // namespace

// ------------------------------------------------------------------ host side
static int device_cu_count() {
  static int cached = 0;
  if (cached == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        n > 0)
      cached = n;
    else
      cached = 256;  // MI355X
    (void)hipGetLastError();
  }
  return cached;
}

GramPlan plan_gram(const Geom& g, int64_t s, tk_dtype prec, int ksplit_override) {
  GramPlan pl;
  pl.prec = prec;
  pl.streamk = prec != TK_F64;
  pl.bk = kRowChunk;
  const int64_t nch = row_chunks(s);
  if (pl.streamk) {
    pl.tile = kSkT;
    SkPlan& sp = pl.sk;
    sp.nt = cdiv(g.d, kSkT);
    sp.ntiles = sp.nt * (sp.nt + 1) / 2;
    sp.nchunks = nch;
    sp.units = sp.ntiles * sp.nchunks;
    int64_t G = ksplit_override > 0 ? ksplit_override : kSkWgPerCu * device_cu_count();
    if (G > sp.units) G = sp.units;
    if (G < 1) G = 1;
    sp.grid = G;
    sp.maxseg = cdiv(cdiv(sp.units, G), sp.nchunks) + 1;
    pl.ntiles = sp.ntiles;
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
  if (pl.streamk)
    return static_cast<size_t>(pl.sk.grid) * static_cast<size_t>(pl.sk.maxseg) * kSkT * kSkT * 4;
  return static_cast<size_t>(pl.ksplit) * static_cast<size_t>(g.d) * static_cast<size_t>(g.d) * 8;
}

void launch_pregather(const Geom& g, const int32_t* idx, const double* weff, int64_t s,
                      const double* Q64, double* rows64, float* rows32, hipStream_t st) {
  const int64_t n = row_chunks(s) * kRowChunk * g.sum_r;
  if (n <= 0) return;
  hipLaunchKernelGGL(pregather_kernel, dim3(static_cast<unsigned>(cdiv(n, kBlock))), dim3(kBlock),
                     0, st, g, idx, weff, s, Q64, rows64, rows32);
}

void launch_gram(const Geom& g, const GramPlan& pl, const double* rows64, const float* rows32,
                 const double* weff, int64_t s, void* partials, hipStream_t st) {
  if (pl.prec == TK_F64) {
    dim3 grid(static_cast<unsigned>(pl.ntiles), static_cast<unsigned>(pl.ksplit));
    hipLaunchKernelGGL(gram_kernel<VarF64>, grid, dim3(kBlock), 0, st, g, rows64, weff, 0, s,
                       pl.chunk, static_cast<double*>(partials));
  } else {
    const bool small = sk_pf_slots(g.sum_r) == kSkPfSmall;
    const dim3 grid(static_cast<unsigned>(pl.sk.grid)), block(kSkThreads);
    float* out = static_cast<float*>(partials);
    if (pl.prec == TK_F32) {
      const size_t lds = SkLayout<VarF32>::bytes(g.sum_r);
      if (small)
        hipLaunchKernelGGL((gram_sk_kernel<VarF32, kSkPfSmall>), grid, block, lds, st, g, pl.sk,
                           rows32, out);
      else
        hipLaunchKernelGGL((gram_sk_kernel<VarF32, kSkPfLarge>), grid, block, lds, st, g, pl.sk,
                           rows32, out);
    } else {
      const size_t lds = SkLayout<VarBF16>::bytes(g.sum_r);
      if (small)
        hipLaunchKernelGGL((gram_sk_kernel<VarBF16, kSkPfSmall>), grid, block, lds, st, g, pl.sk,
                           rows32, out);
      else
        hipLaunchKernelGGL((gram_sk_kernel<VarBF16, kSkPfLarge>), grid, block, lds, st, g, pl.sk,
                           rows32, out);
    }
  }
}

void launch_assemble(const Geom& g, const GramPlan& pl, const void* partials, const double* P,
                     double lambda, double* M, hipStream_t st) {
  dim3 grid(static_cast<unsigned>(cdiv(g.d, kBlock)), static_cast<unsigned>(g.d));
  if (pl.streamk)
    hipLaunchKernelGGL(assemble_sk_kernel<float>, grid, dim3(kBlock), 0, st, g, pl.sk,
                       static_cast<const float*>(partials), P, lambda, M);
  else
    hipLaunchKernelGGL(assemble_kernel<double>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const double*>(partials), pl.ksplit, P, lambda, M);
}

void launch_gather(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                   const int32_t* idx, const double* weight, int64_t s, double* weff, double* xw,
                   unsigned int* missing, int32_t* status, hipStream_t st) {
  if (s <= 0) return;
  dim3 grid(static_cast<unsigned>(cdiv(s, kBlock)));
  if (dt == TK_F64)
    hipLaunchKernelGGL(gather_kernel<double>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const double*>(X), mask, idx, weight, s, weff, xw, missing,
                       status);
  else
    hipLaunchKernelGGL(gather_kernel<float>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const float*>(X), mask, idx, weight, s, weff, xw, missing,
                       status);
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
}  // namespace

int64_t vec_part_doubles(const Geom& g, int64_t s) {
  const VecPlan vp = plan_vec(g, s);
  const int64_t a = vp.nsplit * g.d, b = vp.nr * s;
  return a > b ? a : b;
}

void launch_rows_t_vec(const Geom& g, const double* rows64, const double* c, int64_t s,
                       double* part, double* out, const int32_t* done, hipStream_t st) {
  const VecPlan vp = plan_vec(g, s);
  hipLaunchKernelGGL(rows_t_vec_kernel,
                     dim3(static_cast<unsigned>(vp.nr), static_cast<unsigned>(vp.nsplit)),
                     dim3(kBlock), 0, st, g, rows64, c, s, vp.cps, part, done);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, static_cast<const double*>(part), vp.nsplit, g.d, out,
                     done);
}

void launch_residual_coef(const Geom& g, const double* rows64, const double* xw,
                          const double* weff, const double* h, int64_t s, double* part, double* c,
                          const int32_t* done, hipStream_t st) {
  const VecPlan vp = plan_vec(g, s);
  hipLaunchKernelGGL(rows_dot_kernel,
                     dim3(static_cast<unsigned>(vp.nr), static_cast<unsigned>(vp.nsplit)),
                     dim3(kBlock), 0, st, g, rows64, h, s, vp.cps, part, done);
  hipLaunchKernelGGL(dot_finish_kernel, dim3(static_cast<unsigned>(cdiv(s, kBlock))), dim3(kBlock),
                     0, st, static_cast<const double*>(part), vp.nr, s, xw, weff, c, done);
}

}  // namespace tk
