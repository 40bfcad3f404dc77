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
// A pre-gather pass writes each sample's factor rows contiguously (one
// row of sum_n R_n values per sample), so the hot kernels stream coalesced
// chunks of samples and prefetch the next chunk while computing the current.
// Kronecker rows are formed in LDS with one multiply per element: a design
// index r splits into an outer index o = r / R_N (modes 1..N-1) and the last
// mode's index r % R_N, so y_t[r] = O_t[o] * q^(N)_{i_N}[r % R_N] with
// O_t[o] = sqrt(weff_t) prod_{n<N} q^(n)_{i_n}[digit_n(o)] staged per chunk.
#include "tk_internal.h"

namespace tk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
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
  static constexpr int TILE = 64, BK = 16, LDK = BK + 1;
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
  static constexpr int TILE = 128, BK = 16, LDK = BK + 1;
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
  static constexpr int TILE = 128, BK = 32, LDK = BK + 8;
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
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= s * SR) return;
  const int64_t t = e / SR;
  const int j = static_cast<int>(e - t * SR);
  int n = 0;
  while (n + 1 < g.order && j >= g.soff[n + 1]) ++n;
  int32_t i = idx[static_cast<int64_t>(n) * s + t];
  if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
  const double v = Q64[g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n] + (j - g.soff[n])];
  rows64[e] = v;
  rows32[e] = static_cast<float>(n == 0 ? v * sqrt(weff[t]) : v);
}

// ------------------------------------------------------------------ Gram
template <class V>
struct GramSmem {
  static constexpr int T = V::TILE, BK = V::BK;
  static constexpr int NO = T + 1;  // outer indices a tile can touch (R_N >= 1)
  static constexpr int RS = kMaxSumR + 1;
  typename V::Src rows[BK * RS];    // staged sample rows, row stride sum_r + 1
  typename V::Src sw[BK];
  typename V::Src OA[NO][BK];
  typename V::Src OB[NO][BK];
  unsigned char dig[2][NO][kMaxOrder];
  short rowo[2][T];
  short rowl[2][T];
  alignas(16) typename V::Op YA[T * V::LDK];
  alignas(16) typename V::Op YB[T * V::LDK];
};

// rows: per-sample rows in Src precision; prescaled: mode 0 already carries sqrt(weff)
template <class V>
__global__ __launch_bounds__(kBlock) void gram_kernel(Geom g,
                                                      const typename V::Src* __restrict__ rows,
                                                      const double* __restrict__ weff,
                                                      int prescaled, int64_t s, int64_t chunk,
                                                      typename V::Out* __restrict__ part) {
  using Src = typename V::Src;
  using Op = typename V::Op;
  using Acc = typename V::Acc;
  constexpr int T = V::TILE, BK = V::BK, LDK = V::LDK;
  constexpr int PF = (BK * kMaxSumR + kBlock - 1) / kBlock;  // prefetch registers
  __shared__ GramSmem<V> sm;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = g.order;
  const int RL = g.ranks[N - 1];
  const int SR = g.sum_r;
  const int RS = SR + 1;
  const int sl = g.soff[N - 1];
  const int64_t d = g.d;

  int64_t ti, tj;
  tri_index(blockIdx.x, ti, tj);
  const bool diag = (ti == tj);
  const int64_t r0 = ti * T, c0 = tj * T;
  const int64_t sa = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t sb = (sa + chunk < s) ? sa + chunk : s;

  // outer-index ranges and digits of the two tiles
  int64_t ob[2];
  int no[2];
  for (int side = 0; side < 2; ++side) {
    const int64_t base = side == 0 ? r0 : c0;
    const int64_t last = ((base + T < d) ? base + T : d) - 1;
    ob[side] = base / RL;
    no[side] = static_cast<int>(last / RL - ob[side] + 1);
  }
  for (int e = tid; e < 2 * GramSmem<V>::NO; e += kBlock) {
    const int side = e / GramSmem<V>::NO, oi = e % GramSmem<V>::NO;
    int64_t o = ob[side] + oi;
    for (int n = N - 2; n >= 0; --n) {
      sm.dig[side][oi][n] = static_cast<unsigned char>(o % g.ranks[n]);
      o /= g.ranks[n];
    }
  }
  for (int e = tid; e < 2 * T; e += kBlock) {
    const int side = e / T, i = e % T;
    const int64_t r = (side == 0 ? r0 : c0) + i;
    const int64_t rr = r < d ? r : d - 1;
    sm.rowo[side][i] = static_cast<short>(rr / RL - ob[side]);
    sm.rowl[side][i] = static_cast<short>(rr % RL);
  }

  // chunk loader: BK consecutive sample rows (contiguous in global memory)
  Src pf[PF];
  auto fetch = [&](int64_t t0) {
    const int64_t nvalid = ((sb - t0) < BK ? (sb - t0) : BK) * SR;
    const Src* src = rows + t0 * SR;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kBlock;
      pf[k] = (e < nvalid) ? src[e] : Src(0);
    }
  };
  auto commit = [&](int64_t t0) {
    const int nval = BK * SR;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kBlock;
      if (e < nval) {
        const int t = e / SR, j = e - t * SR;
        sm.rows[t * RS + j] = pf[k];
      }
    }
    for (int t = tid; t < BK; t += kBlock) {
      const int64_t tt = t0 + t;
      sm.sw[t] = tt < sb ? (prescaled ? Src(1) : static_cast<Src>(sqrt(weff[tt]))) : Src(0);
    }
  };

  // wave sub-tile: 2 x 2 waves, each (T/2) x (T/2) = NB x NB MFMA blocks
  constexpr int WT = T / 2, NB = WT / V::MT;
  const int wr = wave >> 1, wc = wave & 1;
  Acc acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < V::NACC; ++v) acc[a][b][v] = 0;

  if (sa < sb) {
    fetch(sa);
    commit(sa);
  }
  __syncthreads();
  for (int64_t t0 = sa; t0 < sb; t0 += BK) {
    const bool more = t0 + BK < sb;
    if (more) fetch(t0 + BK);
    // (b) outer products O[oi][t] (mode 0 carries sqrt(weff) or sw)
    {
      const int nsides = diag ? 1 : 2;
      for (int side = 0; side < nsides; ++side) {
        Src(*O)[BK] = side == 0 ? sm.OA : sm.OB;
        for (int e = tid; e < no[side] * BK; e += kBlock) {
          const int oi = e / BK, t = e % BK;
          Src v = sm.sw[t];  // 1 when mode 0 is prescaled, sqrt(weff_t) otherwise
          for (int n = 0; n < N - 1; ++n) v *= sm.rows[t * RS + g.soff[n] + sm.dig[side][oi][n]];
          O[oi][t] = v;
        }
      }
    }
    __syncthreads();
    // (c) Kronecker rows of both tiles, in operand precision
    {
      const int nsides = diag ? 1 : 2;
      for (int side = 0; side < nsides; ++side) {
        Src(*O)[BK] = side == 0 ? sm.OA : sm.OB;
        Op* Y = side == 0 ? sm.YA : sm.YB;
        const int64_t base = side == 0 ? r0 : c0;
        if constexpr (V::EPL == 8) {
          for (int e = tid; e < T * (BK / 8); e += kBlock) {
            const int i = e / (BK / 8), tg = (e % (BK / 8)) * 8;
            const bool ok = base + i < d;
            const int oi = sm.rowo[side][i], rl = sm.rowl[side][i];
            bf16x8 v;
#pragma unroll
            for (int k = 0; k < 8; ++k)
              v[k] = ok ? V::cvt(O[oi][tg + k] * sm.rows[(tg + k) * RS + sl + rl])
                        : static_cast<__bf16>(0.0f);
            *reinterpret_cast<bf16x8*>(&Y[i * LDK + tg]) = v;
          }
        } else {
          for (int e = tid; e < T * BK; e += kBlock) {
            const int i = e / BK, t = e % BK;
            const bool ok = base + i < d;
            const int oi = sm.rowo[side][i], rl = sm.rowl[side][i];
            Y[i * LDK + t] = ok ? V::cvt(O[oi][t] * sm.rows[t * RS + sl + rl]) : Op(0);
          }
        }
      }
    }
    __syncthreads();
    // (d) MFMA over the chunk; then stage the prefetched chunk
    const Op* YB = diag ? sm.YA : sm.YB;
#pragma unroll
    for (int kk = 0; kk < BK; kk += V::KT) {
      const int kofs = kk + (lane / V::MT) * V::EPL;
      const Op* af[NB];
      const Op* bfr[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a)
        af[a] = &sm.YA[(wr * WT + a * V::MT + lane % V::MT) * LDK + kofs];
#pragma unroll
      for (int b = 0; b < NB; ++b)
        bfr[b] = &YB[(wc * WT + b * V::MT + lane % V::MT) * LDK + kofs];
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = V::mma(af[a], bfr[b], acc[a][b]);
    }
    if (more) commit(t0 + BK);
    __syncthreads();
  }

  // store the tile of this split
  typename V::Out* out = part + static_cast<int64_t>(blockIdx.y) * d * d;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < V::NACC; ++v) {
        const int64_t r = r0 + wr * WT + a * V::MT + V::acc_row(lane, v);
        const int64_t c = c0 + wc * WT + b * V::MT + V::acc_col(lane, v);
        if (r < d && c < d) out[r * d + c] = static_cast<typename V::Out>(acc[a][b][v]);
      }
}

// ------------------------------------------------------------------ assemble
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
  // lambda * prod_n P_n[i_n][j_n]
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
// FP64, contiguous sample rows.  A workgroup owns RW design rows (RW = min(1024,
// 64 R_N), so at most 65 outer indices) and a split of the samples; thread
// tid owns rows r0 + tid + 256 k (k < 4).
constexpr int kVK = 32;      // samples per stage
constexpr int kVO = 65;      // outer indices per workgroup
constexpr int kVPF = (kVK * kMaxSumR + kBlock - 1) / kBlock;

struct VecSmem {
  double rows[kVK * (kMaxSumR + 1)];
  double sc[kVK];
  double O[kVO][kVK];
  unsigned char dig[kVO][kMaxOrder];
  double red[4][kVK];
};

struct VecGeo {
  int64_t r0;
  int rw;          // rows of this workgroup
  int64_t obase;
  int no;
  int my_o[4], my_l[4];
  bool my_ok[4];
};

__host__ __device__ inline int vec_rows_per_wg(const Geom& g) {
  const int RL = g.ranks[g.order - 1];
  const int rw = 64 * RL;
  return rw < 1024 ? rw : 1024;
}

__device__ inline VecGeo vec_setup(const Geom& g, VecSmem& sm) {
  VecGeo vg;
  const int N = g.order;
  const int RL = g.ranks[N - 1];
  const int64_t d = g.d;
  const int RW = vec_rows_per_wg(g);
  vg.r0 = static_cast<int64_t>(blockIdx.x) * RW;
  vg.rw = static_cast<int>((d - vg.r0) < RW ? (d - vg.r0) : RW);
  vg.obase = vg.r0 / RL;
  vg.no = static_cast<int>((vg.r0 + vg.rw - 1) / RL - vg.obase + 1);
  for (int oi = threadIdx.x; oi < vg.no; oi += kBlock) {
    int64_t o = vg.obase + oi;
    for (int n = N - 2; n >= 0; --n) {
      sm.dig[oi][n] = static_cast<unsigned char>(o % g.ranks[n]);
      o /= g.ranks[n];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
    vg.my_ok[k] = i < vg.rw;
    const int64_t r = vg.r0 + (vg.my_ok[k] ? i : 0);
    vg.my_o[k] = static_cast<int>(r / RL - vg.obase);
    vg.my_l[k] = static_cast<int>(r % RL);
  }
  return vg;
}

// stage samples [t0, t0 + kVK) of [.., tend): rows and coefficients into LDS
__device__ inline void vec_fetch(const Geom& g, const double* rows, int64_t t0, int64_t tend,
                                 double* pf) {
  const int SR = g.sum_r;
  const int64_t nvalid = ((tend - t0) < kVK ? (tend - t0) : kVK) * SR;
  const double* src = rows + t0 * SR;
#pragma unroll
  for (int k = 0; k < kVPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    pf[k] = (e < nvalid) ? src[e] : 0.0;
  }
}

__device__ inline void vec_commit(const Geom& g, VecSmem& sm, const double* pf,
                                  const double* coef, int64_t t0, int64_t tend) {
  const int SR = g.sum_r, RS = SR + 1;
  const int nval = kVK * SR;
#pragma unroll
  for (int k = 0; k < kVPF; ++k) {
    const int e = threadIdx.x + k * kBlock;
    if (e < nval) {
      const int t = e / SR, j = e - t * SR;
      sm.rows[t * RS + j] = pf[k];
    }
  }
  for (int t = threadIdx.x; t < kVK; t += kBlock) {
    const int64_t tt = t0 + t;
    sm.sc[t] = tt < tend ? (coef ? coef[tt] : 1.0) : 0.0;
  }
}

// O[oi][t] = coef_t prod_{n < N-1} rows[t][soff_n + digit_n(o)]
__device__ inline void vec_outer(const Geom& g, VecSmem& sm, const VecGeo& vg) {
  const int N = g.order, RS = g.sum_r + 1;
  for (int e = threadIdx.x; e < vg.no * kVK; e += kBlock) {
    const int oi = e / kVK, t = e % kVK;
    double v = sm.sc[t];
    for (int n = 0; n < N - 1; ++n) v *= sm.rows[t * RS + g.soff[n] + sm.dig[oi][n]];
    sm.O[oi][t] = v;
  }
}

// part[split][r] = sum_{t in split} c_t q_t[r]
__global__ __launch_bounds__(kBlock) void rows_t_vec_kernel(Geom g, const double* __restrict__ rows,
                                                            const double* __restrict__ c,
                                                            int64_t s, int64_t chunk,
                                                            double* __restrict__ part,
                                                            const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const VecGeo vg = vec_setup(g, sm);
  const int RS = g.sum_r + 1, sl = g.soff[g.order - 1];
  const int64_t sa = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t sb = (sa + chunk < s) ? sa + chunk : s;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double pf[kVPF];
  if (sa < sb) {
    vec_fetch(g, rows, sa, sb, pf);
    vec_commit(g, sm, pf, c, sa, sb);
  }
  __syncthreads();
  for (int64_t t0 = sa; t0 < sb; t0 += kVK) {
    const bool more = t0 + kVK < sb;
    if (more) vec_fetch(g, rows, t0 + kVK, sb, pf);
    vec_outer(g, sm, vg);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!vg.my_ok[k]) continue;
      const double* Ok = sm.O[vg.my_o[k]];
      const double* ql = sm.rows + sl + vg.my_l[k];
      double a = acc[k];
#pragma unroll 8
      for (int t = 0; t < kVK; ++t) a = fma(Ok[t], ql[t * RS], a);
      acc[k] = a;
    }
    __syncthreads();
    if (more) vec_commit(g, sm, pf, c, t0 + kVK, sb);
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
                                                          int64_t s, int64_t chunk,
                                                          double* __restrict__ part,
                                                          const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const VecGeo vg = vec_setup(g, sm);
  const int RS = g.sum_r + 1, sl = g.soff[g.order - 1];
  double hr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) hr[k] = vg.my_ok[k] ? h[vg.r0 + threadIdx.x + k * kBlock] : 0.0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t sa = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t sb = (sa + chunk < s) ? sa + chunk : s;
  double pf[kVPF];
  if (sa < sb) {
    vec_fetch(g, rows, sa, sb, pf);
    vec_commit(g, sm, pf, nullptr, sa, sb);
  }
  __syncthreads();
  for (int64_t t0 = sa; t0 < sb; t0 += kVK) {
    const bool more = t0 + kVK < sb;
    if (more) vec_fetch(g, rows, t0 + kVK, sb, pf);
    vec_outer(g, sm, vg);
    __syncthreads();
    double v[kVK];
#pragma unroll
    for (int t = 0; t < kVK; ++t) v[t] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!vg.my_ok[k]) continue;
      const double* Ok = sm.O[vg.my_o[k]];
      const double* ql = sm.rows + sl + vg.my_l[k];
#pragma unroll
      for (int t = 0; t < kVK; ++t) v[t] = fma(hr[k] * Ok[t], ql[t * RS], v[t]);
    }
    // butterfly reduction over the wave: after the steps with masks 32..2 lane l
    // holds sample (b5 b4 b3 b2 b1) of its lane index, summed over 32 lanes
#pragma unroll
    for (int w = kVK / 2, m = 32; w >= 1; w >>= 1, m >>= 1) {
      const bool up = (lane & m) != 0;
#pragma unroll
      for (int j = 0; j < w; ++j) {
        const double send = up ? v[j] : v[j + w];
        const double keep = up ? v[j + w] : v[j];
        v[j] = keep + __shfl_xor(send, m, 64);
      }
    }
    v[0] += __shfl_xor(v[0], 1, 64);
    const int tl = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
                   ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
    if ((lane & 1) == 0) sm.red[wave][tl] = v[0];
    __syncthreads();
    if (threadIdx.x < kVK) {
      const int64_t tt = t0 + threadIdx.x;
      if (tt < sb)
        part[static_cast<int64_t>(blockIdx.x) * s + tt] =
            sm.red[0][threadIdx.x] + sm.red[1][threadIdx.x] + sm.red[2][threadIdx.x] +
            sm.red[3][threadIdx.x];
    }
    if (more) vec_commit(g, sm, pf, nullptr, t0 + kVK, sb);
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
  c[t] = a[t] - b[t] * u;
}

}  // namespace

// ------------------------------------------------------------------ host side
GramPlan plan_gram(const Geom& g, int64_t s, tk_dtype prec, int ksplit_override) {
  GramPlan pl;
  pl.prec = prec;
  if (prec == TK_F64) {
    pl.tile = VarF64::TILE;
    pl.bk = VarF64::BK;
  } else if (prec == TK_F32) {
    pl.tile = VarF32::TILE;
    pl.bk = VarF32::BK;
  } else {
    pl.tile = VarBF16::TILE;
    pl.bk = VarBF16::BK;
  }
  const int64_t nt = cdiv(g.d, pl.tile);
  pl.ntiles = nt * (nt + 1) / 2;
  int64_t ks = ksplit_override > 0 ? ksplit_override : cdiv(1024, pl.ntiles);
  const int64_t max_ks = cdiv(s, 4 * pl.bk);
  if (ks > max_ks) ks = max_ks;
  if (ks > 64) ks = 64;
  if (ks < 1) ks = 1;
  // keep partial Grams within 4 GiB
  const int64_t elt = prec == TK_F64 ? 8 : 4;
  while (ks > 1 && ks * g.d * g.d * elt > (int64_t(4) << 30)) --ks;
  pl.chunk = cdiv(cdiv(s, ks), pl.bk) * pl.bk;
  pl.ksplit = static_cast<int>(cdiv(s, pl.chunk));
  if (pl.ksplit < 1) pl.ksplit = 1;
  return pl;
}

size_t gram_partial_bytes(const Geom& g, const GramPlan& pl) {
  const size_t elt = pl.prec == TK_F64 ? 8 : 4;
  return static_cast<size_t>(pl.ksplit) * static_cast<size_t>(g.d) * static_cast<size_t>(g.d) * elt;
}

void launch_pregather(const Geom& g, const int32_t* idx, const double* weff, int64_t s,
                      const double* Q64, double* rows64, float* rows32, hipStream_t st) {
  const int64_t n = s * g.sum_r;
  if (n <= 0) return;
  hipLaunchKernelGGL(pregather_kernel, dim3(static_cast<unsigned>(cdiv(n, kBlock))), dim3(kBlock),
                     0, st, g, idx, weff, s, Q64, rows64, rows32);
}

void launch_gram(const Geom& g, const GramPlan& pl, const double* rows64, const float* rows32,
                 const double* weff, int64_t s, void* partials, hipStream_t st) {
  dim3 grid(static_cast<unsigned>(pl.ntiles), static_cast<unsigned>(pl.ksplit));
  if (pl.prec == TK_F64)
    hipLaunchKernelGGL(gram_kernel<VarF64>, grid, dim3(kBlock), 0, st, g, rows64, weff, 0, s,
                       pl.chunk, static_cast<double*>(partials));
  else if (pl.prec == TK_F32)
    hipLaunchKernelGGL(gram_kernel<VarF32>, grid, dim3(kBlock), 0, st, g, rows32, weff, 1, s,
                       pl.chunk, static_cast<float*>(partials));
  else
    hipLaunchKernelGGL(gram_kernel<VarBF16>, grid, dim3(kBlock), 0, st, g, rows32, weff, 1, s,
                       pl.chunk, static_cast<float*>(partials));
}

void launch_assemble(const Geom& g, const GramPlan& pl, const void* partials, const double* P,
                     double lambda, double* M, hipStream_t st) {
  dim3 grid(static_cast<unsigned>(cdiv(g.d, kBlock)), static_cast<unsigned>(g.d));
  if (pl.prec == TK_F64)
    hipLaunchKernelGGL(assemble_kernel<double>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const double*>(partials), pl.ksplit, P, lambda, M);
  else
    hipLaunchKernelGGL(assemble_kernel<float>, grid, dim3(kBlock), 0, st, g,
                       static_cast<const float*>(partials), pl.ksplit, P, lambda, M);
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
  int64_t chunk;   // samples per split
};

VecPlan plan_vec(const Geom& g, int64_t s) {
  VecPlan vp;
  vp.nr = cdiv(g.d, vec_rows_per_wg(g));
  int64_t ns = cdiv(1024, vp.nr);
  const int64_t maxs = cdiv(s, kVK * 4);
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  vp.chunk = cdiv(cdiv(s, ns), kVK) * kVK;
  vp.nsplit = cdiv(s, vp.chunk);
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
                     dim3(kBlock), 0, st, g, rows64, c, s, vp.chunk, part, done);
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
                     dim3(kBlock), 0, st, g, rows64, h, s, vp.chunk, part, done);
  hipLaunchKernelGGL(dot_finish_kernel, dim3(static_cast<unsigned>(cdiv(s, kBlock))), dim3(kBlock),
                     0, st, static_cast<const double*>(part), vp.nr, s, xw, weff, c, done);
}

}  // namespace tk
