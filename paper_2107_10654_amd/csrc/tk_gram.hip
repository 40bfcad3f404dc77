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

struct QPtrs {
  const void* p[kMaxOrder];  // whitened rows per mode (Src precision)
};

// lower-triangular tile index -> (ti, tj), ti >= tj
__device__ inline void tri_index(int64_t tau, int64_t& ti, int64_t& tj) {
  int64_t i = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(tau) + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= tau) ++i;
  while (i * (i + 1) / 2 > tau) --i;
  ti = i;
  tj = tau - i * (i + 1) / 2;
}

template <class V>
struct GramSmem {
  static constexpr int T = V::TILE, BK = V::BK;
  static constexpr int NO = T + 1;  // outer indices a tile can touch (R_N >= 1)
  int sidx[kMaxOrder][BK];
  typename V::Src sw[BK];
  typename V::Src QL[kMaxRank][BK];
  typename V::Src OA[NO][BK];
  typename V::Src OB[NO][BK];
  unsigned char dig[2][NO][kMaxOrder];
  short rowo[2][T];
  short rowl[2][T];
  alignas(16) typename V::Op YA[T * V::LDK];
  alignas(16) typename V::Op YB[T * V::LDK];
};

template <class V>
__global__ __launch_bounds__(kBlock) void gram_kernel(Geom g, QPtrs qp,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ weff, int64_t s,
                                                      int64_t chunk,
                                                      typename V::Out* __restrict__ part) {
  using Src = typename V::Src;
  using Op = typename V::Op;
  using Acc = typename V::Acc;
  constexpr int T = V::TILE, BK = V::BK, LDK = V::LDK;
  __shared__ GramSmem<V> sm;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = g.order;
  const int RL = g.ranks[N - 1];
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

  for (int64_t t0 = sa; t0 < sb; t0 += BK) {
    // (a) per-sample indices and sqrt weights
    for (int e = tid; e < N * BK; e += kBlock) {
      const int n = e / BK, t = e % BK;
      const int64_t tt = t0 + t;
      int32_t i = tt < sb ? idx[static_cast<int64_t>(n) * s + tt] : 0;
      if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
      sm.sidx[n][t] = i;
    }
    for (int t = tid; t < BK; t += kBlock) {
      const int64_t tt = t0 + t;
      sm.sw[t] = tt < sb ? static_cast<Src>(sqrt(weff[tt])) : Src(0);
    }
    __syncthreads();
    // (b) last-mode rows and outer products
    {
      const Src* QLg = static_cast<const Src*>(qp.p[N - 1]);
      for (int e = tid; e < RL * BK; e += kBlock) {
        const int rl = e / BK, t = e % BK;
        sm.QL[rl][t] = QLg[static_cast<int64_t>(sm.sidx[N - 1][t]) * RL + rl];
      }
      const int nsides = diag ? 1 : 2;
      for (int side = 0; side < nsides; ++side) {
        Src(*O)[BK] = side == 0 ? sm.OA : sm.OB;
        for (int e = tid; e < no[side] * BK; e += kBlock) {
          const int oi = e / BK, t = e % BK;
          Src v = sm.sw[t];
          for (int n = 0; n < N - 1; ++n) {
            const Src* Qn = static_cast<const Src*>(qp.p[n]);
            v *= Qn[static_cast<int64_t>(sm.sidx[n][t]) * g.ranks[n] + sm.dig[side][oi][n]];
          }
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
              v[k] = ok ? V::cvt(O[oi][tg + k] * sm.QL[rl][tg + k]) : static_cast<__bf16>(0.0f);
            *reinterpret_cast<bf16x8*>(&Y[i * LDK + tg]) = v;
          }
        } else {
          for (int e = tid; e < T * BK; e += kBlock) {
            const int i = e / BK, t = e % BK;
            const bool ok = base + i < d;
            const int oi = sm.rowo[side][i], rl = sm.rowl[side][i];
            Y[i * LDK + t] = ok ? V::cvt(O[oi][t] * sm.QL[rl][t]) : Op(0);
          }
        }
      }
    }
    __syncthreads();
    // (d) MFMA over the chunk
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
constexpr int kVT = 256;  // design rows per workgroup
constexpr int kVK = 16;   // samples per LDS chunk
constexpr int kVO = kVT + 1;

struct VecSmem {
  int sidx[kMaxOrder][kVK];
  double sc[kVK];
  double QL[kMaxRank][kVK];
  double O[kVO][kVK];
  unsigned char dig[kVO][kMaxOrder];
  double red[4][kVK];
};

__device__ inline void vec_setup(const Geom& g, VecSmem& sm, int64_t r0, int64_t& obase, int& no,
                                 int& my_o, int& my_l, bool& my_ok) {
  const int N = g.order;
  const int RL = g.ranks[N - 1];
  const int64_t d = g.d;
  const int64_t last = ((r0 + kVT < d) ? r0 + kVT : d) - 1;
  obase = r0 / RL;
  no = static_cast<int>(last / RL - obase + 1);
  for (int oi = threadIdx.x; oi < no; oi += kBlock) {
    int64_t o = obase + oi;
    for (int n = N - 2; n >= 0; --n) {
      sm.dig[oi][n] = static_cast<unsigned char>(o % g.ranks[n]);
      o /= g.ranks[n];
    }
  }
  const int64_t r = r0 + threadIdx.x;
  my_ok = r < d;
  const int64_t rr = my_ok ? r : d - 1;
  my_o = static_cast<int>(rr / RL - obase);
  my_l = static_cast<int>(rr % RL);
}

// stage sample chunk: sidx, coefficient, QL, O (O includes the coefficient)
__device__ inline void vec_stage(const Geom& g, VecSmem& sm, const QPtrs& qp,
                                 const int32_t* idx, const double* coef, int64_t s, int64_t t0,
                                 int64_t tend, int no) {
  const int N = g.order;
  const int RL = g.ranks[N - 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < N * kVK; e += kBlock) {
    const int n = e / kVK, t = e % kVK;
    const int64_t tt = t0 + t;
    int32_t i = tt < tend ? idx[static_cast<int64_t>(n) * s + tt] : 0;
    if (i < 0 || i >= g.dims[n]) i = 0;  // flagged by the gather pass (weight 0)
    sm.sidx[n][t] = i;
  }
  for (int t = tid; t < kVK; t += kBlock) {
    const int64_t tt = t0 + t;
    sm.sc[t] = (tt < tend && coef) ? coef[tt] : (tt < tend ? 1.0 : 0.0);
  }
  __syncthreads();
  const double* QLg = static_cast<const double*>(qp.p[N - 1]);
  for (int e = tid; e < RL * kVK; e += kBlock) {
    const int rl = e / kVK, t = e % kVK;
    sm.QL[rl][t] = QLg[static_cast<int64_t>(sm.sidx[N - 1][t]) * RL + rl];
  }
  for (int e = tid; e < no * kVK; e += kBlock) {
    const int oi = e / kVK, t = e % kVK;
    double v = sm.sc[t];
    for (int n = 0; n < N - 1; ++n) {
      const double* Qn = static_cast<const double*>(qp.p[n]);
      v *= Qn[static_cast<int64_t>(sm.sidx[n][t]) * g.ranks[n] + sm.dig[oi][n]];
    }
    sm.O[oi][t] = v;
  }
  __syncthreads();
}

// part[chunk][r] = sum_{t in chunk} c_t q_t[r]
__global__ __launch_bounds__(kBlock) void rows_t_vec_kernel(Geom g, QPtrs qp,
                                                            const int32_t* __restrict__ idx,
                                                            const double* __restrict__ c,
                                                            int64_t s, int64_t chunk,
                                                            double* __restrict__ part,
                                                            const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kVT;
  int64_t obase;
  int no, my_o, my_l;
  bool my_ok;
  vec_setup(g, sm, r0, obase, no, my_o, my_l, my_ok);
  const int64_t sa = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t sb = (sa + chunk < s) ? sa + chunk : s;
  double acc = 0.0;
  for (int64_t t0 = sa; t0 < sb; t0 += kVK) {
    vec_stage(g, sm, qp, idx, c, s, t0, sb, no);
#pragma unroll
    for (int t = 0; t < kVK; ++t) acc = fma(sm.O[my_o][t], sm.QL[my_l][t], acc);
    __syncthreads();
  }
  if (my_ok) part[static_cast<int64_t>(blockIdx.y) * g.d + r0 + threadIdx.x] = acc;
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
__global__ __launch_bounds__(kBlock) void rows_dot_kernel(Geom g, QPtrs qp,
                                                          const int32_t* __restrict__ idx,
                                                          const double* __restrict__ h,
                                                          int64_t s, int64_t chunk,
                                                          double* __restrict__ part,
                                                          const int32_t* done) {
  if (done && *done) return;
  __shared__ VecSmem sm;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kVT;
  int64_t obase;
  int no, my_o, my_l;
  bool my_ok;
  vec_setup(g, sm, r0, obase, no, my_o, my_l, my_ok);
  const double hr = my_ok ? h[r0 + threadIdx.x] : 0.0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t sa = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t sb = (sa + chunk < s) ? sa + chunk : s;
  for (int64_t t0 = sa; t0 < sb; t0 += kVK) {
    vec_stage(g, sm, qp, idx, nullptr, s, t0, sb, no);
#pragma unroll
    for (int t = 0; t < kVK; ++t) {
      double v = hr * sm.O[my_o][t] * sm.QL[my_l][t];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) sm.red[wave][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < kVK) {
      const int64_t tt = t0 + threadIdx.x;
      if (tt < sb) {
        const double v = sm.red[0][threadIdx.x] + sm.red[1][threadIdx.x] +
                         sm.red[2][threadIdx.x] + sm.red[3][threadIdx.x];
        part[static_cast<int64_t>(blockIdx.x) * s + tt] = v;
      }
    }
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

void launch_gram(const Geom& g, const GramPlan& pl, const int32_t* idx, const double* weff,
                 int64_t s, const double* Q64, const float* Q32, void* partials, hipStream_t st) {
  QPtrs qp;
  for (int n = 0; n < kMaxOrder; ++n) {
    if (n < g.order)
      qp.p[n] = pl.prec == TK_F64 ? static_cast<const void*>(Q64 + g.qoff[n])
                                  : static_cast<const void*>(Q32 + g.qoff[n]);
    else
      qp.p[n] = nullptr;
  }
  dim3 grid(static_cast<unsigned>(pl.ntiles), static_cast<unsigned>(pl.ksplit));
  if (pl.prec == TK_F64)
    hipLaunchKernelGGL(gram_kernel<VarF64>, grid, dim3(kBlock), 0, st, g, qp, idx, weff, s,
                       pl.chunk, static_cast<double*>(partials));
  else if (pl.prec == TK_F32)
    hipLaunchKernelGGL(gram_kernel<VarF32>, grid, dim3(kBlock), 0, st, g, qp, idx, weff, s,
                       pl.chunk, static_cast<float*>(partials));
  else
    hipLaunchKernelGGL(gram_kernel<VarBF16>, grid, dim3(kBlock), 0, st, g, qp, idx, weff, s,
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

static QPtrs q64_ptrs(const Geom& g, const double* Q64) {
  QPtrs qp;
  for (int n = 0; n < kMaxOrder; ++n) qp.p[n] = n < g.order ? Q64 + g.qoff[n] : nullptr;
  return qp;
}

int64_t rows_t_vec_chunks(const Geom& g, int64_t s) {
  const int64_t nr = cdiv(g.d, kVT);
  int64_t nc = cdiv(512, nr);
  const int64_t maxc = cdiv(s, kVK * 4);
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  return nc;
}

void launch_rows_t_vec(const Geom& g, const int32_t* idx, const double* c, int64_t s,
                       const double* Q64, double* part, double* out, hipStream_t st) {
  // part: rows_t_vec_chunks(g, s) * d doubles
  const int64_t nr = cdiv(g.d, kVT);
  const int64_t nc = rows_t_vec_chunks(g, s);
  const int64_t chunk = cdiv(cdiv(s, nc), kVK) * kVK;
  const int64_t ncc = cdiv(s, chunk);
  hipLaunchKernelGGL(rows_t_vec_kernel, dim3(static_cast<unsigned>(nr), static_cast<unsigned>(ncc)),
                     dim3(kBlock), 0, st, g, q64_ptrs(g, Q64), idx, c, s, chunk, part,
                     static_cast<const int32_t*>(nullptr));
  hipLaunchKernelGGL(sum_parts_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, part, ncc, g.d, out,
                     static_cast<const int32_t*>(nullptr));
}

// Residual coefficient pass of the refinement: part needs cdiv(d,256)*s doubles.
void launch_residual_coef(const Geom& g, const int32_t* idx, const double* xw, const double* weff,
                          const double* h, int64_t s, const double* Q64, double* part, double* c,
                          const int32_t* done, hipStream_t st) {
  const int64_t nr = cdiv(g.d, kVT);
  int64_t nsc = cdiv(1024, nr);
  const int64_t maxc = cdiv(s, kVK * 4);
  if (nsc > maxc) nsc = maxc;
  if (nsc < 1) nsc = 1;
  const int64_t chunk = cdiv(cdiv(s, nsc), kVK) * kVK;
  const int64_t ncc = cdiv(s, chunk);
  hipLaunchKernelGGL(rows_dot_kernel, dim3(static_cast<unsigned>(nr), static_cast<unsigned>(ncc)),
                     dim3(kBlock), 0, st, g, q64_ptrs(g, Q64), idx, h, s, chunk, part, done);
  hipLaunchKernelGGL(dot_finish_kernel, dim3(static_cast<unsigned>(cdiv(s, kBlock))), dim3(kBlock),
                     0, st, part, nr, s, xw, weff, c, done);
}

// rows^T c with the done flag (refinement)
void launch_rows_t_vec_flag(const Geom& g, const int32_t* idx, const double* c, int64_t s,
                            const double* Q64, double* part, double* out, const int32_t* done,
                            hipStream_t st) {
  const int64_t nr = cdiv(g.d, kVT);
  const int64_t nc = rows_t_vec_chunks(g, s);
  const int64_t chunk = cdiv(cdiv(s, nc), kVK) * kVK;
  const int64_t ncc = cdiv(s, chunk);
  hipLaunchKernelGGL(rows_t_vec_kernel, dim3(static_cast<unsigned>(nr), static_cast<unsigned>(ncc)),
                     dim3(kBlock), 0, st, g, q64_ptrs(g, Q64), idx, c, s, chunk, part, done);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, part, ncc, g.d, out, done);
}

}  // namespace tk
