// Product-distribution sampling of multi-indices (Alg. 3 sampler; Lemma 4.1:
// the leverage scores of K = A(1) (x) ... (x) A(N) are products of the
// factor scores, so each mode is drawn independently; proof of Thm 4.2: one
// binary search per mode over the mode's CDF).
//
// Random words come from Philox4x64-10 (Salmon et al., SC'11), a
// counter-based generator: sample t needs no state shared with other
// threads, and the draw is reproducible from (seed, counter, problem, t).
// Key = (seed, 0); counter = (t, counter, problem, b); output word j of block
// b drives mode 4b + j.  The uniform u = floor(r W_n / 2^64) lies in
// [0, W_n) and the row is the first j with cdf_j > u.
//
// Augmented draws (Alg. 1 taken literally: the augmented distribution of
// Sec. 3 over the rows of [K; sqrt(lambda) I]) add one branch coin per
// sample from block kAugBlock: with integer branch weights D = 2^Q (data rows,
// normalised mass d) and C = ceil(c 2^Q) (ridge rows, mass d c), word 0 gives
// u = floor(r (D + C) / 2^64) and u >= D selects ridge row
// k = floor(r' d / 2^64) (word 1), stored as idx[n] = I_n + k_n with k_n the
// row-major digits of k over the ranks.
#include "tk_internal.h"

namespace tk {
namespace {

__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]);
    const uint64_t lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// With STAGE the concatenated tables are first copied to LDS (they are read
// by every sample's binary searches); the grid strides over the samples.
constexpr int64_t kSampleLdsRows = 6144;  // 48 KB of uint64 entries
constexpr uint64_t kAugBlock = 2;          // Philox block of the branch draws (modes use 0, 1)

// aug: 0 plain product draws; 1 augmented draws with ridge branch weight coin_c
// against the data branch's coin_d = 2^Q
template <bool STAGE>
__global__ __launch_bounds__(kBlock) void sample_kernel(Geom g, const uint64_t* __restrict__ cdf,
                                                        int64_t s, uint64_t seed,
                                                        uint64_t counter, uint64_t problem,
                                                        int aug, uint64_t coin_c, uint64_t coin_d,
                                                        int32_t* __restrict__ idx,
                                                        double* __restrict__ weight) {
  extern __shared__ uint64_t cs[];
  if (STAGE) {
    const int64_t n = g.total_rows;
    for (int64_t e0 = threadIdx.x; e0 < n; e0 += 8 * kBlock) {
      uint64_t v[8];  // eight loads in flight (indices clamped into range)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int64_t e = e0 + k * kBlock;
        v[k] = cdf[e < n ? e : n - 1];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (e0 + k * kBlock < n) cs[e0 + k * kBlock] = v[k];
    }
    __syncthreads();
  }
  auto tab = [&](int64_t i) -> uint64_t { return STAGE ? cs[i] : cdf[i]; };
  const int N = g.order;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < s;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    double acc = 1.0;
    for (int b = 0; b * 4 < N; ++b) {
      uint64_t c[4] = {static_cast<uint64_t>(t), counter, problem, static_cast<uint64_t>(b)};
      philox4x64_10(c, seed, 0ull);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 4 * b + j;
        if (n < N) {
          const int64_t o = g.off[n];
          const int64_t I = g.dims[n];
          const uint64_t W = tab(o + I - 1);
          const uint64_t u = __umul64hi(c[j], W);
          int64_t lo = 0, hi = I;
          while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (tab(o + mid) > u)
              hi = mid;
            else
              lo = mid + 1;
          }
          if (lo > I - 1) lo = I - 1;  // only when W == 0 (rank-deficient factor)
          const uint64_t wi = tab(o + lo) - (lo > 0 ? tab(o + lo - 1) : 0ull);
          idx[static_cast<int64_t>(n) * s + t] = static_cast<int32_t>(lo);
          // weight = prod_n W_n / w_i, in mode order, then / s
          acc = acc * (static_cast<double>(W) / static_cast<double>(wi));
        }
      }
    }
    if (!aug) {
      weight[t] = acc / static_cast<double>(s);
      continue;
    }
    uint64_t c[4] = {static_cast<uint64_t>(t), counter, problem, kAugBlock};
    philox4x64_10(c, seed, 0ull);
    const uint64_t tot = coin_d + coin_c;
    if (__umul64hi(c[0], tot) >= coin_d) {
      // ridge row k of the d rows sqrt(lambda) e_k
      uint64_t k = __umul64hi(c[1], static_cast<uint64_t>(g.d));
      for (int n = N - 1; n >= 0; --n) {
        const uint64_t R = static_cast<uint64_t>(g.ranks[n]);
        idx[static_cast<int64_t>(n) * s + t] = static_cast<int32_t>(g.dims[n] + (k % R));
        k /= R;
      }
      const double r = static_cast<double>(tot) / static_cast<double>(coin_c);
      weight[t] = (r * static_cast<double>(g.d)) / static_cast<double>(s);
    } else {
      const double r = static_cast<double>(tot) / static_cast<double>(coin_d);
      weight[t] = (acc * r) / static_cast<double>(s);
    }
  }
}

// ---------------------------------------------------------------- ridge-score mixture
// Draws from the mixture of K's lambda-ridge scores over singular-value tuples
// (tables from ridge tables: tuple CDF over the d tuples, row-major over the
// ranks; the CDF of column c of mode n at qoff[n] + c I_n).  The tuple comes
// from word 0 of Philox block kRidgeBlock, then mode n's row from column t_n's
// table with the word that drives mode n in the product sampler.  With aug
// the branch coin of the augmented distribution is drawn as in sample_kernel;
// ridge rows get their weight here, data draws in ridge_weight_kernel.
constexpr uint64_t kRidgeBlock = 3;

__device__ inline int64_t upper_search(const uint64_t* __restrict__ C, int64_t len, uint64_t u) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (C[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo < len ? lo : len - 1;
}

__global__ __launch_bounds__(kBlock) void ridge_sample_kernel(
    Geom g, const uint64_t* __restrict__ tcdf, const uint64_t* __restrict__ ccdf, int64_t s,
    uint64_t seed, uint64_t counter, uint64_t problem, int aug, uint64_t coin_c, uint64_t coin_d,
    int32_t* __restrict__ idx, double* __restrict__ weight) {
  const int N = g.order;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < s;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    uint64_t c4[4] = {static_cast<uint64_t>(t), counter, problem, kRidgeBlock};
    philox4x64_10(c4, seed, 0ull);
    const uint64_t Wt = tcdf[g.d - 1];
    int64_t tup = upper_search(tcdf, g.d, __umul64hi(c4[0], Wt));
    int32_t col[kMaxOrder];
    for (int n = N - 1; n >= 0; --n) {
      col[n] = static_cast<int32_t>(tup % g.ranks[n]);
      tup /= g.ranks[n];
    }
    for (int b = 0; b * 4 < N; ++b) {
      uint64_t c[4] = {static_cast<uint64_t>(t), counter, problem, static_cast<uint64_t>(b)};
      philox4x64_10(c, seed, 0ull);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 4 * b + j;
        if (n < N) {
          const int64_t I = g.dims[n];
          const uint64_t* C = ccdf + g.qoff[n] + static_cast<int64_t>(col[n]) * I;
          const int64_t i = upper_search(C, I, __umul64hi(c[j], C[I - 1]));
          idx[static_cast<int64_t>(n) * s + t] = static_cast<int32_t>(i);
        }
      }
    }
    if (!aug) continue;
    uint64_t ca[4] = {static_cast<uint64_t>(t), counter, problem, kAugBlock};
    philox4x64_10(ca, seed, 0ull);
    const uint64_t tot = coin_d + coin_c;
    if (__umul64hi(ca[0], tot) >= coin_d) {
      uint64_t k = __umul64hi(ca[1], static_cast<uint64_t>(g.d));
      for (int n = N - 1; n >= 0; --n) {
        const uint64_t R = static_cast<uint64_t>(g.ranks[n]);
        idx[static_cast<int64_t>(n) * s + t] = static_cast<int32_t>(g.dims[n] + (k % R));
        k /= R;
      }
      const double r = static_cast<double>(tot) / static_cast<double>(coin_c);
      weight[t] = (r * static_cast<double>(g.d)) / static_cast<double>(s);
    }
  }
}

// Weight 1/(s P) of a data draw, P = sum_t (w_t / W) prod_n w_{n,t_n,i_n} / W_{n,t_n}:
// one wave per draw.  Lanes form u_n[c] = w_{n,c,i_n} / W_{n,c} in LDS, then the
// sum over tuples is contracted mode by mode from the last mode with rank >= 2
// to the first (Y[p] = sum_c Y[p R + c] u[c], lanes over p), each step a
// short dot product per lane; rank-1 modes multiply the result.  Dynamic LDS:
// sum_r + 2 bufmax doubles.
__global__ __launch_bounds__(64) void ridge_weight_kernel(
    Geom g, const uint64_t* __restrict__ tcdf, const uint64_t* __restrict__ ccdf,
    const int32_t* __restrict__ idx, int64_t s, int aug, uint64_t coin_c, uint64_t coin_d, int64_t bufmax,
    double* __restrict__ weight) {
  extern __shared__ double sm[];
  double* u = sm;                  // [sum_r]
  double* ya = u + g.sum_r;        // [bufmax]
  double* yb = ya + bufmax;        // [bufmax]
  const int lane = threadIdx.x;
  const int N = g.order;
  const double Wt = static_cast<double>(tcdf[g.d - 1]);
  for (int64_t t = blockIdx.x; t < s; t += gridDim.x) {
    if (aug && idx[t] >= g.dims[0]) continue;  // a ridge row: weighted by the sampler
    for (int j = lane; j < g.sum_r; j += 64) {
      int n = 0;
      while (j >= g.soff[n] + g.ranks[n]) ++n;
      const int c = j - g.soff[n];
      const int64_t I = g.dims[n];
      const uint64_t* C = ccdf + g.qoff[n] + static_cast<int64_t>(c) * I;
      const int64_t i = idx[static_cast<int64_t>(n) * s + t];
      const uint64_t Om = C[I - 1];
      const uint64_t om = C[i] - (i > 0 ? C[i - 1] : 0ull);
      u[j] = Om ? static_cast<double>(om) / static_cast<double>(Om) : 0.0;
    }
    __syncthreads();
    // contraction over the modes with rank >= 2, last to first
    int64_t len = g.d;
    const double* src = nullptr;  // nullptr: the tuple weights themselves
    double* dst = ya;
    double scal = 1.0;
    for (int n = N - 1; n >= 0; --n) {
      const int R = g.ranks[n];
      if (R < 2) {
        scal *= u[g.soff[n]];
        continue;
      }
      const int64_t out = len / R;
      const double* un = u + g.soff[n];
      for (int64_t p = lane; p < out; p += 64) {
        double acc = 0.0;
        for (int c = 0; c < R; ++c) {
          const int64_t e = p * R + c;
          const double y = src ? src[e]
                               : static_cast<double>(tcdf[e] - (e > 0 ? tcdf[e - 1] : 0ull));
          acc = fma(y, un[c], acc);
        }
        dst[p] = acc;
      }
      __syncthreads();
      src = dst;
      dst = (dst == ya) ? yb : ya;
      len = out;
    }
    if (lane == 0) {
      const double num =
          (src ? src[0] : static_cast<double>(tcdf[0])) * scal;  // sum_t w_t prod_n u_n[t_n]
      double w = Wt / num;
      if (aug) w = w * (static_cast<double>(coin_d + coin_c) / static_cast<double>(coin_d));
      weight[t] = w / static_cast<double>(s);
    }
    __syncthreads();
  }
}

}  // namespace

void launch_sample_ridge(const Geom& g, const uint64_t* tcdf, const uint64_t* ccdf, int64_t s,
                         uint64_t seed, uint64_t counter, uint64_t problem, int32_t* idx,
                         double* weight, hipStream_t st, int aug, uint64_t coin_c, int qbits) {
  const uint64_t coin_d = 1ull << qbits;
  if (s <= 0) return;
  const int64_t want = cdiv(s, kBlock);
  const int64_t res =
      resident_grid(reinterpret_cast<const void*>(&ridge_sample_kernel), kBlock, 0);
  hipLaunchKernelGGL(ridge_sample_kernel, dim3(static_cast<unsigned>(want < res ? want : res)),
                     dim3(kBlock), 0, st, g, tcdf, ccdf, s, seed, counter, problem, aug, coin_c,
                     coin_d,
                     idx, weight);
  // the largest intermediate of the contraction: d over the last rank >= 2
  int64_t bufmax = 1;
  for (int n = g.order - 1; n >= 0; --n)
    if (g.ranks[n] >= 2) {
      bufmax = g.d / g.ranks[n];
      break;
    }
  const size_t lds = sizeof(double) * (static_cast<size_t>(g.sum_r) + 2 * bufmax);
  ensure_dyn_lds(reinterpret_cast<const void*>(&ridge_weight_kernel), static_cast<int>(lds));
  const int64_t grid = s < 65536 ? s : 65536;
  hipLaunchKernelGGL(ridge_weight_kernel, dim3(static_cast<unsigned>(grid)), dim3(64), lds, st, g,
                     tcdf, ccdf, idx, s, aug, coin_c, coin_d, bufmax, weight);
}

void launch_sample(const Geom& g, const uint64_t* cdf, int64_t s, uint64_t seed, uint64_t counter,
                   uint64_t problem, int32_t* idx, double* weight, hipStream_t st, int aug,
                   uint64_t coin_c, int qbits) {
  const uint64_t coin_d = 1ull << qbits;
  if (s <= 0) return;
  if (g.total_rows <= kSampleLdsRows) {
    // as many workgroups as are resident at once (each stages the tables)
    const size_t lds = sizeof(uint64_t) * g.total_rows;
    const int64_t want = cdiv(s, kBlock);
    const int64_t res =
        resident_grid(reinterpret_cast<const void*>(&sample_kernel<true>), kBlock, lds);
    const unsigned grid = static_cast<unsigned>(want < res ? want : res);
    hipLaunchKernelGGL(sample_kernel<true>, dim3(grid), dim3(kBlock), lds, st, g, cdf, s, seed,
                       counter, problem, aug, coin_c, coin_d, idx, weight);
  } else {
    hipLaunchKernelGGL(sample_kernel<false>, dim3(static_cast<unsigned>(cdiv(s, kBlock))),
                       dim3(kBlock), 0, st, g, cdf, s, seed, counter, problem, aug, coin_c, coin_d,
                       idx,
                       weight);
  }
}

}  // namespace tk
