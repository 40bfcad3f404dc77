// Adjoint of the sampled core update with the sample set held fixed.
//
// The sampled update solves M g = sum_t w_t x_t k_t with
// M = sum_t w_t k_t k_t^T + lambda I (Alg. 1 normal equations, proof of
// Thm 4.2) and k_t = a^(1)_{i_1} (x) ... (x) a^(N)_{i_N}.  For a cotangent
// gbar and v = M^{-1} gbar, differentiating the normal equations gives
//   d<gbar, g>/d x_t = w_t (k_t . v)                       =: beta_t
//   d<gbar, g>/d k_t = w_t (x_t - k_t . g) v - beta_t g     =: alpha_t v - beta_t g
// and, since k_t is multilinear in the factor rows,
//   Abar(n)[i_n, :] += alpha_t (V x_{m != n} a^(m)_{i_m}) - beta_t (G x_{m != n} a^(m)_{i_m})
// with V, G the core-shaped v, g.  The sampling weights are not
// differentiated (the sketch is a fixed operator for this gradient).
//
// alpha_t and -beta_t come from the FP64 row kernels in whitened coordinates
// (k_t . v = q_t . h_v); the kernels here form the all-but-one-mode
// contractions of V and G at each sample's factor rows (FP64) and scatter
// them with FP64 atomics, and scatter beta_t into the dense tensor adjoint.
#include "tk_internal.h"

namespace tk {
namespace {

struct AdjFactors {
  const void* p[kMaxOrder];
};

constexpr int kAdjS = 64;  // samples per workgroup: one per lane of every wave

template <class T>
__global__ __launch_bounds__(kBlock) void adjoint_factor_kernel(
    Geom g, AdjFactors fp, const int32_t* __restrict__ idx, int64_t s,
    const double* __restrict__ V, const double* __restrict__ G,
    const double* __restrict__ alpha, const double* __restrict__ nbeta,
    double* __restrict__ abar) {
  extern __shared__ double adj_rows[];  // [sum_r][kAdjS]: factor row entries per sample
  __shared__ int32_t sidx[kMaxOrder][kAdjS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kAdjS;
  const int N = g.order, SR = g.sum_r;

  for (int e = threadIdx.x; e < SR * kAdjS; e += kBlock) {
    const int j = e / kAdjS, k = e % kAdjS;
    int n = 0;
    while (n + 1 < N && j >= g.soff[n + 1]) ++n;
    const int64_t t = t0 + k;
    double v = 0.0;
    if (t < s) {
      const int32_t i = idx[static_cast<int64_t>(n) * s + t];
      if (i >= 0 && i < g.dims[n])
        v = static_cast<double>(static_cast<const T*>(
            fp.p[n])[static_cast<int64_t>(i) * g.ranks[n] + (j - g.soff[n])]);
    }
    adj_rows[e] = v;
  }
  for (int e = threadIdx.x; e < N * kAdjS; e += kBlock) {
    const int n = e / kAdjS, k = e % kAdjS;
    const int64_t t = t0 + k;
    sidx[n][k] = t < s ? idx[static_cast<int64_t>(n) * s + t] : -1;
  }
  __syncthreads();

  const int64_t t = t0 + lane;
  const bool ok = t < s;
  const double al = ok ? alpha[t] : 0.0;
  const double nb = ok ? nbeta[t] : 0.0;
  int64_t cs[kMaxOrder];  // row-major strides of the core
  {
    int64_t acc = 1;
#pragma unroll
    for (int m = kMaxOrder - 1; m >= 0; --m) {
      cs[m] = acc;
      if (m < N) acc *= g.ranks[m];
    }
  }

  for (int j = wave; j < SR; j += kBlock / 64) {
    int n = 0;
    while (n + 1 < N && j >= g.soff[n + 1]) ++n;
    const int rn = j - g.soff[n];
    double zv = 0.0, zg = 0.0;
    if (N == 1) {
      zv = V[rn];
      zg = G[rn];
    } else {
      // innermost other mode: the last mode that is not n
      const int mi = (n == N - 1) ? N - 2 : N - 1;
      const int Ri = g.ranks[mi];
      const int64_t csi = cs[mi];
      const double* rowi = adj_rows + g.soff[mi] * kAdjS + lane;
      int dig[kMaxOrder];
#pragma unroll
      for (int m = 0; m < kMaxOrder; ++m) dig[m] = 0;
      const int64_t nout = g.d / (static_cast<int64_t>(g.ranks[n]) * Ri);
      for (int64_t oc = 0; oc < nout; ++oc) {
        int64_t base = rn * cs[n];
        double po = 1.0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
          if (m < N && m != n && m != mi) {
            base += dig[m] * cs[m];
            po *= adj_rows[(g.soff[m] + dig[m]) * kAdjS + lane];
          }
        }
        for (int k = 0; k < Ri; ++k) {
          const double a = po * rowi[k * kAdjS];
          zv = fma(a, V[base + k * csi], zv);
          zg = fma(a, G[base + k * csi], zg);
        }
        // next combination of the remaining modes (last one fastest)
#pragma unroll
        for (int m = kMaxOrder - 1; m >= 0; --m) {
          if (m < N && m != n && m != mi) {
            if (++dig[m] < g.ranks[m]) break;
            dig[m] = 0;
          }
        }
      }
    }
    if (ok) {
      const double c = al * zv + nb * zg;  // alpha_t V - beta_t G contracted
      const int32_t i = sidx[n][lane];
      if (i >= 0 && i < g.dims[n] && c != 0.0)
        unsafeAtomicAdd(&abar[g.qoff[n] + static_cast<int64_t>(i) * g.ranks[n] + rn], c);
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void adjoint_x_kernel(Geom g, const int32_t* __restrict__ idx,
                                                         int64_t s,
                                                         const double* __restrict__ nbeta,
                                                         T* __restrict__ xbar) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= s) return;
  int64_t flat = 0;
  for (int n = 0; n < g.order; ++n) {
    const int32_t i = idx[static_cast<int64_t>(n) * s + t];
    if (i < 0 || i >= g.dims[n]) return;  // flagged by the gather pass
    flat += static_cast<int64_t>(i) * g.strides[n];
  }
  const double b = -nbeta[t];
  if (b != 0.0) unsafeAtomicAdd(&xbar[flat], static_cast<T>(b));
}

__global__ __launch_bounds__(kBlock) void zero_words_kernel(uint32_t* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
    p[i] = 0u;
}

}  // namespace

size_t adjoint_lds_bytes(const Geom& g) {
  return sizeof(double) * static_cast<size_t>(g.sum_r) * kAdjS;
}

void launch_adjoint_factors(const Geom& g, const void* const* factors, tk_dtype dt,
                            const int32_t* idx, int64_t s, const double* V, const double* G,
                            const double* alpha, const double* nbeta, double* abar,
                            hipStream_t st) {
  AdjFactors fp;
  for (int n = 0; n < kMaxOrder; ++n) fp.p[n] = n < g.order ? factors[n] : nullptr;
  const dim3 grid(static_cast<unsigned>(cdiv(s, kAdjS)));
  const size_t lds = adjoint_lds_bytes(g);
  if (dt == TK_F64) {
    ensure_dyn_lds(reinterpret_cast<const void*>(&adjoint_factor_kernel<double>),
                   static_cast<int>(lds));
    hipLaunchKernelGGL(adjoint_factor_kernel<double>, grid, dim3(kBlock), lds, st, g, fp, idx, s,
                       V, G, alpha, nbeta, abar);
  } else {
    ensure_dyn_lds(reinterpret_cast<const void*>(&adjoint_factor_kernel<float>),
                   static_cast<int>(lds));
    hipLaunchKernelGGL(adjoint_factor_kernel<float>, grid, dim3(kBlock), lds, st, g, fp, idx, s, V,
                       G, alpha, nbeta, abar);
  }
}

void launch_adjoint_x(const Geom& g, const int32_t* idx, int64_t s, const double* nbeta,
                      void* xbar, tk_dtype dt, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(cdiv(s, kBlock)));
  if (dt == TK_F64)
    hipLaunchKernelGGL(adjoint_x_kernel<double>, grid, dim3(kBlock), 0, st, g, idx, s, nbeta,
                       static_cast<double*>(xbar));
  else
    hipLaunchKernelGGL(adjoint_x_kernel<float>, grid, dim3(kBlock), 0, st, g, idx, s, nbeta,
                       static_cast<float*>(xbar));
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>(bytes / 4);
  if (words <= 0) return;
  int64_t blocks = cdiv(words, kBlock);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_words_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st,
                     static_cast<uint32_t*>(p), words);
}

}  // namespace tk
