// Mode-n products and small FP64 helpers.
//
// n-mode product (Sec. 2): (T x_n M)[.., j, ..] = sum_i M[j, i] T[.., i, ..].
// A row-major tensor is viewed as (P, I, Q) around mode n; every thread owns
// one (p, q) fibre and produces all J outputs, so each input element is read
// once and reads are coalesced along q.  Large contractions run on FP64 MFMA:
// when mode n is the last mode (Q = 1) rows of the input are staged through
// LDS; otherwise each p is a (J x I) (I x Q) product read along q.
#include "tk_internal.h"

namespace tk {
namespace {

template <class T>
__device__ inline double ldd(const T* p, int64_t i) {
  return static_cast<double>(p[i]);
}

// Mat(j, i): M stored J x I (trans = false) or I x J (trans = true)
__device__ inline double mat(const double* M, int64_t I, int64_t J, bool trans, int64_t j,
                             int64_t i) {
  return trans ? M[i * J + j] : M[j * I + i];
}

// outputs j in [j0, j0 + jn), jn <= JMAX; input range i in [ia, ib) of split blockIdx.y
// (ib - ia = ilen); writes out + blockIdx.y * split_stride.
template <class T, int JMAX>
__global__ __launch_bounds__(kBlock) void ttm_fibre_kernel(const T* __restrict__ in, int64_t P,
                                                           int64_t I, int64_t Q,
                                                           const double* __restrict__ M, int64_t J,
                                                           bool trans, int64_t j0, int jn,
                                                           int64_t ilen, int64_t split_stride,
                                                           double* __restrict__ out,
                                                           const int32_t* done) {
  if (done && *done) return;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= P * Q) return;
  const int64_t p = e / Q, q = e % Q;
  const int64_t ia = static_cast<int64_t>(blockIdx.y) * ilen;
  const int64_t ib = (ia + ilen < I) ? ia + ilen : I;
  double acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) acc[j] = 0.0;
  const T* src = in + p * I * Q + q;
#pragma unroll 4
  for (int64_t i = ia; i < ib; ++i) {
    const double x = ldd(src, i * Q);
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
      if (j < jn) acc[j] = fma(mat(M, I, J, trans, j0 + j, i), x, acc[j]);
  }
  double* dst = out + static_cast<int64_t>(blockIdx.y) * split_stride + p * J * Q + q;
#pragma unroll
  for (int j = 0; j < JMAX; ++j)
    if (j < jn) dst[(j0 + j) * Q] = acc[j];
}

__global__ void sum_splits_kernel(const double* __restrict__ part, int64_t nsplit, int64_t n,
                                  double* __restrict__ out, const int32_t* done) {
  if (done && *done) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int64_t k = 0; k < nsplit; ++k) v += part[k * n + i];
  out[i] = v;
}

// Q == 1: out[p][j] = sum_i Mat(j, i) in[p][i] -- a (P x I) (I x J) product,
// J <= 64, run on v_mfma_f64_16x16x4: 64 rows per workgroup (a 16-row strip
// per wave), i in chunks of 32 staged through LDS in FP64 (the input converted
// exactly) with coalesced 16-byte loads, the next chunk prefetched into
// registers while the current one is multiplied.
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double ttm_doublex4;
constexpr int kTlRows = 64, kTlK = 32, kTlLd = kTlK + 1;

template <class T>
struct TlLoad;
template <>
struct TlLoad<float> {  // 64 rows x 32 floats = 512 x 16 bytes: two per thread
  static constexpr int N = 2;
  typedef float __attribute__((ext_vector_type(4))) vec;
  static constexpr int W = 4;
};
template <>
struct TlLoad<double> {  // 64 rows x 32 doubles = 1024 x 16 bytes: four per thread
  static constexpr int N = 4;
  typedef double __attribute__((ext_vector_type(2))) vec;
  static constexpr int W = 2;
};

template <class T>
__global__ __launch_bounds__(kBlock) void ttm_last_kernel(const T* __restrict__ in, int64_t P,
                                                          int64_t I, const double* __restrict__ M,
                                                          int64_t J, bool trans,
                                                          double* __restrict__ out,
                                                          const int32_t* done) {
  if (done && *done) return;
  using LD = TlLoad<T>;
  using vec = typename LD::vec;
  constexpr int W = LD::W, PER_ROW = kTlK / W;
  __shared__ double Xs[kTlRows * kTlLd];
  __shared__ double Ws[kMaxRank * kTlLd];  // Ws[j][i]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * kTlRows;
  const int jb = static_cast<int>((J + 15) / 16);
  // vectors of the chunk this thread loads: e = tid + 256 q -> row e / PER_ROW, cols W (e % PER_ROW)
  vec pf[LD::N];
  const bool vec_ok = (I % W) == 0;  // whole vectors inside each row
  auto fetch = [&](int64_t i0) {
#pragma unroll
    for (int q = 0; q < LD::N; ++q) {
      const int e = tid + q * kBlock;
      const int r = e / PER_ROW, c = (e % PER_ROW) * W;
      const int64_t p = p0 + r < P ? p0 + r : P - 1;
      const int64_t i = i0 + c;
      if (vec_ok && i + W <= I) {
        pf[q] = *reinterpret_cast<const vec*>(in + p * I + i);
      } else {
#pragma unroll
        for (int t = 0; t < W; ++t) pf[q][t] = i + t < I ? in[p * I + i + t] : T(0);
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int q = 0; q < LD::N; ++q) {
      const int e = tid + q * kBlock;
      const int r = e / PER_ROW, c = (e % PER_ROW) * W;
#pragma unroll
      for (int t = 0; t < W; ++t) Xs[r * kTlLd + c + t] = static_cast<double>(pf[q][t]);
    }
  };
  ttm_doublex4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = ttm_doublex4{0, 0, 0, 0};
  fetch(0);
  for (int64_t i0 = 0; i0 < I; i0 += kTlK) {
    __syncthreads();  // the previous chunk's LDS reads are done
    commit();
    for (int e = tid; e < jb * 16 * kTlK; e += kBlock) {
      const int j = e / kTlK, c = e % kTlK;
      const int64_t i = i0 + c;
      Ws[j * kTlLd + c] = (j < J && i < I) ? mat(M, I, J, trans, j, i) : 0.0;
    }
    __syncthreads();
    if (i0 + kTlK < I) fetch(i0 + kTlK);
#pragma unroll 2
    for (int kk = 0; kk < kTlK; kk += 4) {
      const double av = Xs[(wave * 16 + lane % 16) * kTlLd + kk + lane / 16];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        if (cb < jb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              av, Ws[(cb * 16 + lane % 16) * kTlLd + kk + lane / 16], acc[cb], 0, 0, 0);
    }
  }
  // accumulator register v of lane l: row l / 16 + 4 v, column l % 16 of the 16 x 16 block
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    if (cb >= jb) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t p = p0 + wave * 16 + lane / 16 + 4 * v;
      const int64_t j = cb * 16 + lane % 16;
      if (p < P && j < J) out[p * J + j] = acc[cb][v];
    }
  }
}

// Q == 1 with few outputs (J <= 8) and I J <= 4096: out[p][j] = sum_i Mat(j, i)
// in[p][i] streamed at HBM speed without padding J to an MFMA block.  Lane l
// owns the columns i = 64 W m + W l + k (W elements of 16 bytes per load, m < NM)
// and keeps Mat for them in registers (NM W J doubles); a wave takes two rows
// at a time, each lane forms J partial sums per row with FP64 FMAs, and the
// partials are added across the wave by an xor tree.  Columns past I carry
// zero weights (their loads are clamped into the row).
template <class T>
struct SkinnyVec;
template <>
struct SkinnyVec<float> {
  typedef float __attribute__((ext_vector_type(4))) vec;
  static constexpr int W = 4;
};
template <>
struct SkinnyVec<double> {
  typedef double __attribute__((ext_vector_type(2))) vec;
  static constexpr int W = 2;
};

template <class T, int J, int NM>
__global__ __launch_bounds__(kBlock) void ttm_last_skinny_kernel(const T* __restrict__ in,
                                                                 int64_t P, int64_t I,
                                                                 const double* __restrict__ M,
                                                                 bool trans,
                                                                 double* __restrict__ out,
                                                                 const int32_t* done) {
  if (done && *done) return;
  using V = SkinnyVec<T>;
  using vec = typename V::vec;
  constexpr int W = V::W;
  const int lane = threadIdx.x & 63;
  double w[NM][W][J];
  int64_t col[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int64_t c0 = static_cast<int64_t>(m) * 64 * W + lane * W;
    col[m] = c0 + W <= I ? c0 : (I - W);  // clamped: a whole vector inside the row
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
      for (int j = 0; j < J; ++j) w[m][k][j] = c0 + W <= I ? mat(M, I, J, trans, j, c0 + k) : 0.0;
  }
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / 64);
  const int64_t wid = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
  for (int64_t p0 = 2 * wid; p0 < P; p0 += 2 * waves) {
    const bool two = p0 + 1 < P;
    vec x[2][NM];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const T* row = in + (r == 1 && two ? p0 + 1 : p0) * I;
#pragma unroll
      for (int m = 0; m < NM; ++m) x[r][m] = *reinterpret_cast<const vec*>(row + col[m]);
    }
    double acc[2][J];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < J; ++j) acc[r][j] = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double xv = static_cast<double>(x[r][m][k]);
#pragma unroll
          for (int j = 0; j < J; ++j) acc[r][j] = fma(xv, w[m][k][j], acc[r][j]);
        }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        double v = acc[r][j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[r][j] = v;
      }
    if (lane < J) {
      double v0 = 0.0, v1 = 0.0;
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (j == lane) {
          v0 = acc[0][j];
          v1 = acc[1][j];
        }
      out[p0 * J + lane] = v0;
      if (two) out[(p0 + 1) * J + lane] = v1;
    }
  }
}

// The same product when a row is too long for one wave's registers: the
// workgroup's four waves split each row's columns (wave v owns the columns
// 64 W (4 m + v) + W l + k), each forms its J partial sums, and the four
// partials are added in wave order through LDS.  Two rows per iteration.
template <class T, int J, int NM>
__global__ __launch_bounds__(kBlock) void ttm_last_skinny_wg_kernel(const T* __restrict__ in,
                                                                    int64_t P, int64_t I,
                                                                    const double* __restrict__ M,
                                                                    bool trans,
                                                                    double* __restrict__ out,
                                                                    const int32_t* done) {
  if (done && *done) return;
  using V = SkinnyVec<T>;
  using vec = typename V::vec;
  constexpr int W = V::W;
  __shared__ double red[2][kBlock / 64][J];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double w[NM][W][J];
  int64_t col[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int64_t c0 = (static_cast<int64_t>(m) * (kBlock / 64) + wave) * 64 * W + lane * W;
    col[m] = c0 + W <= I ? c0 : (I - W);  // clamped: a whole vector inside the row
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
      for (int j = 0; j < J; ++j) w[m][k][j] = c0 + W <= I ? mat(M, I, J, trans, j, c0 + k) : 0.0;
  }
  for (int64_t p0 = 2 * static_cast<int64_t>(blockIdx.x); p0 < P; p0 += 2 * gridDim.x) {
    const bool two = p0 + 1 < P;
    vec x[2][NM];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const T* row = in + (r == 1 && two ? p0 + 1 : p0) * I;
#pragma unroll
      for (int m = 0; m < NM; ++m) x[r][m] = *reinterpret_cast<const vec*>(row + col[m]);
    }
    double acc[2][J];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < J; ++j) acc[r][j] = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double xv = static_cast<double>(x[r][m][k]);
#pragma unroll
          for (int j = 0; j < J; ++j) acc[r][j] = fma(xv, w[m][k][j], acc[r][j]);
        }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        double v = acc[r][j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[r][j] = v;
      }
    __syncthreads();  // the previous rows' partials have been read
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < J; ++j) red[r][wave][j] = acc[r][j];
    }
    __syncthreads();
    if (threadIdx.x < 2 * J) {
      const int r = threadIdx.x / J, j = threadIdx.x % J;
      if (r == 0 || two) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) v += red[r][q][j];
        out[(p0 + r) * J + j] = v;
      }
    }
  }
}

template <class T, int J>
bool skinny_launch_j(const T* in, int64_t P, int64_t I, const double* M, bool trans, double* out,
                     hipStream_t st, const int32_t* done) {
  constexpr int W = SkinnyVec<T>::W;
  const int64_t nm = cdiv(I, 64 * W);
  const int64_t want = cdiv(P, 2 * (kBlock / 64));
  const dim3 grid(static_cast<unsigned>(want < 4096 ? want : 4096));
#define TK_SKINNY(NMV)                                                                          \
  if constexpr (NMV * W * J <= 64) {                                                            \
    if (nm <= NMV) {                                                                            \
      hipLaunchKernelGGL((ttm_last_skinny_kernel<T, J, NMV>), grid, dim3(kBlock), 0, st, in, P, \
                         I, M, trans, out, done);                                               \
      return true;                                                                              \
    }                                                                                           \
  }
  TK_SKINNY(1)
  TK_SKINNY(2)
  TK_SKINNY(4)
  TK_SKINNY(8)
  TK_SKINNY(16)
#undef TK_SKINNY
  // rows longer than one wave holds: four waves per row
  const int64_t nmw = cdiv(I, 4 * 64 * W);
  const int64_t wantw = cdiv(P, 2);
  const dim3 gridw(static_cast<unsigned>(wantw < 8192 ? wantw : 8192));
#define TK_SKINNY_WG(NMV)                                                                     \
  if constexpr (NMV * W * J <= 64) {                                                          \
    if (nmw <= NMV) {                                                                         \
      hipLaunchKernelGGL((ttm_last_skinny_wg_kernel<T, J, NMV>), gridw, dim3(kBlock), 0, st, \
                         in, P, I, M, trans, out, done);                                      \
      return true;                                                                            \
    }                                                                                         \
  }
  TK_SKINNY_WG(1)
  TK_SKINNY_WG(2)
  TK_SKINNY_WG(4)
  TK_SKINNY_WG(8)
  TK_SKINNY_WG(16)
#undef TK_SKINNY_WG
  return false;
}

template <class T>
bool skinny_launch(const T* in, int64_t P, int64_t I, const double* M, int64_t J, bool trans,
                   double* out, hipStream_t st, const int32_t* done) {
  constexpr int W = SkinnyVec<T>::W;
  if (I % W != 0 || I < W || (reinterpret_cast<uintptr_t>(in) % 16) != 0) return false;
  if (J == 1) return skinny_launch_j<T, 1>(in, P, I, M, trans, out, st, done);
  if (J == 2) return skinny_launch_j<T, 2>(in, P, I, M, trans, out, st, done);
  if (J == 4) return skinny_launch_j<T, 4>(in, P, I, M, trans, out, st, done);
  if (J == 8) return skinny_launch_j<T, 8>(in, P, I, M, trans, out, st, done);
  return false;
}

// Q > 1: out[p][j][q] = sum_i Mat(j, i) in[p][i][q] -- per p a (J x I) (I x Q)
// product on v_mfma_f64_16x16x4, J <= 16 JB.  A wave owns 64 consecutive q (four
// 16-column blocks) and all J outputs; Mat is staged through LDS in chunks of
// 64 i (the A operand, zero beyond I and J); the input is read directly in the
// B operand layout (lane l: i = k + l / 16, q = 16 t + l % 16, so each row
// contributes 16 consecutive elements), with indices clamped into range.
constexpr int kTmK = 64, kTmLd = kTmK + 1;

template <class T, int JB>
__global__ __launch_bounds__(kBlock) void ttm_mid_kernel(const T* __restrict__ in, int64_t I,
                                                         int64_t Q, const double* __restrict__ M,
                                                         int64_t J, bool trans,
                                                         double* __restrict__ out,
                                                         const int32_t* done) {
  if (done && *done) return;
  __shared__ double Ms[JB * 16 * kTmLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t p = blockIdx.y;
  const int64_t qw = static_cast<int64_t>(blockIdx.x) * 256 + wave * 64;
  const T* src = in + p * I * Q;
  int64_t qc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t q = qw + 16 * t + lr;
    qc[t] = q < Q ? q : Q - 1;
  }
  ttm_doublex4 acc[JB][4];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[jb][t] = ttm_doublex4{0, 0, 0, 0};
  for (int64_t i0 = 0; i0 < I; i0 += kTmK) {
    __syncthreads();  // the previous chunk's LDS reads are done
    for (int e = tid; e < JB * 16 * kTmK; e += kBlock) {
      const int j = e / kTmK, c = e % kTmK;
      const int64_t i = i0 + c;
      Ms[j * kTmLd + c] = (j < J && i < I) ? mat(M, I, J, trans, j, i) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kTmK; kk += 4) {
      const int64_t i = i0 + kk + lk;
      const T* row = src + (i < I ? i : I - 1) * Q;
      double b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = static_cast<double>(row[qc[t]]);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const double a = Ms[(jb * 16 + lr) * kTmLd + kk + lk];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[jb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[jb][t], 0, 0, 0);
      }
    }
  }
  // accumulator register v of lane l: row (j) l / 16 + 4 v, column (q) l % 16
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = jb * 16 + lk + 4 * v;
        const int64_t q = qw + 16 * t + lr;
        if (j < J && q < Q) out[(p * J + j) * Q + q] = acc[jb][t][v];
      }
}

// Q > 1 with few outputs (J <= 8): out[p][j][q] = sum_i Mat(j, i) in[p][i][q]
// without padding J to an MFMA block.  A thread owns W consecutive q (one
// 16-byte load per i) and walks i with four rows of loads in flight, keeping
// J W FP64 partial sums; Mat(j, i) is the same for the whole wave.
template <class T, int J>
__global__ __launch_bounds__(kBlock) void ttm_mid_skinny_kernel(const T* __restrict__ in,
                                                                int64_t I, int64_t Q,
                                                                const double* __restrict__ M,
                                                                bool trans,
                                                                double* __restrict__ out,
                                                                const int32_t* done) {
  if (done && *done) return;
  using V = SkinnyVec<T>;
  using vec = typename V::vec;
  constexpr int W = V::W;
  const int64_t p = blockIdx.y;
  const int64_t q0 = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) * W;
  if (q0 >= Q) return;
  const T* src = in + p * I * Q + q0;
  double acc[J][W];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int k = 0; k < W; ++k) acc[j][k] = 0.0;
  int64_t i = 0;
  for (; i + 4 <= I; i += 4) {
    vec x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = *reinterpret_cast<const vec*>(src + (i + u) * Q);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const double mv = mat(M, I, J, trans, j, i + u);
#pragma unroll
        for (int k = 0; k < W; ++k) acc[j][k] = fma(mv, static_cast<double>(x[u][k]), acc[j][k]);
      }
  }
  for (; i < I; ++i) {
    const vec x = *reinterpret_cast<const vec*>(src + i * Q);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const double mv = mat(M, I, J, trans, j, i);
#pragma unroll
      for (int k = 0; k < W; ++k) acc[j][k] = fma(mv, static_cast<double>(x[k]), acc[j][k]);
    }
  }
  double* dst = out + p * J * Q + q0;
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int k = 0; k < W; ++k) dst[j * Q + k] = acc[j][k];
}

template <class T>
bool mid_skinny_launch(const T* in, int64_t P, int64_t I, int64_t Q, const double* M, int64_t J,
                       bool trans, double* out, hipStream_t st, const int32_t* done) {
  constexpr int W = SkinnyVec<T>::W;
  if (Q % W != 0 || (reinterpret_cast<uintptr_t>(in) % 16) != 0 || P > 65535) return false;
  const dim3 grid(static_cast<unsigned>(cdiv(Q / W, kBlock)), static_cast<unsigned>(P));
  switch (J) {
    case 1:
      hipLaunchKernelGGL((ttm_mid_skinny_kernel<T, 1>), grid, dim3(kBlock), 0, st, in, I, Q, M,
                         trans, out, done);
      return true;
    case 2:
      hipLaunchKernelGGL((ttm_mid_skinny_kernel<T, 2>), grid, dim3(kBlock), 0, st, in, I, Q, M,
                         trans, out, done);
      return true;
    case 4:
      hipLaunchKernelGGL((ttm_mid_skinny_kernel<T, 4>), grid, dim3(kBlock), 0, st, in, I, Q, M,
                         trans, out, done);
      return true;
    case 8:
      hipLaunchKernelGGL((ttm_mid_skinny_kernel<T, 8>), grid, dim3(kBlock), 0, st, in, I, Q, M,
                         trans, out, done);
      return true;
    default:
      return false;
  }
}

constexpr int64_t kTtmThreadsWanted = 65536;

// Mq = M (x) I_Q in M's storage: trans (M is I x J): Mq[(i Q + q) (J Q) + j Q + q'] =
// M[i J + j] [q == q']; else (M is J x I): Mq[(j Q + q') (I Q) + i Q + q] = M[j I + i] [q == q'].
__global__ void kron_identity_kernel(const double* __restrict__ M, int64_t I, int64_t J, int64_t Q,
                                     bool trans, double* __restrict__ Mq) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= I * Q * J * Q) return;
  if (trans) {
    const int64_t row = e / (J * Q), col = e % (J * Q);
    const int64_t i = row / Q, q = row % Q, j = col / Q, q2 = col % Q;
    Mq[e] = q == q2 ? M[i * J + j] : 0.0;
  } else {
    const int64_t row = e / (I * Q), col = e % (I * Q);
    const int64_t j = row / Q, q2 = row % Q, i = col / Q, q = col % Q;
    Mq[e] = q == q2 ? M[j * I + i] : 0.0;
  }
}

template <class T>
void ttm_dispatch(const T* in, const int64_t* dims, int order, int mode, const double* M,
                  int64_t J, bool trans, double* out, double* scratch, hipStream_t st,
                  const int32_t* done) {
  int64_t P = 1, Q = 1;
  for (int m = 0; m < mode; ++m) P *= dims[m];
  for (int m = mode + 1; m < order; ++m) Q *= dims[m];
  const int64_t I = dims[mode];
  // A few trailing entries per fibre (Q small): read X as [P][I Q] rows and
  // contract them with M (x) I_Q, whose output [P][J Q] is the mode product's
  // [P][J][Q]; the rows are then long and contiguous.
  if (Q > 1 && Q <= 4 && J * Q <= kMaxRank && P >= 64 * 256 && scratch &&
      I * Q * J * Q <= kTtmScratchDoubles) {
    const int64_t e = I * Q * J * Q;
    hipLaunchKernelGGL(kron_identity_kernel, dim3(static_cast<unsigned>(cdiv(e, kBlock))),
                       dim3(kBlock), 0, st, M, I, J, Q, trans, scratch);
    hipLaunchKernelGGL(ttm_last_kernel<T>, dim3(static_cast<unsigned>(cdiv(P, 64))), dim3(kBlock),
                       0, st, in, P, I * Q, scratch, J * Q, trans, out, done);
    return;
  }
  if (Q == 1 && J <= 8 && I * J <= 16384 && P >= 4096 &&
      skinny_launch(in, P, I, M, J, trans, out, st, done))
    return;
  if (Q == 1 && J <= kMaxRank && P >= 64 * 256) {
    hipLaunchKernelGGL(ttm_last_kernel<T>, dim3(static_cast<unsigned>(cdiv(P, 64))), dim3(kBlock),
                       0, st, in, P, I, M, J, trans, out, done);
    return;
  }
  if (Q >= 256 && J <= 8 && P * cdiv(Q, 1024) >= 256 &&
      mid_skinny_launch(in, P, I, Q, M, J, trans, out, st, done))
    return;
  if (Q >= 64 && J <= kMaxRank && P <= 65535 && P * cdiv(Q, 256) >= 512) {
    const dim3 grid(static_cast<unsigned>(cdiv(Q, 256)), static_cast<unsigned>(P));
    if (J <= 16)
      hipLaunchKernelGGL((ttm_mid_kernel<T, 1>), grid, dim3(kBlock), 0, st, in, I, Q, M, J, trans,
                         out, done);
    else if (J <= 32)
      hipLaunchKernelGGL((ttm_mid_kernel<T, 2>), grid, dim3(kBlock), 0, st, in, I, Q, M, J, trans,
                         out, done);
    else
      hipLaunchKernelGGL((ttm_mid_kernel<T, 4>), grid, dim3(kBlock), 0, st, in, I, Q, M, J, trans,
                         out, done);
    return;
  }
  // split the contraction over i when there are too few fibres to fill the GPU
  int64_t nsplit = 1;
  if (scratch && P * Q < kTtmThreadsWanted) {
    nsplit = cdiv(kTtmThreadsWanted, P * Q);
    const int64_t maxs = cdiv(I, 8);
    if (nsplit > maxs) nsplit = maxs;
    if (nsplit > kTtmScratchDoubles / (P * J * Q)) nsplit = kTtmScratchDoubles / (P * J * Q);
    if (nsplit < 1) nsplit = 1;
  }
  const int64_t ilen = cdiv(I, nsplit);
  nsplit = cdiv(I, ilen);
  double* dst = nsplit > 1 ? scratch : out;
  const int64_t stride = P * J * Q;
  const dim3 grid(static_cast<unsigned>(cdiv(P * Q, kBlock)), static_cast<unsigned>(nsplit));
  for (int64_t j0 = 0; j0 < J; j0 += 64) {
    const int jn = static_cast<int>((J - j0) < 64 ? (J - j0) : 64);
    if (jn <= 8)
      hipLaunchKernelGGL((ttm_fibre_kernel<T, 8>), grid, dim3(kBlock), 0, st, in, P, I, Q, M, J,
                         trans, j0, jn, ilen, stride, dst, done);
    else if (jn <= 16)
      hipLaunchKernelGGL((ttm_fibre_kernel<T, 16>), grid, dim3(kBlock), 0, st, in, P, I, Q, M, J,
                         trans, j0, jn, ilen, stride, dst, done);
    else if (jn <= 32)
      hipLaunchKernelGGL((ttm_fibre_kernel<T, 32>), grid, dim3(kBlock), 0, st, in, P, I, Q, M, J,
                         trans, j0, jn, ilen, stride, dst, done);
    else
      hipLaunchKernelGGL((ttm_fibre_kernel<T, 64>), grid, dim3(kBlock), 0, st, in, P, I, Q, M, J,
                         trans, j0, jn, ilen, stride, dst, done);
  }
  if (nsplit > 1)
    hipLaunchKernelGGL(sum_splits_kernel, dim3(static_cast<unsigned>(cdiv(stride, kBlock))),
                       dim3(kBlock), 0, st, static_cast<const double*>(scratch), nsplit, stride,
                       out, done);
}

template <class To, class From>
__global__ void cast_kernel(int64_t n, const From* __restrict__ x, To* __restrict__ y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] = static_cast<To>(x[i]);
}

template <class T>
__global__ void fill_kernel(int64_t n, T v, T* __restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// The per-call words of a sampled update in their starting state.
__global__ void init_words_kernel(int32_t* status, int32_t* done, int32_t* steps, double* relres,
                                  double* min_pivot, uint32_t* missing) {
  *status = 0;
  *done = 0;
  *steps = 0;
  *relres = 0.0;
  *min_pivot = 1e308;
  *missing = 0u;
}

// r <- r - lambda * ph (when ph != null); relres = ||r|| / ||rhs||; done when <= tol.
__global__ __launch_bounds__(1024) void refine_check_kernel(int64_t d, double* __restrict__ r,
                                                            const double* __restrict__ ph,
                                                            const double* __restrict__ bvec,
                                                            double lambda,
                                                            const double* __restrict__ rhs,
                                                            double tol, int32_t* done,
                                                            int32_t* steps, double* relres,
                                                            int count_step) {
  if (*done) return;
  __shared__ double s1[1024], s2[1024];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    double v = r[i];
    if (bvec) v += bvec[i];
    if (ph) v = fma(-lambda, ph[i], v);
    if (bvec || ph) r[i] = v;
    a = fma(v, v, a);
    b = fma(rhs[i], rhs[i], b);
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double rel = s2[0] > 0.0 ? sqrt(s1[0] / s2[0]) : sqrt(s1[0]);
    *relres = rel;
    if (rel <= tol) {
      *done = 1;
    } else if (count_step) {
      *steps += 1;
    }
  }
}

__global__ void info_kernel(double* info, int64_t s, const unsigned int* missing,
                            const int32_t* steps, const double* relres, const double* min_pivot) {
  if (threadIdx.x != 0) return;
  info[0] = static_cast<double>(s);
  info[1] = missing ? static_cast<double>(*missing) : 0.0;
  info[2] = steps ? static_cast<double>(*steps) : 0.0;
  info[3] = relres ? *relres : 0.0;
  info[4] = min_pivot ? *min_pivot : 0.0;
  info[5] = info[6] = info[7] = 0.0;
}

__global__ void finish_refine_kernel(const int32_t* done, int refine_enabled, int32_t* status) {
  if (threadIdx.x == 0 && refine_enabled && !*done)
    atomicMax(status, static_cast<int32_t>(TK_E_NO_CONVERGE));
}

}  // namespace

void launch_ttm(const double* T, const int64_t* dims, int order, int mode, const double* M,
                int64_t J, bool transpose_M, double* out, double* scratch, hipStream_t st,
                const int32_t* done) {
  ttm_dispatch<double>(T, dims, order, mode, M, J, transpose_M, out, scratch, st, done);
}

void launch_ttm_any(const void* T, tk_dtype dt, const int64_t* dims, int order, int mode,
                    const double* M, int64_t J, bool transpose_M, double* out, double* scratch,
                    hipStream_t st) {
  if (dt == TK_F64)
    ttm_dispatch<double>(static_cast<const double*>(T), dims, order, mode, M, J, transpose_M, out,
                         scratch, st, nullptr);
  else
    ttm_dispatch<float>(static_cast<const float*>(T), dims, order, mode, M, J, transpose_M, out,
                        scratch, st, nullptr);
}

void launch_copy_f64(int64_t n, const double* x, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((cast_kernel<double, double>), dim3(static_cast<unsigned>(cdiv(n, kBlock))),
                     dim3(kBlock), 0, st, n, x, y);
}

void launch_cast_out(int64_t n, const double* x, void* y, tk_dtype dt, hipStream_t st) {
  if (n <= 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(n, kBlock)));
  if (dt == TK_F64)
    hipLaunchKernelGGL((cast_kernel<double, double>), grid, dim3(kBlock), 0, st, n, x,
                       static_cast<double*>(y));
  else
    hipLaunchKernelGGL((cast_kernel<float, double>), grid, dim3(kBlock), 0, st, n, x,
                       static_cast<float*>(y));
}

void launch_cast_in(int64_t n, const void* x, tk_dtype dt, double* y, hipStream_t st) {
  if (n <= 0) return;
  const dim3 grid(static_cast<unsigned>(cdiv(n, kBlock)));
  if (dt == TK_F64)
    hipLaunchKernelGGL((cast_kernel<double, double>), grid, dim3(kBlock), 0, st, n,
                       static_cast<const double*>(x), y);
  else
    hipLaunchKernelGGL((cast_kernel<double, float>), grid, dim3(kBlock), 0, st, n,
                       static_cast<const float*>(x), y);
}

void launch_fill_i32(int64_t n, int32_t v, int32_t* p, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<int32_t>, dim3(static_cast<unsigned>(cdiv(n, kBlock))),
                     dim3(kBlock), 0, st, n, v, p);
}

void launch_fill_f64(int64_t n, double v, double* p, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(static_cast<unsigned>(cdiv(n, kBlock))),
                     dim3(kBlock), 0, st, n, v, p);
}

void launch_init_words(int32_t* status, int32_t* done, int32_t* steps, double* relres,
                       double* min_pivot, uint32_t* missing, hipStream_t st) {
  hipLaunchKernelGGL(init_words_kernel, dim3(1), dim3(1), 0, st, status, done, steps, relres,
                     min_pivot, missing);
}

void launch_fill_u32(int64_t n, uint32_t v, uint32_t* p, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(static_cast<unsigned>(cdiv(n, kBlock))),
                     dim3(kBlock), 0, st, n, v, p);
}

void launch_refine_check(int64_t d, double* r, const double* ph, const double* b, double lambda,
                         const double* rhs, double tol, int32_t* done, int32_t* steps,
                         double* relres, int count_step, hipStream_t st) {
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(1024), 0, st, d, r, ph, b, lambda, rhs, tol,
                     done, steps, relres, count_step);
}

void launch_info(double* info, int64_t s, const unsigned int* missing, const int32_t* steps,
                 const double* relres, const double* min_pivot, hipStream_t st) {
  hipLaunchKernelGGL(info_kernel, dim3(1), dim3(64), 0, st, info, s, missing, steps, relres,
                     min_pivot);
}

void launch_finish_refine(const int32_t* done, int refine_enabled, int32_t* status,
                          hipStream_t st) {
  hipLaunchKernelGGL(finish_refine_kernel, dim3(1), dim3(64), 0, st, done, refine_enabled, status);
}

}  // namespace tk
