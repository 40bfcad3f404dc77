// MFMA operand variants shared by the Gram kernels (FP64, FP32, BF16 on
// gfx950) and the lower-triangular tile numbering.
#pragma once
#include "tk_internal.h"

namespace tk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
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

}  // namespace tk
