// Stream-K sketched Gram on MFMA (FP32 or BF16 operands, FP32 accumulation)
// for one problem or a batch of problems in one persistent launch.
//
// The Gram of a problem is sum_t w_t q_t q_t^T over its samples (proof of
// Thm 4.2: s outer products of design rows), with q_t the whitened Kronecker
// row of sample t.  Its lower triangle is cut into T x T output tiles.  A
// unit of work is (tile, chunk of 32 samples); the units of all problems of
// a launch are laid out problem by problem, tile by tile, and workgroup w of
// G walks units [w U / G, (w + 1) U / G).  Where that range crosses a tile
// (or problem) boundary the workgroup writes the finished partial tile to its
// next slot; an index kernel gives every workgroup its first slot and first
// tile, and the assembly kernel sums a tile's slots in workgroup order
// (deterministic for a fixed grid).
//
// Per chunk a workgroup stages the chunk's factor rows in LDS (prefetched in
// registers while the previous chunk's MFMAs run), forms the two Kronecker
// row tiles y[r][t] = O[r / R_L][t] q_L[r % R_L][t] in the operand precision,
// O[o][t] being the product of the entries of all modes but the last mode L
// of rank >= 2 (each thread reads its rows' outer factors straight from the
// staged rows), and runs the 32 x 32 MFMAs.  Up to three (T = 128) or four
// (T = 64) workgroups share a CU, so some form rows while others run MFMA.
#include <string.h>

#include <type_traits>

#include "tk_mfma.h"

namespace tk {
namespace {

// Padded LDS rows of the staged factor entries.  One-row items read 16 bytes
// from consecutive rows: a stride of 36 floats spreads 16 lanes over all 64
// banks.  Four-row items read 128 contiguous bytes from each of two rows 4
// apart per 16 lanes: a stride of 40 floats puts them half a bank sweep apart.
constexpr int kSkRT = kRowChunk + 4;
constexpr int kSkRT4 = kRowChunk + 8;
constexpr size_t kSkMaxLds = 160 * 1024;  // LDS per CU on gfx950

// Tile edge T: 64 and 128 use 2 x 2 waves (32 x 32 or 64 x 64 each, up to 4
// or 3 workgroups per CU); 256 uses 4 x 4 waves of 64 x 64 in one
// 1024-thread workgroup per CU, which halves the row formation per MFMA and
// keeps four waves per SIMD to hide the formation's LDS latency.
template <int T>
struct SkTile {
  static constexpr int NO = T / 2 + 1;  // outer indices per tile when R_L >= 2
  static constexpr int WAVES_R = T == 256 ? 4 : 2;
  static constexpr int WAVES_C = T == 256 ? 4 : 2;
  static constexpr int THREADS = 64 * WAVES_R * WAVES_C;
  static constexpr int WG_PER_CU = T == 128 ? 3 : (T == 64 ? 4 : 1);
};

// LDS: NBUF sets of the two Kronecker row tiles, the outer-factor offsets,
// then NBUF staged chunks of factor rows (sum_r rows plus one zero row each).
template <class V, int T, int NBUF>
struct SkLayout {
  static constexpr int BK = V::BK;
  static constexpr int NO = SkTile<T>::NO;
  static constexpr size_t y_bytes = sizeof(typename V::Op) * T * V::LDK;   // one side
  static constexpr size_t offs_bytes = 2 * NO * kMaxOrder;
  static constexpr size_t fixed = NBUF * 2 * y_bytes + offs_bytes;
  __host__ __device__ static size_t rows_elems(int sum_r) {
    return static_cast<size_t>(sum_r + 1) * kSkRT4;  // room for either stride
  }
  __host__ __device__ static size_t bytes(int sum_r) {
    return fixed + NBUF * sizeof(typename V::Src) * rows_elems(sum_r);
  }
};

// prefetch registers (16-byte) per thread: a chunk holds kRowChunk * sum_r values
template <int THREADS>
struct SkPf {
  static constexpr int SMALL = THREADS >= 1024 ? 1 : 2;  // sum_r <= 128 / 64
  static constexpr int LARGE = (kRowChunk * kMaxSumR / 4 + THREADS - 1) / THREADS;
  static constexpr bool small(int sum_r) { return kRowChunk * sum_r <= 4 * THREADS * SMALL; }
};

__host__ __device__ inline int64_t sk_unit_start(int64_t w, int64_t units, int64_t grid) {
  return (w * units) / grid;
}

__device__ inline int sk_problem_of(const SkBatch& b, int64_t u) {
  int p = 0;
  while (p + 1 < b.count && b.p[p + 1].unit0 <= u) ++p;
  return p;
}

__device__ inline int64_t sk_tile_of(const SkBatch& b, int64_t u) {
  const int p = sk_problem_of(b, u);
  return b.p[p].tile0 + (u - b.p[p].unit0) / row_chunks(b.p[p].s);
}

// Geometry of one problem, derived from its descriptor.
struct SkGeom {
  int order, last, sum_r, rl, sl;
  int64_t d, nchunks;
  int ranks[kMaxOrder], soff[kMaxOrder];
};

__device__ inline SkGeom sk_geom(const SkProb& q) {
  SkGeom g;
  g.order = q.order;
  g.last = q.last;
  g.sum_r = q.sum_r;
  g.d = 1;
  int so = 0;
#pragma unroll
  for (int n = 0; n < kMaxOrder; ++n) {
    const int r = n < q.order ? q.ranks[n] : 1;
    g.ranks[n] = r;
    g.soff[n] = so;
    so += n < q.order ? r : 0;
    g.d *= r;
  }
  g.rl = g.ranks[g.last];
  g.sl = g.soff[g.last];
  g.nchunks = row_chunks(q.s);
  return g;
}

// LDS row positions of the outer factors of outer index o: for the modes
// before L, soff_n + digit_n(o); modes after L have rank 1 (digit 0).
__device__ inline void sk_outer_offsets(const SkGeom& g, int64_t o, unsigned char* offs) {
  unsigned char tmp[kMaxOrder];
  int64_t rem = o;
  for (int n = g.last - 1; n >= 0; --n) {
    tmp[n] = static_cast<unsigned char>(g.soff[n] + rem % g.ranks[n]);
    rem /= g.ranks[n];
  }
  int k = 0;
  for (int n = 0; n < g.last; ++n) offs[k++] = tmp[n];
  for (int n = g.last + 1; n < g.order; ++n) offs[k++] = static_cast<unsigned char>(g.soff[n]);
  for (; k < kMaxOrder; ++k) offs[k] = 0;
}

// index[w] = first slot of workgroup w, index[G + w] = its first tile (-1: empty range)
__global__ __launch_bounds__(1024) void sk_index_kernel(SkBatch b, int64_t* __restrict__ index) {
  __shared__ int64_t part[1024];
  const int64_t G = b.grid;
  int64_t carry = 0;
  for (int64_t w0 = 0; w0 < G; w0 += 1024) {
    const int64_t w = w0 + threadIdx.x;
    int64_t segs = 0, first = -1;
    if (w < G) {
      const int64_t u0 = sk_unit_start(w, b.units, G), u1 = sk_unit_start(w + 1, b.units, G);
      if (u1 > u0) {
        first = sk_tile_of(b, u0);
        segs = sk_tile_of(b, u1 - 1) - first + 1;
      }
      index[G + w] = first;
    }
    part[threadIdx.x] = segs;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
      const int64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += v;
      __syncthreads();
    }
    if (w < G) index[w] = carry + part[threadIdx.x] - segs;
    carry += part[1023];
    __syncthreads();
  }
}

// DB: two sets of row tiles and staged chunks, so that the rows of chunk
// c + 1 are formed while the MFMAs of chunk c run, one barrier per chunk.
template <class V, int T, int PF4, bool DB>
__global__ __launch_bounds__(SkTile<T>::THREADS, SkTile<T>::WG_PER_CU) void gram_sk_kernel(
    SkBatch b, typename V::Out* __restrict__ slots, const int64_t* __restrict__ index) {
  using Src = typename V::Src;
  using Op = typename V::Op;
  using Acc = typename V::Acc;
  constexpr int NBUF = DB ? 2 : 1;
  using L = SkLayout<V, T, NBUF>;
  constexpr int BK = V::BK, LDK = V::LDK, RT = kSkRT, NO = L::NO;
  constexpr int IW = V::EPL == 8 ? 8 : 4;         // samples per formation item
  constexpr int IPR = BK / IW;                    // items per row
  constexpr int kSkThreads = SkTile<T>::THREADS;
  constexpr int ITEMS = T * IPR / kSkThreads;     // items per thread per side
  static_assert(BK == kRowChunk, "chunk size");
  static_assert(ITEMS >= 1, "tile too small for the workgroup");
  extern __shared__ __align__(16) unsigned char sk_smem[];
  Op* YA = reinterpret_cast<Op*>(sk_smem);
  Op* YBs = reinterpret_cast<Op*>(sk_smem + L::y_bytes);
  unsigned char* offs = sk_smem + NBUF * 2 * L::y_bytes;            // [2][NO][kMaxOrder]
  Src* rT = reinterpret_cast<Src*>(sk_smem + L::fixed);             // [sum_r + 1][RT]
  // second set (DB): row tiles after the first pair, staged rows after rT
  Op* YA2 = reinterpret_cast<Op*>(sk_smem + 2 * L::y_bytes);
  Op* YB2s = reinterpret_cast<Op*>(sk_smem + 3 * L::y_bytes);
  Src* rT2 = rT + L::rows_elems(b.max_sum_r);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t w = blockIdx.x;
  const int64_t u0 = sk_unit_start(w, b.units, b.grid), u1 = sk_unit_start(w + 1, b.units, b.grid);
  if (u0 >= u1) return;
  const int64_t slot0 = index[w];

  constexpr int WR = T / SkTile<T>::WAVES_R, WC = T / SkTile<T>::WAVES_C;
  constexpr int NBR = WR / V::MT, NBC = WC / V::MT;
  const int wr = wave / SkTile<T>::WAVES_C, wc = wave % SkTile<T>::WAVES_C;
  Acc acc[NBR][NBC];

  f32x4 pf[PF4];
  int64_t u = u0;
  int seg = 0;
  while (u < u1) {
    const int pi = sk_problem_of(b, u);
    const SkProb& pd = b.p[pi];
    const SkGeom g = sk_geom(pd);
    const int N = g.order, RL = g.rl, SR = g.sum_r, sl = g.sl;
    const int64_t d = g.d;
    const Src* rows = pd.rows;
    const int nval4 = BK * SR / 4;
    const int64_t lu = u - pd.unit0;  // unit within the problem
    const int64_t tau = lu / g.nchunks;
    const int64_t c_begin = lu - tau * g.nchunks;
    const int64_t tile_end = pd.unit0 + (tau + 1) * g.nchunks;
    const int64_t c_end = (u1 < tile_end ? u1 : tile_end) - pd.unit0 - tau * g.nchunks;
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
    // the formation this tile takes (four-row items, below) fixes the stride
    // of the staged rows
    bool use4 = false;
    if constexpr (V::EPL == 8 && T == 256) use4 = RL % 4 == 0 && N <= 4 && !diag;
    const int rt = use4 ? kSkRT4 : kSkRT;
    auto fetch = [&](int64_t c) __attribute__((always_inline)) {
      const f32x4* src = reinterpret_cast<const f32x4*>(rows + c * BK * SR);
#pragma unroll
      for (int k = 0; k < PF4; ++k) {
        const int e = tid + k * kSkThreads;
        if (e < nval4) pf[k] = src[e];
      }
    };
    auto commit = [&](Src* rs) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < PF4; ++k) {
        const int e = tid + k * kSkThreads;
        if (e < nval4) {
          const int f = 4 * e;  // element index j * 32 + t
          *reinterpret_cast<f32x4*>(&rs[(f >> 5) * rt + (f & 31)]) = pf[k];
        }
      }
    };
    __syncthreads();  // the previous segment's LDS use is complete
    for (int e = tid; e < rt; e += kSkThreads) {  // zero rows
      rT[SR * rt + e] = Src(0);
      if (DB) rT2[SR * rt + e] = Src(0);
    }
#pragma unroll 1
    for (int e = tid; e < 2 * NO; e += kSkThreads) {
      const int side = e / NO, oi = e - side * NO;
      sk_outer_offsets(g, ob[side] + oi, offs + (side * NO + oi) * kMaxOrder);
    }
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
      for (int bb = 0; bb < NBC; ++bb)
#pragma unroll
        for (int v = 0; v < V::NACC; ++v) acc[a][bb][v] = 0;

    fetch(c_begin);
    commit(rT);
    __syncthreads();
    // a formation functor takes NM1 (= N - 1 outer factors) as a constant so
    // that its LDS reads issue together
    auto by_order = [&](auto form, const Src* rs, Op* ya, Op* yb) __attribute__((always_inline)) {
      static_assert(kMaxOrder == 8, "one case per order");
      switch (N) {
        case 1: form(std::integral_constant<int, 0>{}, rs, ya, yb); break;
        case 2: form(std::integral_constant<int, 1>{}, rs, ya, yb); break;
        case 3: form(std::integral_constant<int, 2>{}, rs, ya, yb); break;
        case 4: form(std::integral_constant<int, 3>{}, rs, ya, yb); break;
        case 5: form(std::integral_constant<int, 4>{}, rs, ya, yb); break;
        case 6: form(std::integral_constant<int, 5>{}, rs, ya, yb); break;
        case 7: form(std::integral_constant<int, 6>{}, rs, ya, yb); break;
        default: form(std::integral_constant<int, 7>{}, rs, ya, yb); break;
      }
    };
    // MFMAs of one chunk over its two row tiles
    auto mma_chunk = [&](const Op* ya, const Op* ybs) __attribute__((always_inline)) {
      const Op* yb = diag ? ya : ybs;
#pragma unroll
      for (int kk = 0; kk < BK; kk += V::KT) {
        const int kofs = kk + (lane / V::MT) * V::EPL;
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
          for (int bb = 0; bb < NBC; ++bb)
            acc[a][bb] = V::mma(&ya[(wr * WR + a * V::MT + lane % V::MT) * LDK + kofs],
                                &yb[(wc * WC + bb * V::MT + lane % V::MT) * LDK + kofs],
                                acc[a][bb]);
      }
    };
    // the chunks [c_begin, c_end) of the tile with a given row formation
    auto run = [&](auto form_rows) __attribute__((always_inline)) {
      if constexpr (DB) {
        // chunk c_begin + j lives in set j % 2; its rows are formed one
        // iteration ahead, and chunk c + 2 is staged where chunk c was
        if (c_begin + 1 < c_end) fetch(c_begin + 1);
        form_rows(rT, YA, YBs);
        if (c_begin + 1 < c_end) commit(rT2);
        __syncthreads();
        for (int64_t c = c_begin; c < c_end; ++c) {
          const bool odd = ((c - c_begin) & 1) != 0;
          Src* rcur = odd ? rT2 : rT;
          const Src* rnext = odd ? rT : rT2;
          if (c + 2 < c_end) fetch(c + 2);
          mma_chunk(odd ? YA2 : YA, odd ? YB2s : YBs);
          if (c + 1 < c_end) form_rows(rnext, odd ? YA : YA2, odd ? YBs : YB2s);
          if (c + 2 < c_end) commit(rcur);
          __syncthreads();
        }
      } else {
        for (int64_t c = c_begin; c < c_end; ++c) {
          const bool more = c + 1 < c_end;
          if (more) fetch(c + 1);
          form_rows(rT, YA, YBs);
          __syncthreads();
          mma_chunk(YA, YBs);  // then stage the prefetched chunk
          if (more) commit(rT);
          __syncthreads();
        }
      }
    };
    // Kronecker rows of both tiles: y[r][t] = (prod over the outer modes of
    // their factor entries) * q_L[r % R_L][t], rounded once to the operand
    // precision
    bool formed = false;
    if constexpr (V::EPL == 8 && T == 256) {
      if (use4) {
        // BF16 operands, 256 tiles, R_L a multiple of 4, off-diagonal: an
        // item is 4 rows x 4 samples, the 4 rows sharing their outer index
        // (d and the tile origins are multiples of 4, so a row quad is
        // wholly inside or past d), so the outer factors are read and
        // multiplied once per 4 rows.  The products are taken in the same
        // order as below.  Eight consecutive lanes cover one quad's 32
        // samples.  (A diagonal tile forms one side only, which the one-row
        // items below spread over all threads.)
        constexpr int SG = BK / 4;
        constexpr int PER_SIDE = (T / 4) * SG;
        constexpr int ITEMS4 = 2 * PER_SIDE / kSkThreads;
        static_assert(ITEMS4 >= 1 && (2 * PER_SIDE) % kSkThreads == 0 && PER_SIDE % 64 == 0,
                      "items per thread");
        int qo[ITEMS4], qs[ITEMS4], yo[ITEMS4];
        uint64_t pk[ITEMS4];
#pragma unroll
        for (int k = 0; k < ITEMS4; ++k) {
          const int it = tid + k * kSkThreads;
          const int side = it / PER_SIDE, e = it - side * PER_SIDE;
          const int sg = e % SG, rb = e / SG;
          const int64_t r = (side == 0 ? r0 : c0) + 4 * rb;
          const bool in = r < d;
          const int64_t rr = in ? r : d - 1;
          const int oi = static_cast<int>(rr / RL - ob[side]);
          qo[k] = (in ? sl + static_cast<int>(rr % RL) : SR) * kSkRT4 + 4 * sg;
          qs[k] = in ? kSkRT4 : 0;  // past d: the zero row four times
          yo[k] = 4 * rb * LDK + 4 * sg;
          pk[k] = *reinterpret_cast<const uint64_t*>(offs + (side * NO + oi) * kMaxOrder);
        }
        auto form4 = [&](auto nm1, const Src* rs, Op* ya, Op* yb) __attribute__((always_inline)) {
          constexpr int NM1 = decltype(nm1)::value;
#pragma unroll
          for (int k = 0; k < ITEMS4; ++k) {
            const int it = tid + k * kSkThreads;
            const int side = it / PER_SIDE;
            const int t4 = 4 * (it % SG);
            f32x4 o = {1.0f, 1.0f, 1.0f, 1.0f};
#pragma unroll
            for (int m = 0; m < NM1; ++m)
              o *= *reinterpret_cast<const f32x4*>(
                  rs + static_cast<int>((pk[k] >> (8 * m)) & 0xff) * kSkRT4 + t4);
            Op* y = (side == 0 ? ya : yb) + yo[k];
            const Src* qp = rs + qo[k];
            f32x4 q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) q[j] = *reinterpret_cast<const f32x4*>(qp + j * qs[k]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              bf16x4 v;
              v[0] = V::cvt(o.x * q[j].x);
              v[1] = V::cvt(o.y * q[j].y);
              v[2] = V::cvt(o.z * q[j].z);
              v[3] = V::cvt(o.w * q[j].w);
              *reinterpret_cast<bf16x4*>(y + j * LDK) = v;
            }
          }
        };
        run([&](const Src* rs, Op* ya, Op* yb) __attribute__((always_inline)) {
          switch (N) {
            case 1: form4(std::integral_constant<int, 0>{}, rs, ya, yb); break;
            case 2: form4(std::integral_constant<int, 1>{}, rs, ya, yb); break;
            case 3: form4(std::integral_constant<int, 2>{}, rs, ya, yb); break;
            default: form4(std::integral_constant<int, 3>{}, rs, ya, yb); break;
          }
        });
        formed = true;
      }
    }
    if (!formed) {
      // an item is one row x IW samples: outer index within the tile and
      // LDS offset of the last-mode row in rT (the zero row when the design
      // row is past d)
      int oidx[2][ITEMS], iofs_q[2][ITEMS];
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          // consecutive lanes take consecutive rows: conflict-free LDS stores
          const int e = tid + k * kSkThreads;
          const int i = e % T, tg = (e / T) * IW;
          const int64_t r = (side == 0 ? r0 : c0) + i;
          const int64_t rr = r < d ? r : d - 1;
          oidx[side][k] = static_cast<int>(rr / RL - ob[side]);
          iofs_q[side][k] = (r < d ? (sl + static_cast<int>(rr % RL)) : SR) * RT + tg;
        }
      // the rT rows of each item's outer factors (modes other than L), one
      // byte per mode, packed
      uint64_t pk[2][ITEMS];
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
          pk[side][k] = *reinterpret_cast<const uint64_t*>(
              offs + (side * NO + oidx[side][k]) * kMaxOrder);
      auto form = [&](auto nm1, const Src* rs, Op* ya, Op* yb) __attribute__((always_inline)) {
        constexpr int NM1 = decltype(nm1)::value;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (side == 1 && diag) break;
          Op* Y = side == 0 ? ya : yb;
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) {
            const int e = tid + k * kSkThreads;
            const int i = e % T, tg = (e / T) * IW;
            const f32x4* qp = reinterpret_cast<const f32x4*>(rs + iofs_q[side][k]);
            if constexpr (V::EPL == 8) {
              f32x4 o0 = {1.0f, 1.0f, 1.0f, 1.0f}, o1 = o0;
#pragma unroll
              for (int m = 0; m < NM1; ++m) {
                const f32x4* fp = reinterpret_cast<const f32x4*>(
                    rs + static_cast<int>((pk[side][k] >> (8 * m)) & 0xff) * RT + tg);
                o0 *= fp[0];
                o1 *= fp[1];
              }
              const f32x4 q0 = qp[0], q1 = qp[1];
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
              f32x4 o = {1.0f, 1.0f, 1.0f, 1.0f};
#pragma unroll
              for (int m = 0; m < NM1; ++m)
                o *= *reinterpret_cast<const f32x4*>(
                    rs + static_cast<int>((pk[side][k] >> (8 * m)) & 0xff) * RT + tg);
              const f32x4 q = qp[0];
              Op* y = &Y[i * LDK + tg];
              y[0] = V::cvt(o.x * q.x);
              y[1] = V::cvt(o.y * q.y);
              y[2] = V::cvt(o.z * q.z);
              y[3] = V::cvt(o.w * q.w);
            }
          }
        }
      };
      run([&](const Src* rs, Op* ya, Op* yb)
              __attribute__((always_inline)) { by_order(form, rs, ya, yb); });
    }
    typename V::Out* out = slots + (slot0 + seg) * static_cast<int64_t>(T * T);
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
      for (int bb = 0; bb < NBC; ++bb)
#pragma unroll
        for (int v = 0; v < V::NACC; ++v) {
          const int r = wr * WR + a * V::MT + V::acc_row(lane, v);
          const int cc = wc * WC + bb * V::MT + V::acc_col(lane, v);
          out[r * T + cc] = static_cast<typename V::Out>(acc[a][bb][v]);
        }
    ++seg;
    u = pd.unit0 + tau * g.nchunks + c_end;
  }
}

// M[i][j] (i >= j) = sum of the tile's slots + lambda prod_n P_n[i_n][j_n].
// The slots of the (at most kBlock / T) tiles a workgroup's columns touch are
// listed once per workgroup in LDS (the workgroup ranges are found with 64-bit
// divisions, too costly per element); a tile with more than kAsmMaxSlots
// slots is summed by walking the ranges per element instead.
constexpr int kAsmMaxSlots = 16;
constexpr int kAsmRows = 16;  // rows per workgroup (all in one tile row: kAsmRows divides T)
constexpr int kAsmMaxP = 2048;  // P_n entries staged in LDS (sum_n R_n^2)

template <int T>
__global__ __launch_bounds__(kBlock) void assemble_sk_kernel(
    Geom g, int64_t units, int64_t grid, int64_t unit0, int64_t tile0, int64_t nchunks,
    const float* __restrict__ slots, const int64_t* __restrict__ index,
    const double* __restrict__ P, double lambda, double* __restrict__ M) {
  static_assert(T % kAsmRows == 0, "a workgroup's rows share one tile row");
  constexpr int TPB = kBlock >= T ? kBlock / T : 1;  // tiles per workgroup row
  __shared__ int64_t slot_of[TPB][kAsmMaxSlots];
  __shared__ int nslot[TPB];
  __shared__ double Ps[kAsmMaxP];  // the P_n (mode n at roff[n]) when they fit
  const int64_t d = g.d;
  const int64_t jb = static_cast<int64_t>(blockIdx.x) * kBlock;
  const int64_t j = jb + threadIdx.x;
  const int64_t ib = static_cast<int64_t>(blockIdx.y) * kAsmRows;
  const int64_t ilast = (ib + kAsmRows < d ? ib + kAsmRows : d) - 1;
  const int64_t ti = ib / T;
  if (jb > ilast) return;  // the whole workgroup is above the diagonal
  // the slots of the workgroup's tiles, in workgroup order (-1: too many)
  if (threadIdx.x < TPB) {
    const int64_t tj = jb / T + threadIdx.x;
    int n = 0;
    if (tj <= ti) {
      const int64_t tau = ti * (ti + 1) / 2 + tj;
      const int64_t ua = unit0 + tau * nchunks, ub = ua + nchunks;  // the tile's units
      int64_t w = (ua * grid) / units;
      while (w > 0 && sk_unit_start(w, units, grid) > ua) --w;
      while (sk_unit_start(w + 1, units, grid) <= ua) ++w;
      for (; w < grid && sk_unit_start(w, units, grid) < ub; ++w) {
        const int64_t first = index[grid + w];
        if (first < 0) continue;  // empty range
        if (n < kAsmMaxSlots) slot_of[threadIdx.x][n] = index[w] + (tile0 + tau - first);
        ++n;
      }
    }
    nslot[threadIdx.x] = n <= kAsmMaxSlots ? n : -1;
  }
  int np = 0;
  for (int n = 0; n < g.order; ++n) np += g.ranks[n] * g.ranks[n];
  const bool pl = np <= kAsmMaxP;
  if (pl)
    for (int e = threadIdx.x; e < np; e += kBlock) Ps[e] = P[e];
  __syncthreads();
  const double* Pb = pl ? Ps : P;
  const int64_t tj = j / T;
  const int tl = static_cast<int>(tj - jb / T);
  const int ns = nslot[tl];
  // column digits of j, reused for every row
  uint32_t jd[kMaxOrder];
  {
    uint32_t b = static_cast<uint32_t>(j < d ? j : 0);
#pragma unroll
    for (int n = kMaxOrder - 1; n >= 0; --n) {
      const uint32_t R = n < g.order ? static_cast<uint32_t>(g.ranks[n]) : 1u;
      jd[n] = b % R;
      b /= R;
    }
  }
  // lambda prod_n P_n[i_n][j_n] (32-bit digit arithmetic: d < 2^31)
  auto lam_p = [&](int64_t i) __attribute__((always_inline)) {
    double p = 1.0;
    uint32_t a = static_cast<uint32_t>(i);
#pragma unroll
    for (int n = kMaxOrder - 1; n >= 0; --n) {
      if (n < g.order) {
        const uint32_t R = static_cast<uint32_t>(g.ranks[n]);
        p *= Pb[g.roff[n] + (a % R) * R + jd[n]];
        a /= R;
      }
    }
    return p;
  };
  if (ns >= 0) {
    // rows in groups of four (all in one tile row): a slot's four entries
    // are loaded together, and each row's sum keeps the slot order
    static_assert(kAsmRows % 4 == 0, "row groups");
    for (int64_t i0 = ib; i0 <= ilast; i0 += 4) {
      if (j > i0 + 3) continue;  // the group is above the diagonal in column j
      const int64_t off0 = (i0 - ti * T) * T + (j - tj * T);
      double v4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < ns; ++k) {
        const float* sp = slots + slot_of[tl][k] * static_cast<int64_t>(T * T) + off0;
        // rows i0 .. i0 + 3 lie in the slot's T x T tile even past d (i0 % 4
        // == 0 and 4 divides T), so the four loads need no guard
        float x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = sp[r * T];
#pragma unroll
        for (int r = 0; r < 4; ++r) v4[r] += static_cast<double>(x[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + r;
        if (i <= ilast && j <= i) M[i * d + j] = fma(lambda, lam_p(i), v4[r]);
      }
    }
    return;
  }
  // a tile with more slots than the list holds: its ranges are walked per entry
  for (int64_t i = ib; i <= ilast; ++i) {
    if (j > i) continue;
    const int64_t off = (i - ti * T) * T + (j - tj * T);
    const int64_t tau = ti * (ti + 1) / 2 + tj;
    const int64_t ua = unit0 + tau * nchunks, ub = ua + nchunks;
    int64_t w = (ua * grid) / units;
    while (w > 0 && sk_unit_start(w, units, grid) > ua) --w;
    while (sk_unit_start(w + 1, units, grid) <= ua) ++w;
    double v = 0.0;
    for (; w < grid && sk_unit_start(w, units, grid) < ub; ++w) {
      const int64_t first = index[grid + w];
      if (first < 0) continue;
      const int64_t slot = index[w] + (tile0 + tau - first);
      v += static_cast<double>(slots[slot * static_cast<int64_t>(T * T) + off]);
    }
    M[i * d + j] = fma(lambda, lam_p(i), v);
  }
}

// Smallest w with sk_unit_start(w) >= u (grid when there is none).
__device__ inline int64_t sk_first_wg_at(int64_t u, int64_t units, int64_t grid) {
  int64_t w = (u * grid) / units;
  if (w > grid) w = grid;
  while (w > 0 && sk_unit_start(w - 1, units, grid) >= u) --w;
  while (w < grid && sk_unit_start(w, units, grid) < u) ++w;
  return w;
}

// The same sum when a tile collects many slots (few tiles, many workgroups):
// a workgroup of 16 waves takes 64 consecutive j of row i, each wave sums a
// contiguous sixteenth of the tile's contributing workgroups eight slots at a
// time, and the waves' sums are added in wave order (deterministic).
constexpr int kAsmWaves = 16;

template <int T>
__global__ __launch_bounds__(64 * kAsmWaves) void assemble_sk_split_kernel(
    Geom g, int64_t units, int64_t grid, int64_t unit0, int64_t tile0, int64_t nchunks,
    const float* __restrict__ slots, const int64_t* __restrict__ index,
    const double* __restrict__ P, double lambda, double* __restrict__ M) {
  __shared__ double red[kAsmWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t d = g.d;
  const int64_t i = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const bool act = j <= i;
  const int64_t jc = act ? j : i;  // lanes past the diagonal stay inside row i's tile
  const int64_t ti = i / T, tj = jc / T;
  const int64_t tau = ti * (ti + 1) / 2 + tj;
  const int64_t ua = unit0 + tau * nchunks, ub = ua + nchunks;
  const int64_t wlo = sk_first_wg_at(ua + 1, units, grid) - 1;
  const int64_t wend = sk_first_wg_at(ub, units, grid);
  const int64_t n = wend - wlo;
  const int64_t wa = wlo + (n * wave) / kAsmWaves, wb = wlo + (n * (wave + 1)) / kAsmWaves;
  const int64_t off = (i - ti * T) * T + (jc - tj * T);
  constexpr int64_t TT = static_cast<int64_t>(T) * T;
  double v = 0.0;
  int64_t w = wa;
  for (; w + 8 <= wb; w += 8) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t first = index[grid + w + k];
      const int64_t slot = first >= 0 ? index[w + k] + (tile0 + tau - first) : 0;
      const float y = slots[slot * TT + off];
      x[k] = first >= 0 ? y : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v += static_cast<double>(x[k]);
  }
  for (; w < wb; ++w) {
    const int64_t first = index[grid + w];
    if (first < 0) continue;
    v += static_cast<double>(slots[(index[w] + (tile0 + tau - first)) * TT + off]);
  }
  red[wave][lane] = v;
  __syncthreads();
  if (wave != 0 || !act) return;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kAsmWaves; ++k) sum += red[k][lane];
  // lambda prod_n P_n[i_n][j_n] (32-bit digit arithmetic: d < 2^31)
  double p = 1.0;
  uint32_t a = static_cast<uint32_t>(i), b = static_cast<uint32_t>(j);
  for (int nn = g.order - 1; nn >= 0; --nn) {
    const uint32_t R = static_cast<uint32_t>(g.ranks[nn]);
    p *= P[g.roff[nn] + (a % R) * R + (b % R)];
    a /= R;
    b /= R;
  }
  M[i * d + j] = fma(lambda, p, sum);
}

// One tile in the whole launch: every workgroup with units holds exactly one
// slot, in workgroup order, so the tile's slots are 0 .. nslots - 1 and no
// index lookups are needed.  Same split as above (16 waves per 64 entries of
// row i, eight slots in flight per wave, waves added in order).
template <int T>
__global__ __launch_bounds__(64 * kAsmWaves) void assemble_sk_one_tile_kernel(
    Geom g, int64_t nslots, const float* __restrict__ slots, const double* __restrict__ P,
    double lambda, double* __restrict__ M) {
  __shared__ double red[kAsmWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t d = g.d;
  const int64_t i = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const bool act = j <= i;
  const int64_t off = i * T + (act ? j : i);
  constexpr int64_t TT = static_cast<int64_t>(T) * T;
  const int64_t wa = (nslots * wave) / kAsmWaves, wb = (nslots * (wave + 1)) / kAsmWaves;
  double v = 0.0;
  int64_t w = wa;
  for (; w + 8 <= wb; w += 8) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = slots[(w + k) * TT + off];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += static_cast<double>(x[k]);
  }
  for (; w < wb; ++w) v += static_cast<double>(slots[w * TT + off]);
  red[wave][lane] = v;
  __syncthreads();
  if (wave != 0 || !act) return;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kAsmWaves; ++k) sum += red[k][lane];
  // lambda prod_n P_n[i_n][j_n] (32-bit digit arithmetic: d < 2^31)
  double p = 1.0;
  uint32_t a = static_cast<uint32_t>(i), b = static_cast<uint32_t>(j);
  for (int nn = g.order - 1; nn >= 0; --nn) {
    const uint32_t R = static_cast<uint32_t>(g.ranks[nn]);
    p *= P[g.roff[nn] + (a % R) * R + (b % R)];
    a /= R;
    b /= R;
  }
  M[i * d + j] = fma(lambda, p, sum);
}

template <class V, int T, int PF4, bool DB>
void gram_sk_launch_k(const SkBatch& b, float* slots, const int64_t* index, hipStream_t st) {
  const size_t lds = SkLayout<V, T, DB ? 2 : 1>::bytes(b.max_sum_r);
  if (lds > 64 * 1024)
    ensure_dyn_lds(reinterpret_cast<const void*>(&gram_sk_kernel<V, T, PF4, DB>),
                   static_cast<int>(kSkMaxLds));
  hipLaunchKernelGGL((gram_sk_kernel<V, T, PF4, DB>), dim3(static_cast<unsigned>(b.grid)),
                     dim3(SkTile<T>::THREADS), lds, st, b, slots, index);
}

// The double-buffered loop for the one-workgroup-per-CU 256 tile when both
// sets fit in LDS; the single-buffered one otherwise (and for the smaller
// tiles, whose several workgroups per CU already overlap formation and MFMA).
template <class V, int T>
void gram_sk_launch(const SkBatch& b, float* slots, const int64_t* index, hipStream_t st) {
  using Pf = SkPf<SkTile<T>::THREADS>;
  if constexpr (T == 256) {
    if (SkLayout<V, T, 2>::bytes(b.max_sum_r) <= kSkMaxLds) {
      if (Pf::small(b.max_sum_r)) gram_sk_launch_k<V, T, Pf::SMALL, true>(b, slots, index, st);
      else gram_sk_launch_k<V, T, Pf::LARGE, true>(b, slots, index, st);
      return;
    }
  }
  if (Pf::small(b.max_sum_r)) gram_sk_launch_k<V, T, Pf::SMALL, false>(b, slots, index, st);
  else gram_sk_launch_k<V, T, Pf::LARGE, false>(b, slots, index, st);
}


}  // namespace

#ifndef TK_SK_BIG_TILE_D
#define TK_SK_BIG_TILE_D 2048
#endif

SkConfig sk_default_config(int64_t d) {
  // the 256 tile halves the row formation per MFMA once there are enough
  // tiles to spread over the CUs
  if (d >= TK_SK_BIG_TILE_D) return SkConfig{256, SkTile<256>::WG_PER_CU};
  // a single 64 tile covers the whole Gram: no padding rows
  if (d <= 64) return SkConfig{64, SkTile<64>::WG_PER_CU};
  return SkConfig{128, SkTile<128>::WG_PER_CU};
}

bool sk_config_valid(const SkConfig& c) {
  return (c.tile == 64 || c.tile == 128 || c.tile == 256) && c.wg_per_cu >= 1 &&
         c.wg_per_cu <= 8;
}

SkProb sk_prob(const Geom& g, int64_t s, const float* rows32) {
  SkProb q;
  memset(&q, 0, sizeof(q));
  q.rows = rows32;
  q.s = static_cast<int32_t>(s);
  q.order = static_cast<uint8_t>(g.order);
  q.last = static_cast<uint8_t>(g.last);
  q.sum_r = static_cast<uint8_t>(g.sum_r);
  for (int n = 0; n < g.order; ++n) q.ranks[n] = static_cast<uint8_t>(g.ranks[n]);
  return q;
}

void sk_finalize(SkBatch& b, tk_dtype prec, const SkConfig& cfg) {
  b.tile = cfg.tile;
  b.prec = prec;
  int64_t units = 0, tiles = 0;
  int msr = 1;
  for (int k = 0; k < b.count; ++k) {
    SkProb& q = b.p[k];
    int64_t d = 1;
    for (int n = 0; n < q.order; ++n) d *= q.ranks[n];
    const int64_t nt = cdiv(d, cfg.tile);
    const int64_t nti = nt * (nt + 1) / 2;
    q.unit0 = units;
    q.tile0 = tiles;
    units += nti * row_chunks(q.s);
    tiles += nti;
    if (q.sum_r > msr) msr = q.sum_r;
  }
  b.units = units;
  b.tiles = tiles;
  b.max_sum_r = msr;
  int64_t G = static_cast<int64_t>(cfg.wg_per_cu) * device_cu_count();
  if (G > units) G = units;
  if (G < 1) G = 1;
  b.grid = G;
}

size_t sk_slot_bytes(const SkBatch& b) {
  // every workgroup writes one slot per tile its range touches: at most
  // grid + tiles slots in all
  return static_cast<size_t>(b.grid + b.tiles) * b.tile * b.tile * sizeof(float);
}

size_t sk_index_bytes(const SkBatch& b) { return static_cast<size_t>(2 * b.grid) * 8; }

void launch_gram_sk(const SkBatch& b, float* slots, int64_t* index, hipStream_t st) {
  if (b.count < 1 || b.units < 1) return;
  hipLaunchKernelGGL(sk_index_kernel, dim3(1), dim3(1024), 0, st, b, index);
  const bool bf = b.prec == TK_BF16;
  if (b.tile == 256) {
    if (bf) gram_sk_launch<VarBF16, 256>(b, slots, index, st);
    else gram_sk_launch<VarF32, 256>(b, slots, index, st);
  } else if (b.tile == 128) {
    if (bf) gram_sk_launch<VarBF16, 128>(b, slots, index, st);
    else gram_sk_launch<VarF32, 128>(b, slots, index, st);
  } else {
    if (bf) gram_sk_launch<VarBF16, 64>(b, slots, index, st);
    else gram_sk_launch<VarF32, 64>(b, slots, index, st);
  }
}

void launch_assemble_sk(const SkBatch& b, int k, const Geom& g, const float* slots,
                        const int64_t* index, const double* P, double lambda, double* M,
                        hipStream_t st) {
  const SkProb& q = b.p[k];
  const int64_t nch = row_chunks(q.s);
  if (b.tiles == 1 && b.count == 1) {
    // a single tile: the workgroups with units hold slots 0 .. min(grid, units) - 1
    const int64_t nslots = b.units < b.grid ? b.units : b.grid;
    const dim3 grid(static_cast<unsigned>(cdiv(g.d, 64)), static_cast<unsigned>(g.d));
    const dim3 block(64 * kAsmWaves);
    if (b.tile == 256)
      hipLaunchKernelGGL(assemble_sk_one_tile_kernel<256>, grid, block, 0, st, g, nslots, slots, P,
                         lambda, M);
    else if (b.tile == 128)
      hipLaunchKernelGGL(assemble_sk_one_tile_kernel<128>, grid, block, 0, st, g, nslots, slots, P,
                         lambda, M);
    else
      hipLaunchKernelGGL(assemble_sk_one_tile_kernel<64>, grid, block, 0, st, g, nslots, slots, P,
                         lambda, M);
    return;
  }
  if (b.grid >= 8 * b.tiles) {
    // many slots per tile: split each element's sum over 16 waves
    const dim3 grid(static_cast<unsigned>(cdiv(g.d, 64)), static_cast<unsigned>(g.d));
    const dim3 block(64 * kAsmWaves);
    if (b.tile == 256)
      hipLaunchKernelGGL(assemble_sk_split_kernel<256>, grid, block, 0, st, g, b.units, b.grid,
                         q.unit0, q.tile0, nch, slots, index, P, lambda, M);
    else if (b.tile == 128)
      hipLaunchKernelGGL(assemble_sk_split_kernel<128>, grid, block, 0, st, g, b.units, b.grid,
                         q.unit0, q.tile0, nch, slots, index, P, lambda, M);
    else
      hipLaunchKernelGGL(assemble_sk_split_kernel<64>, grid, block, 0, st, g, b.units, b.grid,
                         q.unit0, q.tile0, nch, slots, index, P, lambda, M);
    return;
  }
  const dim3 grid(static_cast<unsigned>(cdiv(g.d, kBlock)),
                  static_cast<unsigned>(cdiv(g.d, kAsmRows)));
  if (b.tile == 256)
    hipLaunchKernelGGL(assemble_sk_kernel<256>, grid, dim3(kBlock), 0, st, g, b.units, b.grid,
                       q.unit0, q.tile0, nch, slots, index, P, lambda, M);
  else if (b.tile == 128)
    hipLaunchKernelGGL(assemble_sk_kernel<128>, grid, dim3(kBlock), 0, st, g, b.units, b.grid,
                       q.unit0, q.tile0, nch, slots, index, P, lambda, M);
  else
    hipLaunchKernelGGL(assemble_sk_kernel<64>, grid, dim3(kBlock), 0, st, g, b.units, b.grid,
                       q.unit0, q.tile0, nch, slots, index, P, lambda, M);
}

}  // namespace tk
