// Factor update over the observed entries only (Alg. 2 factor step restricted
// to the observed entries, the tensor completion setting of Sec. 4.2): row i
// of A(n) solves
//   a_i = argmin_y sum_{j observed in row i} (x_(n),ij - y . k_j)^2 + lambda ||y||^2,
// k_j the column j of K_n = G_(n) ((x)_{m != n} A(m))^T, so every row has its
// own R_n x R_n Gram  sum_{j obs} k_j k_j^T  and right side  sum_{j obs} x_ij k_j.
//
// Layout of the pass.  Besides n, one "inner" mode J is singled out: the last
// mode, or the one before it when n is the last.  The remaining modes form the
// outer index o.  For fixed o the design column of entry (o, i, j) is
//   k_{o,j} = T_o a_J(j),   T_o[r][c] = sum_{c'} G[r at n, c at J, c' elsewhere] z_o[c'],
//   z_o[c'] = prod_{m outer} A(m)[o_m][c'_m],
// shared by every row i.  A workgroup owns a block of rows and a range of
// outer indices; per o it forms T_o, then per tile of kJt inner indices the
// design columns (in LDS) and the tile of X and of the mask for its rows, and
// accumulates the rows' Gram and right-side entries in registers.  The work
// of a row is split into items of 4 x 4 Gram entries (tile pairs rt >= st of
// 4 ranks each) and items of 4 right-side entries; thread = (item, row).  Each
// workgroup writes one partial per (row, item); the solve kernel adds them in
// workgroup order (deterministic), adds lambda I and solves by Cholesky in
// FP64.
#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kJt = 32;         // inner indices per tile
constexpr int kZChunk = 2048;   // outer-product entries staged in LDS at a time
constexpr int kMfuMaxThreads = 1024;
constexpr int kTSlots = 8;      // entries of T_o per thread (R_n R_J <= kTSlots * threads)

struct MfuGeom {
  const double* A64;        // FP64 factors, I_m x R_m rows at qoff[m]
  const double* Gp;         // core permuted to [R_n][R_J][outer ranks, row-major]
  const void* X;
  const uint32_t* mask;
  int32_t dt;               // TK_F64 or TK_F32
  int32_t Rn, RJ, T, RB;    // ranks; T = ceil(R_n / 4) rank tiles, RB = 4 T
  int32_t items, rows_blk;  // items per row, rows per workgroup
  int32_t gram_items;       // T (T + 1) / 2 Gram items precede the T right-side items
  int32_t nout;             // number of outer modes
  int32_t dprime;           // prod of the outer ranks
  int32_t inner_contig;     // 1: stride_J == 1 (n is not the last mode)
  int64_t In, IJ, O;        // rows, inner size, outer indices
  int64_t stride_n, stride_J;
  int64_t qoffJ;
  int64_t odim[kMaxOrder];
  int64_t ostride[kMaxOrder];
  int64_t oqoff[kMaxOrder];
  int32_t orank[kMaxOrder];
  int32_t groups;           // workgroups along the outer indices
};

__device__ inline void item_tiles(int item, int gram_items, int T, int& rt, int& st, bool& rhs) {
  if (item >= gram_items) {
    rhs = true;
    rt = item - gram_items;
    st = 0;
    return;
  }
  rhs = false;
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= item) ++r;  // tile pairs (r, s), s <= r, row-major
  rt = r;
  st = item - r * (r + 1) / 2;
  (void)T;
}

__global__ __launch_bounds__(kMfuMaxThreads) void mfu_accum_kernel(MfuGeom p, double* part) {
  extern __shared__ double sm[];
  const int ldr = p.rows_blk + 1;         // padded row stride of the X / mask tiles
  double* xs = sm;                        // [kJt][ldr]  m_ij x_ij
  double* ws = xs + kJt * ldr;            // [kJt][ldr]  m_ij
  double* ks = ws + kJt * ldr;            // [kJt][RB]   design columns, ranks >= R_n zero
  double* To = ks + kJt * p.RB;           // [R_n][R_J]
  double* zs = To + p.Rn * p.RJ;          // [kZChunk]   outer products z_o

  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int item = tid / p.rows_blk;
  const int rl = tid % p.rows_blk;
  const bool active = item < p.items;
  int rt = 0, st = 0;
  bool is_rhs = false;
  if (active) item_tiles(item, p.gram_items, p.T, rt, st, is_rhs);

  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * p.rows_blk;
  const int nrows = static_cast<int>(min(static_cast<int64_t>(p.rows_blk), p.In - i0));
  const int64_t o_beg = p.O * blockIdx.x / p.groups;
  const int64_t o_end = p.O * (blockIdx.x + 1) / p.groups;
  const int RnRJ = p.Rn * p.RJ;

  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;

  __shared__ int64_t s_rowoff[kMaxOrder];  // A64 offset of the outer modes' rows of o
  __shared__ int64_t s_base;               // X offset of (o, 0, 0)
  for (int64_t o = o_beg; o < o_end; ++o) {
    if (tid == 0) {
      int64_t rem = o, base = 0;
      for (int q = p.nout - 1; q >= 0; --q) {
        const int64_t dig = rem % p.odim[q];
        rem /= p.odim[q];
        s_rowoff[q] = p.oqoff[q] + dig * p.orank[q];
        base += dig * p.ostride[q];
      }
      s_base = base;
    }
    __syncthreads();
    const int64_t base = s_base;
    // T_o = Gp (x) z_o, z_o staged in chunks; thread e owns entries e, e + nthreads, ...
    double tacc[kTSlots];  // entries tid + u nthreads, u < kTSlots (RnRJ <= kTSlots nthreads)
#pragma unroll
    for (int u = 0; u < kTSlots; ++u) tacc[u] = 0.0;
    for (int c0 = 0; c0 < p.dprime; c0 += kZChunk) {
      const int cn = min(kZChunk, p.dprime - c0);
      for (int c = tid; c < cn; c += nthreads) {
        int rem = c0 + c;
        double z = 1.0;
        for (int q = p.nout - 1; q >= 0; --q) {
          const int dig = rem % p.orank[q];
          rem /= p.orank[q];
          z *= p.A64[s_rowoff[q] + dig];
        }
        zs[c] = z;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kTSlots; ++u) {
        const int e = tid + u * nthreads;
        if (e < RnRJ) {
          const double* g = p.Gp + static_cast<int64_t>(e) * p.dprime + c0;
          double s = tacc[u];
          for (int c = 0; c < cn; ++c) s = fma(g[c], zs[c], s);
          tacc[u] = s;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kTSlots; ++u) {
      const int e = tid + u * nthreads;
      if (e < RnRJ) To[e] = tacc[u];
    }
    __syncthreads();

    for (int64_t j0 = 0; j0 < p.IJ; j0 += kJt) {
      const int nj = static_cast<int>(min(static_cast<int64_t>(kJt), p.IJ - j0));
      // design columns k[jj][r] = sum_c To[r][c] a_J(j0 + jj)[c]
      for (int e = tid; e < kJt * p.RB; e += nthreads) {
        const int jj = e / p.RB, r = e % p.RB;
        double s = 0.0;
        if (jj < nj && r < p.Rn) {
          const double* aj = p.A64 + p.qoffJ + (j0 + jj) * p.RJ;
          const double* tr = To + r * p.RJ;
          for (int c = 0; c < p.RJ; ++c) s = fma(tr[c], aj[c], s);
        }
        ks[e] = s;
      }
      // X and mask tile of the block's rows, loaded along X's contiguous index
      for (int e = tid; e < kJt * p.rows_blk; e += nthreads) {
        int jj, r;
        if (p.inner_contig) {
          jj = e % kJt;
          r = e / kJt;
        } else {
          r = e % p.rows_blk;
          jj = e / p.rows_blk;
        }
        double xv = 0.0, wv = 0.0;
        if (jj < nj && r < nrows) {
          const int64_t f = base + (i0 + r) * p.stride_n + (j0 + jj) * p.stride_J;
          const bool obs = ((p.mask[f >> 5] >> (f & 31)) & 1u) != 0u;
          if (obs) {
            xv = p.dt == TK_F64 ? static_cast<const double*>(p.X)[f]
                                : static_cast<double>(static_cast<const float*>(p.X)[f]);
            wv = 1.0;
          }
        }
        xs[jj * ldr + r] = xv;
        ws[jj * ldr + r] = wv;
      }
      __syncthreads();
      if (active && rl < nrows) {
        if (is_rhs) {
          for (int jj = 0; jj < nj; ++jj) {
            const double xv = xs[jj * ldr + rl];
            const double* kr = ks + jj * p.RB + 4 * rt;
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = fma(xv, kr[a], acc[a]);
          }
        } else {
          for (int jj = 0; jj < nj; ++jj) {
            const double wv = ws[jj * ldr + rl];
            const double* kr = ks + jj * p.RB + 4 * rt;
            const double* kc = ks + jj * p.RB + 4 * st;
            double ka[4], kb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              ka[a] = wv * kr[a];
              kb[a] = kc[a];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a * 4 + b] = fma(ka[a], kb[b], acc[a * 4 + b]);
          }
        }
      }
      __syncthreads();
    }
  }
  if (active && rl < nrows) {
    double* dst = part + ((static_cast<int64_t>(blockIdx.x) * p.In + i0 + rl) * p.items + item) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[e] = acc[e];
  }
}

// Row i: the Gram and right side from the partials (added in workgroup order),
// plus lambda I, FP64 Cholesky and the two triangular solves; one wave per row.
template <class OutT>
__global__ __launch_bounds__(64) void mfu_solve_kernel(const double* __restrict__ part, int groups,
                                                        int64_t In, int Rn, int T, int items,
                                                        int gram_items, double lambda,
                                                        OutT* __restrict__ out, int32_t* status) {
  __shared__ double Lm[kMaxRank * kMaxRank];
  __shared__ double b[kMaxRank];
  __shared__ int bad;
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane == 0) bad = 0;
  for (int v = lane; v < items * 16; v += 64) {
    double s = 0.0;
    for (int g = 0; g < groups; ++g) s += part[((static_cast<int64_t>(g) * In + i) * items) * 16 + v];
    const int item = v / 16, e = v % 16, a = e / 4, c = e % 4;
    if (item >= gram_items) {  // right-side item: entries 0..3 are rows 4 rt + e
      const int r = 4 * (item - gram_items) + e;
      if (e < 4 && r < Rn) b[r] = s;
    } else {
      int rt = 0;
      while ((rt + 1) * (rt + 2) / 2 <= item) ++rt;
      const int st = item - rt * (rt + 1) / 2;
      const int r = 4 * rt + a, q = 4 * st + c;
      if (r < Rn && q < Rn && q <= r) Lm[r * Rn + q] = s + (r == q ? lambda : 0.0);
    }
  }
  (void)T;
  __syncthreads();
  // lower Cholesky in place (entries q <= r)
  for (int j = 0; j < Rn; ++j) {
    if (lane == 0) {
      double piv = Lm[j * Rn + j];
      if (!(piv > 0.0)) {
        bad = 1;
        piv = 1.0;
      }
      Lm[j * Rn + j] = sqrt(piv);
    }
    __syncthreads();
    const double ljj = Lm[j * Rn + j];
    for (int r = j + 1 + lane; r < Rn; r += 64) Lm[r * Rn + j] /= ljj;
    __syncthreads();
    for (int r = j + 1 + lane; r < Rn; r += 64) {
      const double lr = Lm[r * Rn + j];
      for (int q = j + 1; q <= r; ++q) Lm[r * Rn + q] = fma(-lr, Lm[q * Rn + j], Lm[r * Rn + q]);
    }
    __syncthreads();
  }
  if (lane == 0) {
    if (bad) atomicMax(status, static_cast<int32_t>(TK_E_NOT_SPD));
    for (int a = 0; a < Rn; ++a) {
      double s = b[a];
      for (int c = 0; c < a; ++c) s = fma(-Lm[a * Rn + c], b[c], s);
      b[a] = s / Lm[a * Rn + a];
    }
    for (int a = Rn - 1; a >= 0; --a) {
      double s = b[a];
      for (int c = a + 1; c < Rn; ++c) s = fma(-Lm[c * Rn + a], b[c], s);
      b[a] = s / Lm[a * Rn + a];
    }
  }
  __syncthreads();
  for (int a = lane; a < Rn; a += 64) out[i * Rn + a] = static_cast<OutT>(b[a]);
}

// Strides of the core's outer modes, in increasing mode order.
struct OuterCore {
  int32_t nout, dprime, RJ;
  int32_t rank[kMaxOrder];
  int64_t stride[kMaxOrder];
};

// Gp[r][c][c'] = G[digits: r at mode n, c at mode J, c' over the outer modes
// in increasing mode order, row-major].
__global__ void mfu_permute_core_kernel(const double* __restrict__ G64, int64_t d, OuterCore oc,
                                        int64_t nstride, int64_t Jstride,
                                        double* __restrict__ Gp) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d) return;
  int64_t rem = e;
  int64_t cp = rem % oc.dprime;
  rem /= oc.dprime;
  const int64_t c = rem % oc.RJ;
  const int64_t r = rem / oc.RJ;
  int64_t src = r * nstride + c * Jstride;
  for (int k = oc.nout - 1; k >= 0; --k) {
    src += (cp % oc.rank[k]) * oc.stride[k];
    cp /= oc.rank[k];
  }
  Gp[e] = G64[src];
}

struct MfuPlan {
  MfuGeom g;
  int threads;
  size_t lds;
};

MfuPlan plan_mfu(const Geom& g, int n) {
  MfuPlan pl;
  MfuGeom& p = pl.g;
  p = MfuGeom{};
  const int L = g.order - 1;
  const int J = n < L ? L : L - 1;
  p.Rn = g.ranks[n];
  p.RJ = g.ranks[J];
  p.T = (p.Rn + 3) / 4;
  p.RB = 4 * p.T;
  p.gram_items = p.T * (p.T + 1) / 2;
  p.items = p.gram_items + p.T;
  int rows = 64;
  while (rows > 1 && rows * p.items > kMfuMaxThreads) rows /= 2;
  p.rows_blk = rows;
  p.In = g.dims[n];
  p.IJ = g.dims[J];
  p.O = g.numel / (p.In * p.IJ);
  p.stride_n = g.strides[n];
  p.stride_J = g.strides[J];
  p.inner_contig = p.stride_J == 1 ? 1 : 0;
  p.qoffJ = g.qoff[J];
  p.nout = 0;
  p.dprime = 1;
  for (int m = 0; m < g.order; ++m) {
    if (m == n || m == J) continue;
    p.odim[p.nout] = g.dims[m];
    p.ostride[p.nout] = g.strides[m];
    p.oqoff[p.nout] = g.qoff[m];
    p.orank[p.nout] = g.ranks[m];
    p.dprime *= g.ranks[m];
    ++p.nout;
  }
  const int64_t row_blocks = cdiv(p.In, p.rows_blk);
  int64_t groups = 512 / row_blocks;
  if (groups < 1) groups = 1;
  if (groups > p.O) groups = p.O;
  p.groups = static_cast<int32_t>(groups);
  const int t = p.rows_blk * p.items;
  pl.threads = static_cast<int>(cdiv(t, 64) * 64);
  pl.lds = sizeof(double) * (2 * static_cast<size_t>(kJt) * (p.rows_blk + 1) +
                             static_cast<size_t>(kJt) * p.RB + p.Rn * p.RJ + kZChunk);
  return pl;
}

}  // namespace

bool factor_masked_ok(const Geom& g) { return g.order >= 2; }

size_t factor_masked_bytes(const Geom& g) {
  size_t mx = 0;
  for (int n = 0; n < g.order; ++n) {
    const MfuPlan pl = plan_mfu(g, n);
    const size_t b = static_cast<size_t>(pl.g.groups) * pl.g.In * pl.g.items * 16 * sizeof(double);
    mx = b > mx ? b : mx;
  }
  return mx + static_cast<size_t>(g.d) * sizeof(double) + 256;
}

void launch_factor_masked(const Geom& g, int n, const void* X, tk_dtype dt, const uint32_t* mask,
                          const double* A64, const double* G64, double lambda, void* out,
                          int32_t* status, void* scratch, hipStream_t st) {
  MfuPlan pl = plan_mfu(g, n);
  MfuGeom& p = pl.g;
  double* Gp = static_cast<double*>(scratch);
  double* part = Gp + ((g.d + 31) & ~int64_t(31));
  p.A64 = A64;
  p.Gp = Gp;
  p.X = X;
  p.mask = mask;
  p.dt = dt;
  const int L = g.order - 1;
  const int J = n < L ? L : L - 1;
  // core strides (row-major over the ranks)
  int64_t cs[kMaxOrder];
  int64_t acc = 1;
  for (int m = g.order - 1; m >= 0; --m) {
    cs[m] = acc;
    acc *= g.ranks[m];
  }
  OuterCore oc;
  oc.nout = p.nout;
  oc.dprime = p.dprime;
  oc.RJ = p.RJ;
  int k = 0;
  for (int m = 0; m < g.order; ++m)
    if (m != n && m != J) {
      oc.rank[k] = g.ranks[m];
      oc.stride[k] = cs[m];
      ++k;
    }
  hipLaunchKernelGGL(mfu_permute_core_kernel, dim3(static_cast<unsigned>(cdiv(g.d, kBlock))),
                     dim3(kBlock), 0, st, G64, g.d, oc, cs[n], cs[J], Gp);
  ensure_dyn_lds(reinterpret_cast<const void*>(mfu_accum_kernel), static_cast<int>(pl.lds));
  const unsigned row_blocks = static_cast<unsigned>(cdiv(p.In, p.rows_blk));
  hipLaunchKernelGGL(mfu_accum_kernel, dim3(p.groups, row_blocks), dim3(pl.threads), pl.lds, st, p,
                     part);
  if (dt == TK_F64)
    hipLaunchKernelGGL(mfu_solve_kernel<double>, dim3(static_cast<unsigned>(p.In)), dim3(64), 0, st,
                       part, p.groups, p.In, p.Rn, p.T, p.items, p.gram_items, lambda,
                       static_cast<double*>(out), status);
  else
    hipLaunchKernelGGL(mfu_solve_kernel<float>, dim3(static_cast<unsigned>(p.In)), dim3(64), 0, st,
                       part, p.groups, p.In, p.Rn, p.T, p.items, p.gram_items, lambda,
                       static_cast<float*>(out), status);
}

}  // namespace tk
