// Internal declarations of the gfx950 HIP library behind include/tucker.h.
// Device helpers, kernel launch wrappers and the workspace carving shared by
// the entry points in tk_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "tucker.h"

namespace tk {

constexpr int kMaxOrder = TK_MAX_ORDER;
constexpr int kMaxRank = TK_MAX_RANK;
constexpr int kBlock = 256;

// Problem geometry passed by value to kernels.
struct Geom {
  int32_t order;
  int32_t ranks[kMaxOrder];
  int64_t dims[kMaxOrder];
  int64_t strides[kMaxOrder];   // row-major element strides of X
  int64_t off[kMaxOrder];       // offsets of mode n in concatenated per-mode arrays
  int64_t qoff[kMaxOrder];      // offsets of mode n in concatenated I_n x R_n row arrays
  int64_t roff[kMaxOrder];      // offsets of mode n in concatenated R_n x R_n arrays
  int64_t total_rows;           // sum I_n
  int64_t total_q;              // sum I_n R_n
  int64_t total_rr;             // sum R_n^2
  int64_t numel;                // prod I_n
  int64_t d;                    // prod R_n
  int32_t soff[kMaxOrder];      // offsets of mode n inside a concatenated sample row (sum R_m)
  int32_t sum_r;                // sum R_n: length of a concatenated sample row
  int32_t last;                 // split mode: the last mode with R_n >= 2 (N-1 when d == 1)
};

constexpr int kMaxSumR = 160;   // longest concatenated sample row the kernels stage in LDS
// Pre-gathered sample rows are stored chunk-transposed: chunk c of kRowChunk
// samples holds element (sample t, row position j) at
// c * sum_r * kRowChunk + j * kRowChunk + (t - c * kRowChunk); padding samples are 0.
constexpr int kRowChunk = 32;

Geom make_geom(const tk_problem* p);

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Carver {
  char* base;
  size_t used;
  explicit Carver(void* b) : base(static_cast<char*>(b)), used(0) {}
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* r = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return r;
  }
};

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; all enqueue on `st` and never synchronise)

// Leverage scores / tables / whitening (tk_leverage.hip).
// L, Linv and P (= (L^T L)^{-1}) per mode at geom.roff; Q64 / Q32 whitened rows
// at geom.qoff; scores and cdf at geom.off.
// qbits: fixed-point bits Q of the integer sampling weights ceil(l 2^Q).
void launch_leverage(const Geom& g, const void* const* factors, tk_dtype dt, double* scores,
                     uint64_t* cdf, double* L, double* Linv, double* P, double* Q64, float* Q32,
                     int32_t* status, hipStream_t st, int qbits = TK_Q_BITS);

// Rows times a per-mode R_n x R_n FP64 matrix M (at geom.roff):
// out[i][c] = sum_k A(n)[i][k] M[k][c], or M transposed when trans != 0; out64
// (and out32 unless null) at geom.qoff.  With weights != null also the row
// scores ||out[i]||^2 (into scores unless null) and their integer weights, both
// at geom.off.
void launch_mode_rows(const Geom& g, const void* const* factors, tk_dtype dt, const double* M,
                      int trans, double* out64, float* out32, double* scores, uint64_t* weights,
                      hipStream_t st, int qbits = TK_Q_BITS);

// Sampler (tk_sample.hip).
// aug != 0: augmented draws over [K; sqrt(lambda) I] with ridge branch weight
// coin_c against the data branch's 2^qbits (tk_sample.hip); g.ranks and g.d
// give the ridge rows' digits.
void launch_sample(const Geom& g, const uint64_t* cdf, int64_t s, uint64_t seed, uint64_t counter,
                   uint64_t problem, int32_t* idx, double* weight, hipStream_t st, int aug = 0,
                   uint64_t coin_c = 0, int qbits = TK_Q_BITS);

// Ridge-score mixture of K (tk_leverage.hip, tk_sample.hip): from the
// eigenpairs of eig_modes (lamm[n * 64 + c], W_n = A(n) V_n rows at qoff) the
// tuple CDF [d] and the column CDFs (mode n column c at qoff[n] + c I_n),
// d_eff = sum_t pi_t (device double); then draws from the mixture (with the
// augmented coin when aug != 0), weights 1/(s P).
void launch_ridge_tables(const Geom& g, const double* lamm, const double* W, double lambda,
                         uint64_t* tcdf, uint64_t* ccdf, double* deff, hipStream_t st,
                         int qbits = TK_Q_BITS);
void launch_sample_ridge(const Geom& g, const uint64_t* tcdf, const uint64_t* ccdf, int64_t s,
                         uint64_t seed, uint64_t counter, uint64_t problem, int32_t* idx,
                         double* weight, hipStream_t st, int aug = 0, uint64_t coin_c = 0,
                         int qbits = TK_Q_BITS);

// Whitened row tables of the augmented design (tk_leverage.hip): in the
// geometry ga (dims I_n + R_n), rows i < I_n of mode n copy Q64's rows and
// row I_n + k is column k of L_n^{-1}, times sqrt(lambda) in mode 0, so that
// the Kronecker row of ridge draw (I_n + k_n)_n is sqrt(lambda) W e_k.
void launch_aug_tables(const Geom& g, const Geom& ga, const double* Q64, const double* Linv,
                       double lambda, double* Q64a, hipStream_t st);

// Per-sample factor rows (chunk-transposed, see kRowChunk): q^(n)_{i_n}[r] at row
// position soff_n + r; rows32 the same in FP32 with mode 0 scaled by sqrt(weff_t).
__host__ __device__ inline int64_t row_chunks(int64_t s) { return (s + kRowChunk - 1) / kRowChunk; }
void launch_pregather(const Geom& g, const int32_t* idx, const double* weff, int64_t s,
                      const double* Q64, double* rows64, float* rows32, hipStream_t st);

// Gather x_t and mask bits: weff_t = w_t [obs], xw_t = w_t x_t [obs].
// ridge != 0: draws with every i_n in [I_n, I_n + R_n) are ridge rows
// (x_t = 0, always observed).
void launch_gather(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                   const int32_t* idx, const double* weight, int64_t s, double* weff, double* xw,
                   unsigned int* missing, int32_t* status, hipStream_t st, int ridge = 0);

// Sketched Gram of whitened rows (tk_gram.hip).  FP64: partial Grams per
// sample split (64 x 64 tiles).  FP32 / BF16: stream-K over 256 x 256 tiles
// with partial tiles in per-workgroup slots.
// Stream-K Gram (tk_gram_sk.hip).  One launch computes the sketched Grams of
// up to kSkMaxBatch problems: the (lower-triangular tile, 32-sample chunk)
// units of all problems are laid out problem by problem and tile by tile, and
// workgroup w of `grid` walks units [w U / grid, (w + 1) U / grid).
constexpr int kSkMaxBatch = 64;
struct SkProb {
  const float* rows;  // chunk-transposed f32 sample rows, sqrt(weight) folded into mode 0
  int64_t unit0;      // first unit of the problem in the launch
  int64_t tile0;      // first tile of the problem (tile numbering over the launch)
  int32_t s;          // samples
  uint8_t order, last, sum_r, pad;
  uint8_t ranks[kMaxOrder];
};
struct SkBatch {
  int32_t count;
  int32_t tile;       // output tile edge T: 64 or 128
  int32_t prec;       // TK_F32 or TK_BF16
  int32_t max_sum_r;
  int64_t units, grid, tiles;
  SkProb p[kSkMaxBatch];
};
// The knobs of a stream-K launch chosen by the batched call's tuner.
struct SkConfig {
  int32_t tile;       // 64 or 128
  int32_t wg_per_cu;  // workgroups per compute unit of the persistent grid
};
SkProb sk_prob(const Geom& g, int64_t s, const float* rows32);
// Fills unit0 / tile0 of every problem and the launch totals from cfg.
void sk_finalize(SkBatch& b, tk_dtype prec, const SkConfig& cfg);
size_t sk_slot_bytes(const SkBatch& b);   // partial tiles
size_t sk_index_bytes(const SkBatch& b);  // per-workgroup slot bases and first tiles
// Index kernel plus the persistent Gram kernel.
void launch_gram_sk(const SkBatch& b, float* slots, int64_t* index, hipStream_t st);
// M (d x d lower triangle, FP64) = sum of problem k's partial tiles + lambda P.
void launch_assemble_sk(const SkBatch& b, int k, const Geom& g, const float* slots,
                        const int64_t* index, const double* P, double lambda, double* M,
                        hipStream_t st);
bool sk_config_valid(const SkConfig& c);
// Tile and grid of a single problem's stream-K Gram.
SkConfig sk_default_config(int64_t d);

// Grouped FP64 Gram (tk_gram_grouped.hip): with L = geom.last the samples
// are grouped by i_L and G = sum_k B_k (x) e_k e_k^T (B_k over the group's
// rows of the modes before L, e_k the whitened row k of mode L).
struct GroupedPlan {
  int32_t on;      // 1: replaces the sample-split FP64 Gram and its assembly
  int32_t L, RL;   // grouping mode and its rank
  int64_t s;       // samples
  int64_t dp;      // d / R_L
  int64_t groups;  // rows of mode L in the row geometry
  int64_t nb;      // sort blocks of 256 samples
  int64_t ncnt;    // count-table entries groups nb + 1
  int64_t nparts;  // scan partials of the count table
  int64_t ptiles;  // lower 64 x 64 tiles of d' x d'
  int32_t sp;      // S' = sum_{n<L} R_n: length of a sample's rows of the modes before L
  // pair form (two modes before L): B_k kept as C_k[i0][i1], i0 and i1 the index
  // pairs r >= r' of modes 0 and 1 (n0, n1 of them), in ptiles = tiles0 tcn tiles
  int32_t pair, tcn, n0, n1;
};
// On for FP64 when d >= 256, R_L >= 2 and the grouped form needs clearly
// fewer multiply-adds; gr is the row geometry (the augmented one for
// augmented draws).
GroupedPlan plan_grouped(const Geom& gr, int64_t s, tk_dtype prec);
size_t grouped_bytes(const GroupedPlan& gp);
// M (d x d, lower triangle) = sum_t weff_t q_t q_t^T + lambda (x)_n P_n from the
// samples' indices idx ([order][s]) and the row tables Q64 (at gr.qoff);
// ws: grouped_bytes(gp) bytes.
// xw: per-sample w_t x_t, kept (sorted) for launch_grouped_resid.
void launch_grouped_gram(const Geom& gr, const GroupedPlan& gp, const int32_t* idx,
                         const double* Q64, const double* weff, const double* xw, const double* P,
                         double lambda, void* ws, double* M, hipStream_t st);
// After launch_grouped_gram on the same ws: out = sum_t q_t (xw_t - weff_t q_t.h), or
// the right side sum_t xw_t q_t when h is null (FP64, grouped by i_L the same way).
bool grouped_resid_ok(const GroupedPlan& gp);
void launch_grouped_resid(const Geom& gr, const GroupedPlan& gp, const double* Q64, void* ws,
                          const double* h, double* out, hipStream_t st);

struct GramPlan {
  tk_dtype prec;
  bool streamk;
  GroupedPlan grp; // FP64: the grouped Gram when grp.on
  SkBatch sk;      // FP32 / BF16: a stream-K batch of one
  int tile;        // FP64: output tile edge
  int bk;          // samples per LDS chunk
  int ksplit;      // FP64: sample splits (partials)
  int64_t chunk;   // FP64: samples per split
  int64_t ntiles;  // FP64: lower-triangular tiles
};
GramPlan plan_gram(const Geom& g, int64_t s, tk_dtype prec, int ksplit_override);
size_t gram_partial_bytes(const Geom& g, const GramPlan& pl);
void launch_gram(const Geom& g, const GramPlan& pl, const double* rows64, const float* rows32,
                 const double* weff, int64_t s, void* partials, hipStream_t st);
// M = sum of partials (lower triangle) + lambda * ((x) P_n); FP64, full d x d row-major.
void launch_assemble(const Geom& g, const GramPlan& pl, const void* partials, const double* P,
                     double lambda, double* M, hipStream_t st);

// Host-side device queries (tk_gram.hip).  Each caches its answer per HIP
// device under one mutex (host threads may launch concurrently).  A failing
// query falls back to a safe value and clears only the HIP error it raised
// itself: an error already pending from an earlier call is never cleared, so
// the entry point's final hipGetLastError() check (and the caller) still see it.
//
// Workgroups of `kernel` (with `threads` threads and dyn_lds bytes of dynamic
// LDS) resident on the whole current device at once: a grid-stride pass with
// equal shares per workgroup runs in one wave only if its grid is no larger.
int resident_grid(const void* kernel, int threads, size_t dyn_lds);
// Compute units of the current device (256 on MI355X).
int device_cu_count();
// Raises `kernel`'s dynamic-LDS limit to `bytes` on the current device (once
// per device and kernel; later calls with the same or a smaller size return at once).
void ensure_dyn_lds(const void* kernel, int bytes);

// out[r] = sum_t c_t q_t[r] (q_t the whitened Kronecker row), FP64, deterministic.
// part: vec_part_doubles(g, s) scratch.
int64_t vec_part_doubles(const Geom& g, int64_t s);
void launch_rows_t_vec(const Geom& g, const double* rows64, const double* c, int64_t s,
                       double* part, double* out, const int32_t* done, hipStream_t st);
// Small Kronecker dimension (resid_small_ok): out = sum_t c_t q_t with
// c_t = a_t - b_t (q_t . h) (a term absent when a is null, dot when h is null),
// from the sample indices and the whitened factor tables in one pass; part:
// vec_part_doubles.
bool resid_small_ok(const Geom& g);
void launch_resid_small(const Geom& g, const int32_t* idx, const double* Q64, const double* a,
                        const double* b, const double* h, int64_t s, double* part, double* out,
                        const int32_t* done, hipStream_t st);
// Larger Kronecker dimension (resid_big_ok: d <= 4096, at most 512 outer
// indices, R_L <= 32, sum_r <= 64): the same sum from the FP64 sample rows in
// one pass; part: vec_part_doubles.
bool resid_big_ok(const Geom& g);
void launch_resid_big(const Geom& g, const double* rows64, const double* a, const double* b,
                      const double* h, int64_t s, double* part, double* out, const int32_t* done,
                      hipStream_t st);
// The per-workgroup partials of the same sum only (part[k][r], k < return value).
int64_t launch_resid_small_parts(const Geom& g, const int32_t* idx, const double* Q64,
                                 const double* a, const double* b, const double* h, int64_t s,
                                 double* part, const int32_t* done, hipStream_t st);

// One refinement step for d <= 256 in one workgroup (tk_refine.hip): r = the
// summed partials + b - lambda P h, relres = ||r|| / ||norm_ref||, done once
// relres <= tol, else (when do_solve) h += (L L^T)^{-1} r with L in M and the
// diagonal-block inverses; returns at entry once done is set.  first: the
// initial solve instead, h = (L L^T)^{-1} b with no partials (nparts 0), done
// cleared, steps and relres untouched.
bool refine_small_ok(const Geom& g);
// For d <= 8192: P h applied in one workgroup, then r = r + b - lambda P h and the
// same test (done / steps / relres) as launch_refine_check.
bool refine_check_p_ok(const Geom& g);
// out = ((x)_n M_n^T) t (trans) or ((x)_n M_n) t, M_n at roff[n], in one
// workgroup for d <= 8192 (core_chain_small_ok), written in dtype dt.
bool core_chain_small_ok(const Geom& g);
void launch_core_chain_small(const Geom& g, const double* t, const double* mats, bool trans,
                             void* out, tk_dtype dt, hipStream_t st);
// solve_flags / solve_y (nullable): also prepare the next launch_chol_solve
// (prepared = true) with this scratch.
void launch_refine_check_p(const Geom& g, double* r, const double* h, const double* P,
                           const double* b, double lambda, const double* norm_ref, double tol,
                           int32_t* done, int32_t* steps, double* relres, int count_step,
                           hipStream_t st, int32_t* solve_flags = nullptr,
                           double* solve_y = nullptr);
void launch_refine_step_small(const Geom& g, const double* part, int64_t nparts, const double* P,
                              const double* b, double lambda, const double* norm_ref, double tol,
                              const double* L, const double* Linv_diag, double* h, int32_t* done,
                              int32_t* steps, double* relres, int do_solve, hipStream_t st,
                              int first = 0);

// Refinement residual coefficients c_t = xw_t - weff_t (q_t . h); part: vec_part_doubles.
void launch_residual_coef(const Geom& g, const double* rows64, const double* xw,
                          const double* weff, const double* h, int64_t s, double* part, double* c,
                          const int32_t* done, hipStream_t st);

// Dense FP64 Cholesky, lower, in place (tk_chol.hip).  Linv_diag
// (kCholAuxBlocks * ceil(d/nb) blocks of nb x nb doubles) receives the
// inverses of the nb x nb diagonal blocks, then the two triangular solves'
// chain matrices, then holds the factorisation's per-column partial sums;
// min_pivot one double; flags chol_flag_words(d) int32 (the factorisation's
// ticket and tile flags live past the solves' two tickets).
constexpr int kCholNb = 64;
constexpr int kCholAuxBlocks = 5;
inline int64_t chol_flag_words(int64_t d) {
  const int64_t nblk = (d + kCholNb - 1) / kCholNb;
  return 2 + (1 + nblk * (nblk + 1) / 2 + 2 * nblk) * 32;  // one 128-byte line per flag
}
// max_grid > 0 caps the workgroups (at least 2: the chain and one task worker),
// for calls that share the GPU with concurrent work; the tasks are ticketed,
// so a smaller grid only serialises them.  skip (nullable): the kernels return
// at once when *skip != 0 (the system was solved without the factorisation).
void launch_cholesky(double* M, int64_t d, double* Linv_diag, double* min_pivot, int32_t* status,
                     int32_t* flags, hipStream_t st, int max_grid = 0,
                     const int32_t* skip = nullptr);

// Conjugate-gradient solve of M h = b, M symmetric positive definite given by
// its lower triangle (tk_cg.hip): one persistent launch with grid barriers, at
// most max_iter iterations, stopping at ||r|| <= 1e-14 ||b||.  ws: cg_bytes(d)
// bytes.  On convergence h holds the solution, the
// done word (cg_done_word) is 1 and *min_pivot = 0; otherwise h = b and the
// done word is 0, for a factorisation and triangular solves that follow.
// steps / relres: iterations and final recursive ||r|| / ||b||.
bool cg_ok(int64_t d);
size_t cg_bytes(int64_t d);
void launch_cg(const double* M, int64_t d, const double* b, double* h, void* ws, int32_t* steps,
               double* relres, double* min_pivot, int32_t* status, int max_iter,
               hipStream_t st);
const int32_t* cg_done_word(void* ws, int64_t d);
// Solve (L L^T) x = b in place on x (x holds b on entry).  flags: int32
// scratch of 2 * ceil(d/nb) + 2 words.  accum (nullable): accum += x, entry by
// entry as x is published.  prepared: y_tmp already holds kSolvePending and
// flags[0], flags[1] are zero (the refinement check can leave them so), and
// the initialising launch is skipped.
void launch_chol_solve(const double* L, const double* Linv_diag, int64_t d, double* x,
                       double* y_tmp, int32_t* flags, const int32_t* done, int32_t* status,
                       hipStream_t st, double* accum = nullptr, bool prepared = false);
// The triangular solves' "not yet published" word (a signalling-NaN pattern no
// arithmetic result takes).
constexpr unsigned long long kSolvePending = 0x7FF4DEADBEEF0001ull;

// Small FP64 helpers (tk_small.hip).
// T' = T x_mode M  for row-major T of shape dims (order n), M: J x dims[mode]
// (row-major; transpose_M: M stored dims[mode] x J).  scratch (nullable, at
// least kTtmScratchDoubles) lets a contraction with few fibres split over i.
// done (nullable): the kernels return at once when *done != 0.
constexpr int64_t kTtmScratchDoubles = int64_t(2) * 65536 * kMaxRank;
void launch_ttm(const double* T, const int64_t* dims, int order, int mode, const double* M,
                int64_t J, bool transpose_M, double* out, double* scratch, hipStream_t st,
                const int32_t* done = nullptr);
// ttm over an input of element type dt (F32 or F64) -> FP64 output
void launch_ttm_any(const void* T, tk_dtype dt, const int64_t* dims, int order, int mode,
                    const double* M, int64_t J, bool transpose_M, double* out, double* scratch,
                    hipStream_t st);
void launch_copy_f64(int64_t n, const double* x, double* y, hipStream_t st);
void launch_cast_out(int64_t n, const double* x, void* y, tk_dtype dt, hipStream_t st);
void launch_cast_in(int64_t n, const void* x, tk_dtype dt, double* y, hipStream_t st);
void launch_fill_i32(int64_t n, int32_t v, int32_t* p, hipStream_t st);
void launch_fill_f64(int64_t n, double v, double* p, hipStream_t st);
void launch_fill_u32(int64_t n, uint32_t v, uint32_t* p, hipStream_t st);
// status, done, steps = 0, relres = 0, min_pivot = 1e308, missing = 0 in one launch
void launch_init_words(int32_t* status, int32_t* done, int32_t* steps, double* relres,
                       double* min_pivot, uint32_t* missing, hipStream_t st);
// Refinement bookkeeping: residual update, relative residual, convergence flag:
// r <- r + b - lambda ph (b, ph may be NULL); stops (done = 1) once
// ||r|| <= tol ||rhs||.
void launch_refine_check(int64_t d, double* r, const double* ph, const double* b, double lambda,
                         const double* rhs, double tol, int32_t* done, int32_t* steps,
                         double* relres, int count_step, hipStream_t st);
void launch_info(double* info, int64_t s, const unsigned int* missing, const int32_t* steps,
                 const double* relres, const double* min_pivot, hipStream_t st);
// Cholesky pivot sanity of a refinement that did not converge.
void launch_finish_refine(const int32_t* done, int refine_enabled, int32_t* status,
                          hipStream_t st);

// Adjoint of the sampled update (tk_adjoint.hip).
size_t adjoint_lds_bytes(const Geom& g);
// abar[qoff_n + i * R_n + r] += alpha_t (V x_{m!=n} a^(m)) - beta_t (G x_{m!=n} a^(m)) at the
// samples' factor rows (nbeta = -beta); FP64 atomics.
void launch_adjoint_factors(const Geom& g, const void* const* factors, tk_dtype dt,
                            const int32_t* idx, int64_t s, const double* V, const double* G,
                            const double* alpha, const double* nbeta, double* abar,
                            hipStream_t st);
// xbar[flat(idx_t)] += beta_t (dense tensor of the problem dtype).
void launch_adjoint_x(const Geom& g, const int32_t* idx, int64_t s, const double* nbeta,
                      void* xbar, tk_dtype dt, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);

// Masked exact core (tk_masked.hip): fibres along the last mode, P fibres of
// length I, W = W_{N-1} (I x R, row-major).
void launch_masked_rhs(const void* X, tk_dtype dt, const uint32_t* mask, int64_t P, int64_t I,
                       const double* W, int R, double* out, hipStream_t st);
void launch_masked_normal(const double* H, const uint32_t* mask, int64_t P, int64_t I,
                          const double* W, int R, double* out, const int32_t* done,
                          hipStream_t st);
void launch_pcg_guess(const Geom& g, const double* lam, double lambda, const double* b, double* y,
                      hipStream_t st);
void launch_pcg_start(const Geom& g, const double* lam, double lambda, double tol, const double* b,
                      const double* y, const double* q, double* r, double* p, double* scal,
                      int32_t* done, hipStream_t st);
void launch_pcg_step(const Geom& g, const double* lam, double lambda, double tol, const double* q,
                     double* y, double* r, double* p, double* scal, int32_t* done,
                     hipStream_t st);
void launch_pcg_finish(const int32_t* done, int32_t* status, hipStream_t st);

// Exact path (tk_exact.hip).
void launch_eig_modes(const Geom& g, const void* const* factors, tk_dtype dt, double* V,
                      double* lam, double* W, double* C, hipStream_t st);
void launch_gram_modes(const Geom& g, const void* const* factors, tk_dtype dt, double* C,
                       hipStream_t st);
// Cor. B.1 overestimate from the eigenvalues of eig_modes (lam_modes[n * 64 + a]).
void launch_masked_bound(const Geom& g, const double* lam_modes, double lambda, double k,
                         double one_plus_c, double* out, hipStream_t st);
void launch_kron_scale(const Geom& g, const double* lam_modes, double lambda, double* B,
                       hipStream_t st);
void launch_sq_reduce(int64_t n, const void* x, tk_dtype dt, double* part, int64_t nparts,
                      hipStream_t st);
void launch_loss_stream(const Geom& g, const void* X, tk_dtype dt, const uint32_t* mask,
                        const double* H, const double* AN, double* part_sq, double* part_cnt,
                        int64_t nparts, hipStream_t st);
void launch_loss_final(const double* part_sq, const double* part_cnt, int64_t nparts,
                       const double* part_reg, int64_t nreg, double lambda, double* out,
                       hipStream_t st);
void launch_unfold_contract(const double* U, const double* V, int64_t P, int64_t I, int64_t A,
                            int64_t Q, double* out, hipStream_t st);
// Factor update over the observed entries (tk_factor_masked.hip): order >= 2;
// scratch holds factor_masked_bytes(g) bytes; A64 the FP64 factors at
// geom.qoff, G64 the FP64 core; out I_n x R_n of dt.
bool factor_masked_ok(const Geom& g);
size_t factor_masked_bytes(const Geom& g);
void launch_factor_masked(const Geom& g, int n, const void* X, tk_dtype dt, const uint32_t* mask,
                          const double* A64, const double* G64, double lambda, void* out,
                          int32_t* status, void* scratch, hipStream_t st);
void launch_factor_solve(const double* KKt, const double* rhs, int64_t I, int R, double lambda,
                         void* out, tk_dtype dt, int32_t* status, hipStream_t st);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace tk

#define TK_HIP_CHECK(expr)                         \
  do {                                             \
    if ((expr) != hipSuccess) return TK_E_HIP;     \
  } while (0)
