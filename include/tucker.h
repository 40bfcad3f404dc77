/*
 * tucker.h -- C ABI of the MI355X (gfx950) library for the ridge-leverage-score
 * sampled core-tensor update of Tucker ALS.
 *
 * Paper: Fahrbach, Ghadiri, Fu, "Fast Low-Rank Tensor Decomposition by Ridge
 * Leverage Score Sampling" (arXiv 2107.10654).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All tensors are row-major (C order): X[i_1,...,i_N] sits at
 *   sum_n i_n * stride_n with i_N fastest.  The core G is R_1 x ... x R_N
 *   row-major; factor A(n) is I_n x R_n row-major.
 * - The design row of multi-index i is k_i = a(1)[i_1,:] (x) ... (x) a(N)[i_N,:]
 *   (row-major Kronecker), so K = A(1) (x) ... (x) A(N) and K vec(G) = vec(Xhat)
 *   (Sec. 2, elementwise Tucker model; Alg. 2 core step).
 * - Pointers named "device" must point to device memory of the current HIP
 *   device.  The library never allocates, frees or synchronises: the caller
 *   owns every buffer, including the workspace whose size
 *   tucker_workspace_bytes() reports.
 * - Every call is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *   the null stream).  Argument and shape errors are returned synchronously and
 *   nothing is enqueued.  Data-dependent failures (matrix not positive
 *   definite, rank-deficient factor, refinement not converged) are written as a
 *   tk_status code into the device word `dev_status`, which the caller reads
 *   after synchronising the stream.  A call that writes dev_status first clears
 *   it on the stream.
 * - Per-mode arrays of length I_n (scores, weights, CDFs) are concatenated in
 *   mode order: mode n starts at offset sum_{m<n} I_m.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_MAX_ORDER 8     /* largest supported tensor order N */
#define TK_MAX_RANK 64     /* largest supported per-mode rank R_n */
#define TK_Q_BITS 24       /* fixed-point bits Q of the integer sampling weights (default) */
#define TK_Q_BITS_MIN 8    /* range of tk_sketch_opts.cdf_bits when it is not 0 */
#define TK_Q_BITS_MAX 40
#define TK_INFO_LEN 8      /* doubles written to dev_info by the sketched update */
#define TK_NUM_STAGE_EVENTS 10 /* stage boundaries of the sketched update (tk_sketch_opts) */

typedef enum { TK_F64 = 0, TK_F32 = 1, TK_BF16 = 2 } tk_dtype;

typedef enum {
  TK_OK = 0,
  TK_E_ARG = 1,             /* null pointer or bad scalar argument */
  TK_E_SHAPE = 2,           /* unsupported order, rank or size */
  TK_E_DTYPE = 3,           /* unsupported element type */
  TK_E_WORKSPACE = 4,       /* workspace smaller than tucker_workspace_bytes() */
  TK_E_NOT_SPD = 5,         /* Cholesky met a non-positive pivot */
  TK_E_RANK_DEFICIENT = 6,  /* a factor matrix has dependent columns */
  TK_E_NO_CONVERGE = 7,     /* FP64 refinement did not reach its tolerance */
  TK_E_HIP = 8              /* a HIP runtime call failed */
} tk_status;

/* One Tucker problem: the tensor, its optional observation mask, the current
 * factor matrices and the ridge parameter lambda of the regularised loss
 * (Sec. 2, loss L; Alg. 2). */
typedef struct {
  int32_t order;                        /* N, 1..TK_MAX_ORDER */
  int64_t dims[TK_MAX_ORDER];           /* I_n >= 1 */
  int32_t ranks[TK_MAX_ORDER];          /* R_n, 1..TK_MAX_RANK, R_n <= I_n */
  tk_dtype dtype;                       /* element type of X, factors and core: TK_F64 or TK_F32 */
  const void* X;                        /* device, prod(dims) elements */
  const uint32_t* mask;                 /* device or NULL; bit (e & 31) of word e >> 5 is 1
                                           when entry e (row-major offset) is observed */
  const void* factors[TK_MAX_ORDER];    /* device, A(n): dims[n] x ranks[n] */
  double lambda;                        /* ridge parameter, >= 0 */
} tk_problem;

/* Options of the sketched update (Alg. 1 / Alg. 3). */
typedef struct {
  int64_t num_samples;     /* s >= 1; <= 0 selects Alg. 1's count
                              ceil(8 d max{420 ln(4d/delta), 1/(delta eps)}) */
  double eps, delta;       /* used only when num_samples <= 0 */
  uint64_t seed;           /* Philox key word 0 */
  uint64_t counter;        /* Philox counter word 1 (e.g. the ALS iteration) */
  uint64_t problem;        /* Philox counter word 2 (problem index in a batch) */
  tk_dtype gram_precision; /* TK_F64: FP64 Gram and solve, no refinement.
                              TK_F32 / TK_BF16: Gram on MFMA with FP32
                              accumulation, FP64 Cholesky, FP64 refinement. */
  int32_t refine_max;      /* max refinement steps (low-precision Gram only) */
  double refine_tol;       /* stop when ||r||_2 <= refine_tol * ||rhs||_2 */
  void* const* stage_events; /* NULL, or TK_NUM_STAGE_EVENTS hipEvent_t handles created by the
                                caller; the call records event k on `stream` at stage boundary k:
                                0 start, 1 leverage scores and CDFs done, 2 sampling done,
                                3 gather of entries and sample rows done, 4 sketched Gram
                                kernel done, 5 assembly and right side
                                done, 6 Cholesky done, 7 first solve done, 8 refinement done,
                                9 end */
  int32_t augmented;       /* 0: the sketched Gram plus the exact lambda I (unbiased, since
                              E[sketched Gram] = K^T K).  1: Alg. 1 taken literally: draws
                              from the augmented distribution D(l, d'_eff) of Sec. 3 over
                              the rows of [K; sqrt(lambda) I] (a branch coin, then a product
                              draw or a uniform ridge row; see tucker_sample_augmented) and
                              the solve of min ||S Abar g - S bbar||, in which lambda enters
                              only through the sampled ridge rows. */
  double d_eff_lower;      /* augmented = 1: the lower bound d'_eff of the effective
                              dimension; each ridge row has mass c = min{1, d - d'_eff}
                              (clamped at 0), so 0 gives c = 1.  With num_samples <= 0 the
                              count is ceil(4 d (1 + c) max{420 ln(4d/delta), 1/(delta eps)})
                              (Cor. 3.3: beta' = 1 / (1 + c)). */
  int32_t sampling;        /* distribution of the data draws: 0 the product of the factor
                              leverage scores (Alg. 3; Lemma 4.1), 1 the true lambda-ridge
                              leverage scores of K (Sec. 2 SVD form), a mixture over
                              singular-value tuples (tucker_ridge_tables,
                              tucker_sample_ridge) */
  int32_t cdf_bits;        /* fixed-point bits Q of the integer sampling weights the call
                              builds (w = ceil(l 2^Q) for the factor scores, the ridge tuple
                              and column weights, the augmented coin's 2^Q and ceil(c 2^Q)):
                              0 selects TK_Q_BITS, else TK_Q_BITS_MIN..TK_Q_BITS_MAX
                              (TK_E_ARG otherwise).  The entry points that build tables
                              without options (tucker_leverage_scores, tucker_ridge_tables, the
                              augmented coin of tucker_sample_augmented) use TK_Q_BITS. */
} tk_sketch_opts;

/* Which call tucker_workspace_bytes() sizes. */
typedef enum {
  TK_CALL_LEVERAGE = 0,
  TK_CALL_SKETCHED = 1,
  TK_CALL_EXACT = 2,
  TK_CALL_FACTOR = 3,
  TK_CALL_LOSS = 4,
  TK_CALL_ADJOINT = 5,
  TK_CALL_MASKED_BOUND = 6,
  TK_CALL_RIDGE_TABLES = 7
} tk_call;

/* Bytes of workspace the named call needs for this problem (0 on bad input).
 * `opts` is read only for TK_CALL_SKETCHED and TK_CALL_ADJOINT and may be
 * NULL otherwise. */
size_t tucker_workspace_bytes(const tk_problem* p, const tk_sketch_opts* opts, int32_t call);

/* Sample count of Alg. 1 with beta' = 1/2 (Cor. 3.3), as used when
 * num_samples <= 0. */
int64_t tucker_sample_count(int64_t d, double eps, double delta);

/* Sample count of Alg. 1 for draws from the augmented distribution with lower
 * bound d_eff_lower (Cor. 3.3 with the leverage scores as overestimates:
 * beta' = 1/(1 + c), c = min{1, d - d_eff_lower} clamped at 0):
 * ceil(4 d (1 + c) max{420 ln(4d/delta), 1/(delta eps)}); 0 on bad input. */
int64_t tucker_sample_count_augmented(int64_t d, double eps, double delta, double d_eff_lower);

/*
 * Factor leverage scores and sampling tables -- Alg. 3, first step; the
 * statistical leverage score is the ridge score of Sec. 2 at lambda = 0,
 * l_i = a_i (A^T A)^+ a_i^T.  Computed per mode from the FP64 Cholesky
 * factor L_n of C_n = A(n)^T A(n): q_i = L_n^{-1} a_i^T, l_i = ||q_i||^2.
 *
 * Outputs (device, concatenated per mode, total T = sum_n I_n entries):
 *   scores  [T] double   l_i                                   (may be NULL)
 *   cdf     [T] uint64   inclusive prefix sums of w_i = ceil(max(l_i,0) * 2^TK_Q_BITS);
 *                        the last entry of mode n is the mode's total W_n
 *                        (the per-mode CDFs of the proof of Thm 4.2)
 * A factor whose Cholesky pivot falls to <= R_n * 2^-52 * max diag(C_n) is
 * rank deficient: dev_status gets TK_E_RANK_DEFICIENT and the small pivots are
 * replaced by 1, so the outputs stay finite but are not meaningful for that
 * mode (callers check dev_status).  Reads only p->order, dims, ranks, dtype
 * and factors.
 */
tk_status tucker_leverage_scores(const tk_problem* p, double* scores, uint64_t* cdf,
                                 int32_t* dev_status, void* ws, size_t ws_bytes, void* stream);

/*
 * Sample count for missing data -- Sec. 4.2 (Thm 4.3 with Lemma 4.4: the ridge
 * scores of K over-estimate those of the observed-rows design K~ by a factor
 * 1/beta = 1 + 1/(1 - lambda_max(L_{Sbar,Sbar})), L the cross ridge-score
 * matrix of K and Sbar the missing rows) and App. B, Cor. B.1, which bounds it
 * for ANY set of missing rows through the factors' spectral norms:
 *   1/beta <= 2 + prod_n sigma_max(A(n))^2 / lambda.
 * The sampled masked update draws from the unmasked product distribution and
 * drops the draws that land on missing entries, i.e. it samples K~'s rows with
 * these overestimates; Alg. 1's count for them is
 *   beta' = beta / (1 + c),  s = ceil(4 d (1 + c) (1/beta) max{420 ln(4d/delta), 1/(delta eps)}),
 * c = min{1, d - d_eff_lower} clamped at 0.  The bound does not depend on the
 * mask, so p->mask and p->X are not read.  sigma_max(A(n))^2 is the largest
 * eigenvalue of A(n)^T A(n) (FP64 Jacobi).
 *   out  device double [4]: [0] the 1/beta bound, [1] prod_n sigma_max(A(n))^2,
 *        [2] beta', [3] s (as a double: it can exceed 2^53 for small lambda).
 * lambda must be > 0 (TK_E_ARG otherwise).  Workspace:
 * tucker_workspace_bytes(p, NULL, TK_CALL_MASKED_BOUND).
 */
tk_status tucker_masked_sample_bound(const tk_problem* p, double eps, double delta,
                                     double d_eff_lower, double* out, void* ws, size_t ws_bytes,
                                     void* stream);

/*
 * Tables of the true lambda-ridge leverage scores of K = A(1) (x) ... (x) A(N)
 * (Sec. 2: l_i^lambda = sum_k s_k^2/(s_k^2 + lambda) u_ik^2, applied to K's SVD
 * (x)U_n (x)S_n (x)V_n; Sec. 4.1).  The scores are a mixture over the d tuples t
 * of singular-value indices (row-major over the ranks):
 *   l_i^lambda(K) = sum_t pi_t prod_n U_n[i_n, t_n]^2,
 *   pi_t = prod_n s_{n,t_n}^2 / (prod_n s_{n,t_n}^2 + lambda),
 * each component the product of the squared singular-vector columns (unit
 * norm).  With C_n = A(n)^T A(n) = V_n Lambda_n V_n^T (FP64 Jacobi),
 * s_{n,c}^2 = Lambda_n[c] and U_n[:, c] = A(n) V_n[:, c] / s_{n,c}.
 *   tuple_cdf  device uint64 [d]: inclusive prefix sums of ceil(pi_t 2^TK_Q_BITS)
 *              (pi_t = 0 when the eigenvalue product is not positive)
 *   col_cdf    device uint64 [sum_n I_n R_n]: for mode n and column c, at offset
 *              sum_{m<n} I_m R_m + c I_n, the inclusive prefix sums of
 *              ceil(U_n[i, c]^2 2^TK_Q_BITS) over i (a column whose eigenvalue
 *              is <= R_n 2^-52 max is all zero)
 *   d_eff      device double [1] or NULL: sum_t pi_t, the effective dimension
 * Degenerate eigenvalues make the singular vectors, and so these tables, one
 * valid choice among many; the mixture's row probabilities do not depend on it.
 * Workspace: tucker_workspace_bytes(p, NULL, TK_CALL_RIDGE_TABLES).
 */
tk_status tucker_ridge_tables(const tk_problem* p, uint64_t* tuple_cdf, uint64_t* col_cdf,
                              double* d_eff, void* ws, size_t ws_bytes, void* stream);

/*
 * Draws from the ridge-score mixture of K (tables of tucker_ridge_tables): per
 * draw the tuple t from tuple_cdf with word 0 of Philox block 3 (counter
 * (t, counter, problem, 3)), u = floor(r W / 2^64), first t with C_t > u; then
 * mode n's row from the table of column t_n with the word that drives mode n
 * in tucker_sample (block n / 4, word n % 4), by the same search.
 *   weight_t = 1 / (s P(i_t)),  P(i) = sum_t (w_t / W) prod_n w_{n,t_n,i_n} / W_{n,t_n},
 * the sum over all d tuples evaluated in FP64 (contracted mode by mode), so
 * weights agree with another summation order to rounding, not bit for bit.
 * augmented = 1 adds the branch coin of tucker_sample_augmented (same words,
 * same ridge-row encoding and weights; data weights times (D + C) / D).
 * Indices are bit-identical to the FP64 oracle given equal tables.
 */
tk_status tucker_sample_ridge(int32_t order, const int64_t* dims, const int32_t* ranks,
                              const uint64_t* tuple_cdf, const uint64_t* col_cdf, int64_t s,
                              uint64_t seed, uint64_t counter, uint64_t problem,
                              int32_t augmented, double d_eff_lower, int32_t* idx,
                              double* weight, void* stream);

/*
 * Product-distribution sampling of s multi-indices -- Alg. 3 (sample from
 * l(K) with factored scores; Lemma 4.1: leverage scores of a Kronecker
 * product are products of factor scores) and Alg. 1 (s i.i.d. draws with
 * replacement, sketch entry 1/sqrt(P(j) s)).
 *
 *   dims    host [order], I_n >= 1 each
 *   cdf     device, concatenated per-mode integer CDFs (as written above): exactly
 *           sum_n dims[n] uint64 entries, owned by the caller.  The call cannot check
 *           the length of a device buffer; a shorter table is read out of bounds.
 *   idx     device int32 [order][s] (structure of arrays): idx[n*s + t] = i_n of sample t
 *   weight  device double [s]: weight_t = (prod_n W_n / w_{i_n}) / s = 1/(s P(t)),
 *           the product taken in mode order, one IEEE operation at a time
 * Random words: Philox4x64-10 with key (seed, 0) and counter
 * (t, counter, problem, b); word j of block b drives mode 4b + j; the mode
 * draws u = floor(r W_n / 2^64) and takes the first row j with cdf_j > u.
 * Given equal tables the output is bit-identical to the FP64 CPU oracle.
 */
tk_status tucker_sample(int32_t order, const int64_t* dims, const uint64_t* cdf, int64_t s,
                        uint64_t seed, uint64_t counter, uint64_t problem, int32_t* idx,
                        double* weight, void* stream);

/*
 * Draws from the augmented distribution D(l, d'_eff) of Alg. 1 (Sec. 3: the
 * data rows of [K; sqrt(lambda) I] with the product of the factor leverage
 * scores, normalised to mass d, and the d ridge rows with mass c each,
 * c = min{1, d - d_eff_lower} clamped at 0).  Per draw a branch coin, then a
 * product draw (exactly the draw tucker_sample makes for the same t) or a
 * uniform ridge row:
 *   Philox words of block 2 (counter (t, counter, problem, 2)): with integer
 *   branch weights D = 2^TK_Q_BITS and C = ceil(c 2^TK_Q_BITS),
 *   u = floor(r_0 (D + C) / 2^64) < D keeps the data draw; otherwise ridge row
 *   k = floor(r_1 d / 2^64), d = prod(ranks).
 *   idx     device int32 [order][s]: data draws as tucker_sample; a ridge draw
 *           stores idx[n*s + t] = dims[n] + k_n, k_n the row-major digits of k
 *           over the ranks (so every entry lies in [dims[n], dims[n] + ranks[n]))
 *   weight  device double [s], 1/(s P(j)) with the factors in this order, one
 *           IEEE operation each: data ((prod_n W_n / w_{i_n}) * ((D + C) / D)) / s,
 *           ridge (((D + C) / C) * d) / s
 *   ranks   host [order], 1..TK_MAX_RANK, prod <= 16384; other arguments as
 *           tucker_sample.
 * With C = 0 (d_eff_lower >= d) every draw is a data draw and the output equals
 * tucker_sample's bit for bit.
 */
tk_status tucker_sample_augmented(int32_t order, const int64_t* dims, const int32_t* ranks,
                                  const uint64_t* cdf, int64_t s, uint64_t seed, uint64_t counter,
                                  uint64_t problem, double d_eff_lower, int32_t* idx,
                                  double* weight, void* stream);

/*
 * Sampled core-tensor update -- Alg. 3 FastCoreTensorUpdate calling Alg. 1
 * ApproximateRidgeRegression; normal equations as in the proof of Thm 4.2,
 * with the ridge term added to the sketched Gram:
 *   g = argmin_g sum_t weight_t (x_t - k_t . g)^2 + lambda ||g||^2
 *     = (sum_t weight_t k_t k_t^T + lambda I)^{-1} sum_t weight_t x_t k_t.
 * Samples that hit an unobserved entry (mask bit 0) contribute nothing.
 *
 *   idx_in, weight_in  device or NULL.  Both given: use this frozen sample set
 *                      (s = opts->num_samples entries).  Both NULL: compute the
 *                      leverage scores, CDFs and samples from opts.
 *   idx_out, weight_out device or NULL: receive the samples used.
 *   core_out           device, prod(ranks) elements of p->dtype.
 *   dev_info           device double [TK_INFO_LEN] or NULL:
 *                      [0] samples s, [1] samples on missing entries,
 *                      [2] refinement steps taken, [3] final relative residual
 *                      ||r||/||rhs|| (FP64), [4] smallest Cholesky pivot,
 *                      [5..7] reserved (0).
 * Internally the rows are whitened per mode (q_i = L_n^{-1} a_i^T); the
 * solution is mapped back exactly, so the result is the g above.
 * With opts->augmented = 1 the draws come from the augmented distribution
 * (tucker_sample_augmented; frozen sets may contain its ridge draws) and the
 * result is Alg. 1's
 *   g = argmin_g sum_t weight_t (bbar_t - abar_t . g)^2,
 * abar_t = k_t and bbar_t = x_t for data draws (0 and 0 on unobserved
 * entries), abar_t = sqrt(lambda) e_k and bbar_t = 0 for ridge draws: no
 * lambda I is added.
 */
tk_status tucker_core_update_sketched(const tk_problem* p, const tk_sketch_opts* opts,
                                      const int32_t* idx_in, const double* weight_in,
                                      int32_t* idx_out, double* weight_out, void* core_out,
                                      int32_t* dev_status, double* dev_info, void* ws,
                                      size_t ws_bytes, void* stream);

/*
 * The sampled core update of tucker_core_update_sketched for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Arguments, results, status and
 * errors are those of tucker_core_update_sketched, without the workspace: the
 * call uses a device array of TK_NOALLOC_SCRATCH_BYTES built into the library
 * (one copy per GPU, allocated when the library's code is first loaded on that
 * GPU and held until the process ends).  Its device address is looked up on
 * the first call made with each device current; the call itself never
 * allocates, frees or synchronises.
 *   Returns TK_E_WORKSPACE when the problem needs more workspace than that,
 *   i.e. tucker_workspace_bytes(p, opts, TK_CALL_SKETCHED) >
 *   TK_NOALLOC_SCRATCH_BYTES (use tucker_core_update_sketched with a caller
 *   workspace instead); TK_E_HIP when the array's address cannot be found.
 * Every call on one GPU shares that GPU's array and finds it holding the
 * previous call's contents (the update clears what must start at zero).  Calls
 * that overlap in time on one GPU -- on different streams, or from several
 * threads -- race on the array and give undefined results; serialise them.
 */
#define TK_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

tk_status tucker_core_update_sketched_noalloc(const tk_problem* p, const tk_sketch_opts* opts,
                                              const int32_t* idx_in, const double* weight_in,
                                              int32_t* idx_out, double* weight_out,
                                              void* core_out, int32_t* dev_status,
                                              double* dev_info, void* stream);

/*
 * The sketched ridge normal equations that tucker_core_update_sketched
 * factors and solves (Alg. 1; proof of Thm 4.2), in the whitened
 * coordinates of its solver.  With W = (x)_n L_n^{-1} (L_n the Cholesky factor
 * of C_n = A(n)^T A(n), Kronecker product in mode order) and the Kronecker
 * row q_t = W k_t of sample t (entries prod_n (L_n^{-1} a^(n)_{i_n})[r_n]):
 *   M = sum_t weight_t q_t q_t^T + lambda P,   P = W W^T = (x)_n L_n^{-1} L_n^{-T},
 *   b = sum_t weight_t x_t q_t,
 * so that g = W^T M^{-1} b is the sampled core update.  Samples on unobserved
 * entries contribute nothing.  The Gram term is summed on MFMA in
 * opts->gram_precision (TK_F32 / TK_BF16 operands, FP32 accumulation) or in
 * FP64, exactly as the update forms it; lambda P and b are FP64.
 *
 *   idx, weight  device, the sample set (required; s = opts->num_samples
 *                entries, layout as tucker_sample)
 *   M_out        device double [d * d], d = prod(ranks), row-major; entries
 *                with row >= column are written, the others are unspecified
 *   b_out        device double [d]
 * With opts->augmented = 1 the sample set may hold ridge draws (as written by
 * tucker_sample_augmented), whose whitened rows sqrt(lambda) W e_k enter the
 * Gram term, and lambda P is not added.
 * Workspace: tucker_workspace_bytes(p, opts, TK_CALL_SKETCHED).
 */
tk_status tucker_sketched_system(const tk_problem* p, const tk_sketch_opts* opts,
                                 const int32_t* idx, const double* weight, double* M_out,
                                 double* b_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                                 void* stream);

/*
 * Adjoint (reverse-mode derivative) of the sampled core update with the
 * sample set held fixed.  The forward map is the solution of the sketched
 * ridge normal equations of Alg. 1 (proof of Thm 4.2),
 *   g = M^{-1} sum_t w_t x_t k_t,   M = sum_t w_t k_t k_t^T + lambda I,
 * with (idx, weight) constants: the sampling weights are not differentiated
 * through the leverage scores.  For a cotangent gbar and v = M^{-1} gbar:
 *   x_bar[i_t]        += w_t (k_t . v)                         (observed samples)
 *   factor_bar(n)[i_n] += alpha_t (V x_{m!=n} a^(m)_{i_m}) - beta_t (G x_{m!=n} a^(m)_{i_m})
 * with alpha_t = w_t (x_t - k_t . g), beta_t = w_t (k_t . v), V and G the
 * core-shaped v and g.  M is rebuilt from (idx, weight) exactly as the
 * forward call builds it (Gram precision opts->gram_precision, FP64 Cholesky,
 * FP64 refinement of the solve for v).
 *
 *   idx, weight   device, the frozen sample set of the forward call (required;
 *                 s = opts->num_samples entries, layout as tucker_sample)
 *   core          device, the forward result g (prod(ranks) of p->dtype)
 *   core_bar      device, the cotangent gbar (prod(ranks) of p->dtype)
 *   factor_bar    host array of p->order device pointers; factor_bar[n] receives
 *                 dims[n] x ranks[n] values of p->dtype (overwritten)
 *   x_bar         device, dense tensor of p->dtype with the shape of X
 *                 (overwritten: zero except at sampled observed entries), or NULL
 *   dev_info      as for tucker_core_update_sketched (refinement of the v solve)
 * opts->augmented must be 0 (TK_E_ARG otherwise).
 * Workspace: tucker_workspace_bytes(p, opts, TK_CALL_ADJOINT).  Duplicate
 * samples are accumulated with FP64 (factors) or p->dtype (x_bar) atomics, so
 * results agree with a sequential sum to rounding.
 */
tk_status tucker_core_update_sketched_adjoint(const tk_problem* p, const tk_sketch_opts* opts,
                                              const int32_t* idx, const double* weight,
                                              const void* core, const void* core_bar,
                                              void* const* factor_bar, void* x_bar,
                                              int32_t* dev_status, double* dev_info, void* ws,
                                              size_t ws_bytes, void* stream);

/*
 * Batched sampled core updates: `count` (1..TK_MAX_BATCH) independent
 * problems of any shapes and ranks, each updated exactly as
 * tucker_core_update_sketched would (same samples for the same seed,
 * counter and problem fields), with the sketched Grams of all problems
 * computed by ONE persistent stream-K launch: the (tile, 32-sample chunk)
 * units of every problem are laid out back to back and split evenly over the
 * GPU, so small and large problems share the machine.  Leverage scores,
 * sampling, assembly, Cholesky and refinement run per problem on `stream`.
 * The call neither allocates nor synchronises, so it can be captured in a
 * HIP graph and replayed.
 *
 *   probs, opts   host arrays [count]; every opts[k].gram_precision is the same,
 *                 TK_F32 or TK_BF16 (FP32 accumulation; FP64 solve and refinement)
 *   cfg           tile shape and persistent grid of the batched Gram (NULL: tile
 *                 128, 3 workgroups per CU); tucker_tune_batched picks one
 *   core_out      host array [count] of device pointers (prod(ranks_k) of dtype_k)
 *   dev_status    device int32 [count], one status word per problem
 *   dev_info      device double [count][TK_INFO_LEN] or NULL (as for the single call)
 * Workspace: tucker_workspace_bytes_batched(probs, opts, count, cfg).
 */
#define TK_MAX_BATCH 64

typedef struct {
  int32_t tile;      /* Gram output tile edge: 64, 128 or 256 (0: 128) */
  int32_t wg_per_cu; /* workgroups per compute unit in the persistent grid, 1..8 (0: 3) */
} tk_batch_config;

size_t tucker_workspace_bytes_batched(const tk_problem* probs, const tk_sketch_opts* opts,
                                      int32_t count, const tk_batch_config* cfg);

tk_status tucker_core_update_sketched_batched(const tk_problem* probs, const tk_sketch_opts* opts,
                                              int32_t count, const tk_batch_config* cfg,
                                              void* const* core_out, int32_t* dev_status,
                                              double* dev_info, void* ws, size_t ws_bytes,
                                              void* stream);

/*
 * Autotuner of the batched call: runs steps 1-3 of every problem once, then
 * times the batched Gram launch (one warm-up, one timed run, HIP events on
 * `stream`) for each candidate tile shape and grid -- tile 128 with 3 or 2
 * workgroups per CU, tile 256 with 1, tile 64 with 4, 5 or 6 -- and returns
 * the fastest in
 * *best.  Unlike every other call it synchronises `stream`, so run it once
 * per batch shape before capturing the batched call.  The workspace must be
 * tucker_workspace_bytes_batched(probs, opts, count, NULL) bytes (enough for
 * every candidate).  times_ms (host, may be NULL) receives each candidate's
 * time and *n_candidates (may be NULL) their number.
 */
tk_status tucker_tune_batched(const tk_problem* probs, const tk_sketch_opts* opts, int32_t count,
                              void* ws, size_t ws_bytes, void* stream, tk_batch_config* best,
                              double* times_ms, int32_t* n_candidates);

/*
 * Exact core-tensor update -- Alg. 2 core step,
 *   G = argmin ||K vec G - vec X||^2 + lambda ||G||^2,
 * through the eigen form of the proof of Lemma 4.1:
 *   K^T K + lambda I = ((x)V_n) ((x)Lambda_n + lambda I) ((x)V_n)^T,
 *   C_n = A(n)^T A(n) = V_n Lambda_n V_n^T.
 * One streaming pass over X forms K^T vec X.  With a mask, the update is over
 * the observed entries only (the masked design of Sec. 4.2),
 *   (K~^T K~ + lambda I) g = K~^T x~,
 * solved by preconditioned conjugate gradients in the eigenbasis above, where
 * the unmasked operator (x)Lambda_n + lambda I is diagonal and serves as the
 * preconditioner; the start is the unmasked solution.  Each iteration applies
 * the masked operator fibre by fibre along the last mode without forming a
 * tensor of X's size.  Stops at relative residual 1e-10 (FP64); after 64
 * iterations without reaching it dev_status gets TK_E_NO_CONVERGE.  The
 * kernels of the remaining iterations return at once, so the call stays
 * asynchronous.
 */
tk_status tucker_core_update_exact(const tk_problem* p, void* core_out, int32_t* dev_status,
                                   void* ws, size_t ws_bytes, void* stream);

/*
 * Factor-matrix update of Alg. 2 for mode `mode` (0-based): every row solves
 *   a_i = argmin_y ||y K_n - x_(n),i||^2 + lambda ||y||^2,
 *   K_n = G_(n) ((x)_{m != n} A(m))^T,
 * i.e. A(n) = X_(n) K_n^T (K_n K_n^T + lambda I)^{-1}.  One streaming pass over
 * X.  With a mask (tensor completion, Sec. 4.2) each row solves its ridge
 * problem over its observed entries only,
 *   a_i = (sum_{j obs} k_j k_j^T + lambda I)^{-1} sum_{j obs} x_ij k_j,
 * with k_j the column j of K_n: one pass over X and the mask that accumulates
 * every row's R_n x R_n Gram in FP64, then a FP64 Cholesky per row (order >= 2,
 * else TK_E_SHAPE; unobserved entries of X are never read, so they may hold
 * anything, NaN included).  A row whose system is not positive definite
 * (lambda = 0 with too few observations) sets dev_status to TK_E_NOT_SPD.
 *   core        device, prod(ranks) elements of p->dtype
 *   factor_out  device, dims[mode] x ranks[mode] of p->dtype (may alias
 *               p->factors[mode]; it is written last)
 * Workspace: tucker_workspace_bytes(p, NULL, TK_CALL_FACTOR), which depends on
 * whether p->mask is set.
 */
tk_status tucker_factor_update(const tk_problem* p, const void* core, int32_t mode,
                               void* factor_out, int32_t* dev_status, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * Regularised Tucker loss of Sec. 2,
 *   L = ||X - Xhat||_F^2 + lambda (||G||_F^2 + sum_n ||A(n)||_F^2),
 * with the residual over observed entries when a mask is given.
 *   out  device double [3]: [0] L, [1] sum of squared residuals,
 *        [2] number of observed entries (RMSE = sqrt(out[1] / out[2])).
 */
tk_status tucker_loss(const tk_problem* p, const void* core, double* out, void* ws,
                      size_t ws_bytes, void* stream);

/* Human-readable name of a status code (static storage). */
const char* tucker_status_string(tk_status s);

/* ABI revision of this header. */
int32_t tucker_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_H */
