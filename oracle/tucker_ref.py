"""Plain FP64 CPU oracle for the ridge-leverage-score-sampled Tucker core update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP library.

Conventions (the paper's elementwise Tucker model, eq.
tucker_decomposition_elementwise in Sec. 2, is order-free; the paper's ``vec``
stacks columns first, which would pair with the reversed Kronecker order, so the
elementwise definition decides):

* Tensors are row-major (C order): X[i1, ..., iN] with iN fastest.
* The core G is R1 x ... x RN row-major, vec(G) is its C-order flattening.
* Factor A(n) is In x Rn row-major.
* The design row of multi-index i is k_i = a(1)[i1,:] (x) ... (x) a(N)[iN,:]
  (row-major Kronecker), so K = A(1) (x) ... (x) A(N) and K vec(G) = vec(Xhat).

Every routine works in float64 (uint64 for the integer sampling tables).
Inputs of lower precision are converted exactly to float64 first.
"""
import math

import numpy as np

from .philox import philox4x64, mulhi64

#: Fixed-point bits of the integer sampling weights w_i = ceil(l_i * 2^Q).
Q_BITS = 24


# --------------------------------------------------------------------------
# Tensor algebra (Sec. 2, "Tensor Products")
# --------------------------------------------------------------------------

def mode_product(T, M, n):
    """n-mode product T x_n M for M of shape (J, I_n) (Sec. 2, elementwise form)."""
    out = np.tensordot(M, T, axes=([1], [n]))  # J first
    return np.moveaxis(out, 0, n)


def unfold(T, n):
    """Mode-n unfolding, columns ordered row-major over the remaining modes."""
    return np.moveaxis(T, n, 0).reshape(T.shape[n], -1)


def reconstruct(G, factors):
    """Xhat = G x_1 A(1) x_2 ... x_N A(N) (Sec. 2, Tucker decomposition)."""
    T = np.asarray(G, dtype=np.float64)
    for n, A in enumerate(factors):
        T = mode_product(T, np.asarray(A, dtype=np.float64), n)
    return T


def kron_matrix(factors):
    """Explicit K = A(1) (x) ... (x) A(N) (tiny shapes only)."""
    K = np.ones((1, 1))
    for A in factors:
        K = np.kron(K, np.asarray(A, dtype=np.float64))
    return K


def kron_rows(factors, idx):
    """Rows k_t of K for multi-indices idx[:, t], formed from factor rows only.

    This is the implicit design-matrix query of Alg. 3 (initialise a structure
    that answers entries of K without forming it): row t is the Kronecker
    product of the sampled factor rows, in mode order.
    """
    idx = np.asarray(idx)
    s = idx.shape[1]
    rows = np.ones((s, 1))
    for n, A in enumerate(factors):
        a = np.asarray(A, dtype=np.float64)[idx[n]]
        rows = (rows[:, :, None] * a[:, None, :]).reshape(s, -1)
    return rows


def flat_index(idx, dims):
    """Row-major linear offsets of the multi-indices idx[:, t]."""
    return np.ravel_multi_index(tuple(np.asarray(idx, dtype=np.int64)), dims)


def mask_lookup(mask_words, flat):
    """Observed flags of linear offsets from an LSB-first uint32 bit mask."""
    words = np.asarray(mask_words, dtype=np.uint32)[flat >> 5]
    return ((words >> (flat & 31).astype(np.uint32)) & 1).astype(bool)


def unpack_mask(mask_words, dims):
    """Dense boolean observed-mask from LSB-first uint32 words."""
    n = int(np.prod(dims))
    return mask_lookup(mask_words, np.arange(n, dtype=np.int64)).reshape(dims)


# --------------------------------------------------------------------------
# Ridge leverage scores (Sec. 2, eqs. ridge_leverage_score_def,
# ridge_leverage_score_svd_def, d_eff_def)
# --------------------------------------------------------------------------

def ridge_leverage_scores(A, lam=0.0):
    """l_i^lam(A) = a_i (A^T A + lam I)^+ a_i^T, the definition written out."""
    A = np.asarray(A, dtype=np.float64)
    M = np.linalg.pinv(A.T @ A + lam * np.eye(A.shape[1]), hermitian=True)
    return np.einsum("ij,jk,ik->i", A, M, A)


def leverage_scores(A):
    """Statistical leverage scores: the ridge scores at lam = 0 (Sec. 2)."""
    return ridge_leverage_scores(A, 0.0)


def cross_ridge_scores(A, lam=0.0):
    """Matrix of cross ridge scores A (A^T A + lam I)^+ A^T (Sec. 2)."""
    A = np.asarray(A, dtype=np.float64)
    M = np.linalg.pinv(A.T @ A + lam * np.eye(A.shape[1]), hermitian=True)
    return A @ M @ A.T


def ridge_scores_svd(A, lam=0.0):
    """Ridge scores from the compact SVD: sum_k s_k^2/(s_k^2+lam) u_ik^2."""
    A = np.asarray(A, dtype=np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    tol = max(A.shape) * np.finfo(np.float64).eps * (s[0] if s.size else 0.0)
    keep = s > tol
    U, s = U[:, keep], s[keep]
    f = s ** 2 / (s ** 2 + lam)
    return (U ** 2) @ f


def effective_dimension(A, lam):
    """d_eff = sum_i l_i^lam(A) (eq. d_eff_def)."""
    return float(ridge_leverage_scores(A, lam).sum())


def is_rank_deficient(A):
    """True if A has numerically dependent columns."""
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.matrix_rank(A) < A.shape[1]


# --------------------------------------------------------------------------
# Sample count (Alg. 1, Cor. 3.3)
# --------------------------------------------------------------------------

def s_theory(d, eps, delta, beta_prime=0.5):
    """Number of row samples of Alg. 1: ceil(4d/beta' max{420 ln(4d/delta), 1/(delta eps)}).

    With the factor leverage scores as the overestimate and d'_eff = 0, Cor. 3.3
    gives beta' = 1/2 for a full-rank design (Sec. 3).
    """
    return int(math.ceil(4.0 * d / beta_prime
                         * max(420.0 * math.log(4.0 * d / delta), 1.0 / (delta * eps))))


def ridge_row_mass(d, d_eff_lower):
    """c = min{1, d - d'_eff}: the unnormalised mass of each of the d ridge rows
    in the augmented distribution D(l, d'_eff) (Sec. 3, its definition), whose
    data rows carry the overestimates normalised to total mass d.  Clamped at 0
    (a lower bound d'_eff above d leaves the ridge rows no mass)."""
    return min(1.0, max(0.0, float(d) - float(d_eff_lower)))


def s_theory_augmented(d, eps, delta, d_eff_lower=0.0):
    """Alg. 1's sample count with beta' = 1/(rank/d + c) = 1/(1 + c) for a
    full-rank design (Cor. 3.3 with the leverage scores as overestimates):
    ceil(4 d (1 + c) max{420 ln(4d/delta), 1/(delta eps)}); c = 1 (d'_eff = 0)
    gives the count of ``s_theory``."""
    c = ridge_row_mass(d, d_eff_lower)
    return int(math.ceil(4.0 * d * (1.0 + c)
                         * max(420.0 * math.log(4.0 * d / delta), 1.0 / (delta * eps))))


# --------------------------------------------------------------------------
# Missing data (Sec. 4.2): how much the scores of K overestimate those of the
# masked design K~ (Thm 4.3, Lemma 4.4, Cor. B.1)
# --------------------------------------------------------------------------

def masked_inverse_beta(factors, lam, mask):
    """1/beta = 1 + 1/(1 - lambda_max(L_{Sbar,Sbar})) for the missing rows Sbar of
    K (Thm 4.3 with Lemma 4.4: the ridge scores of K are a beta-overestimate for
    those of K~).  L is K's matrix of cross ridge scores, formed explicitly:
    tiny shapes only.  lam > 0."""
    K = kron_matrix(factors)
    L = cross_ridge_scores(K, lam)
    dims = [np.asarray(A).shape[0] for A in factors]
    miss = np.nonzero(~unpack_mask(mask, dims).reshape(-1))[0]
    if len(miss) == 0:
        return 2.0  # lambda_max of an empty block taken as 0
    lmax = float(np.linalg.eigvalsh(L[np.ix_(miss, miss)]).max())
    return 1.0 + 1.0 / (1.0 - lmax)


def masked_inverse_beta_bound(factors, lam):
    """Cor. B.1's bound, valid for any set of missing rows:
    1/beta <= 1 + (1 + prod_n ||A(n)||_2^2 / lam) = 2 + prod_n sigma_max(A(n))^2 / lam."""
    prod = 1.0
    for A in factors:
        prod *= float(np.linalg.norm(np.asarray(A, dtype=np.float64), 2)) ** 2
    return 2.0 + prod / lam


def s_theory_masked(d, eps, delta, inv_beta, d_eff_lower=0.0):
    """Alg. 1's count with a beta-overestimate, beta = 1/inv_beta <= 1:
    beta' = beta / (1 + c), s = ceil(4 d (1 + c) inv_beta max{420 ln(4d/delta), 1/(delta eps)}).
    Returned as a float (the count can exceed 2^63 for small lam)."""
    c = ridge_row_mass(d, d_eff_lower)
    return math.ceil(4.0 * d * (1.0 + c) * inv_beta
                     * max(420.0 * math.log(4.0 * d / delta), 1.0 / (delta * eps)))


# --------------------------------------------------------------------------
# Integer CDF tables and product-distribution sampling
# (Lemma 4.1 product law; Alg. 3 sampler; proof of Thm 4.2: per-mode CDFs
#  and one binary search per mode)
# --------------------------------------------------------------------------

def cdf_table(scores, q_bits=Q_BITS):
    """Integer weights w_i = ceil(max(l_i, 0) * 2^Q) and their inclusive prefix sums.

    The paper asks for a CDF per factor; integer weights make the table exact
    and independent of summation order.  The sampled distribution is q = w / W
    and the rescaling below uses the same q, so this is Alg. 1 run with the
    overestimate w (every row with a nonzero score keeps a nonzero weight).
    """
    sc = np.maximum(np.asarray(scores, dtype=np.float64), 0.0)
    w = np.ceil(sc * float(2 ** q_bits)).astype(np.uint64)
    C = np.cumsum(w, dtype=np.uint64)
    return w, C


def _product_draws(tables, s, seed, counter, problem):
    """Indices of s product-distribution draws and prod_n W_n / w_{i_n} per draw
    (the product in mode order, one IEEE operation at a time)."""
    N = len(tables)
    t = np.arange(s, dtype=np.uint64)
    idx = np.empty((N, s), dtype=np.int32)
    for b in range((N + 3) // 4):
        words = philox4x64(t, np.uint64(counter), np.uint64(problem), np.uint64(b),
                           seed, 0)
        for j in range(4):
            n = 4 * b + j
            if n >= N:
                break
            w, C = tables[n]
            u = mulhi64(words[j], np.uint64(C[-1]))
            idx[n] = np.searchsorted(C, u, side="right").astype(np.int32)
    acc = np.ones(s, dtype=np.float64)
    for n in range(N):
        w, C = tables[n]
        W = np.float64(C[-1])
        acc = acc * (W / w[idx[n]].astype(np.float64))
    return idx, acc


def sample(tables, s, seed, counter, problem=0):
    """Draw s multi-indices i.i.d. from the product of the per-mode distributions.

    tables : list of (w, C) per mode from ``cdf_table``.
    Random words: Philox4x64-10 with key (seed, 0) and counter
    (t, counter, problem, block); word j of block b drives mode 4b + j.
    Mode n draws u = floor(r * W_n / 2^64) and takes the first row j with
    C_j > u (inverse-CDF by binary search).  Draws are with replacement (Alg. 1).

    Returns idx (N, s) int32 and weight (s,) float64, where
    weight_t = (prod_n W_n / w_{i_n}) / s  = 1 / (s * P(row t))
    so that sum_t weight_t k_t k_t^T is the sketched Gram (S K)^T (S K) of Alg. 1
    (sketch entries 1/sqrt(P(j) s)).  The product is taken in mode order,
    one IEEE operation at a time.
    """
    idx, acc = _product_draws(tables, s, seed, counter, problem)
    return idx, acc / np.float64(s)


#: Philox block (counter word 3) of the augmented distribution's branch draws;
#: blocks 0 and 1 drive the modes (orders up to 8).
AUG_BLOCK = 2


def coin_weights(d, d_eff_lower, q_bits=Q_BITS):
    """Integer weights of the two branches of D(l, d'_eff): the data rows
    (total mass d after normalisation) get D = 2^Q, the d ridge rows (total
    mass d c) get C = ceil(c 2^Q), so a draw is a ridge row with probability
    C / (D + C) ~ c / (1 + c)."""
    c = ridge_row_mass(d, d_eff_lower)
    return 2 ** q_bits, int(math.ceil(c * float(2 ** q_bits)))


def sample_augmented(tables, ranks, s, seed, counter, d_eff_lower=0.0, problem=0,
                     q_bits=Q_BITS):
    """s i.i.d. draws from the augmented distribution D(l, d'_eff) of Alg. 1.

    Each draw first flips the branch coin (Sec. 3: branch on the two index
    subsets, then sample the conditional): with the Philox words of block
    AUG_BLOCK, u = floor(r_0 (D + C) / 2^64) < D picks a data row, drawn from
    the product distribution exactly as ``sample`` draws it; otherwise ridge
    row k = floor(r_1 d / 2^64), uniform over the d rows sqrt(lam) e_k.
    A ridge draw is stored as idx[n][t] = I_n + k_n, the digits k_n of k
    (row-major over the ranks).  weight_t = 1 / (s P(j_t)):
      data:  ((prod_n W_n / w_{i_n}) * ((D + C) / D)) / s
      ridge: (((D + C) / C) * d) / s
    each factor one IEEE operation, in this order.
    """
    N = len(tables)
    dims = [len(C) for _, C in tables]
    d = int(np.prod(ranks))
    D, Cw = coin_weights(d, d_eff_lower, q_bits)
    idx, acc = _product_draws(tables, s, seed, counter, problem)
    t = np.arange(s, dtype=np.uint64)
    words = philox4x64(t, np.uint64(counter), np.uint64(problem), np.uint64(AUG_BLOCK), seed, 0)
    u = mulhi64(words[0], np.uint64(D + Cw))
    ridge = u >= np.uint64(D)
    k = mulhi64(words[1], np.uint64(d)).astype(np.int64)
    rem = k.copy()
    for n in range(N - 1, -1, -1):
        dig = rem % ranks[n]
        rem //= ranks[n]
        idx[n] = np.where(ridge, dims[n] + dig, idx[n]).astype(np.int32)
    w_data = (acc * (np.float64(D + Cw) / np.float64(D))) / np.float64(s)
    w_ridge = ((np.float64(D + Cw) / np.float64(Cw)) * np.float64(d)) / np.float64(s) if Cw else 0.0
    weight = np.where(ridge, w_ridge, w_data)
    return idx, weight


def sampling_probabilities(tables, idx):
    """P(row t) = prod_n w_{i_n} / W_n, the probability each sample was drawn with."""
    p = np.ones(np.asarray(idx).shape[1])
    for n, (w, C) in enumerate(tables):
        p = p * (w[idx[n]].astype(np.float64) / np.float64(C[-1]))
    return p


# --------------------------------------------------------------------------
# True lambda-ridge leverage scores of K (Sec. 2 SVD form; Sec. 4.1): a mixture
# over the tuples of singular values, sampled without forming K
# --------------------------------------------------------------------------

#: Philox block (counter word 3) of the tuple draw of the ridge-score sampler.
RIDGE_BLOCK = 3


def ridge_tables(factors, lam, q_bits=Q_BITS):
    """Integer tables of the ridge-score mixture of K = A(1) (x) ... (x) A(N).

    With the SVDs A(n) = U_n S_n V_n^T, K's ridge scores are
      l_i^lam(K) = sum_t pi_t prod_n U_n[i_n, t_n]^2,
      pi_t = prod_n s_{n,t_n}^2 / (prod_n s_{n,t_n}^2 + lam)
    (the SVD form of the ridge score applied to K's SVD (x)U_n (x)S_n (x)V_n),
    a mixture over tuples t (row-major over the ranks) of product distributions
    whose mode-n factor is column t_n of U_n squared (columns have unit norm).
    Returns (tuple table (w, C) over the d tuples with w_t = ceil(pi_t 2^Q),
    list over modes of lists over columns c of (w, C) with
    w_i = ceil(U_n[i, c]^2 2^Q), and d_eff = sum_t pi_t).
    """
    Us, S2 = [], []
    for A in factors:
        U, sv, _ = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
        Us.append(U)
        S2.append(sv ** 2)
    prod = np.ones(1)
    for s2 in S2:
        prod = np.kron(prod, s2)
    pi = prod / (prod + lam)
    tuple_tab = cdf_table(pi, q_bits)
    cols = [[cdf_table(U[:, c] ** 2, q_bits) for c in range(U.shape[1])] for U in Us]
    return tuple_tab, cols, float(pi.sum())


def ridge_mixture_probabilities(tuple_tab, cols, ranks, idx):
    """P(row i) of the quantised mixture, sum_t (w_t / W) prod_n w_{n,t_n,i_n} / W_{n,t_n},
    for every column of idx (a sum over all d tuples)."""
    idx = np.asarray(idx)
    wt, Ct = tuple_tab
    W = float(Ct[-1])
    P = np.zeros(idx.shape[1])
    for t in range(len(wt)):
        rem, dig = t, []
        for R in reversed(ranks):
            dig.append(rem % R)
            rem //= R
        dig = dig[::-1]
        term = np.full(idx.shape[1], float(wt[t]) / W)
        for n, c in enumerate(dig):
            w, C = cols[n][c]
            term = term * (w[idx[n]].astype(np.float64) / float(C[-1]))
        P += term
    return P


def sample_ridge(tuple_tab, cols, ranks, s, seed, counter, problem=0, d_eff_lower=None,
                 q_bits=Q_BITS):
    """s i.i.d. draws from the ridge-score mixture.

    Per draw: the tuple t from the tuple table with word 0 of Philox block
    RIDGE_BLOCK (u = floor(r W / 2^64), first t with C_t > u); then mode n's row
    from the table of column t_n of U_n with the word that drives mode n in
    ``sample`` (block n // 4, word n % 4), by the same inverse-CDF search.
    weight_t = 1 / (s P(row t)) with P from ``ridge_mixture_probabilities``.
    With ``d_eff_lower`` the draws are those of the augmented distribution of
    Alg. 1 with these scores as the overestimate: the branch coin of
    ``sample_augmented`` (same words) replaces a draw by a ridge row, and data
    weights are multiplied by (D + C) / D.
    """
    N = len(cols)
    t = np.arange(s, dtype=np.uint64)
    wt, Ct = tuple_tab
    tw = philox4x64(t, np.uint64(counter), np.uint64(problem), np.uint64(RIDGE_BLOCK), seed, 0)
    tup = np.searchsorted(Ct, mulhi64(tw[0], np.uint64(Ct[-1])), side="right").astype(np.int64)
    digits = []
    rem = tup.copy()
    for n in range(N - 1, -1, -1):
        digits.append(rem % ranks[n])
        rem //= ranks[n]
    digits = digits[::-1]
    idx = np.empty((N, s), dtype=np.int32)
    for b in range((N + 3) // 4):
        words = philox4x64(t, np.uint64(counter), np.uint64(problem), np.uint64(b), seed, 0)
        for j in range(4):
            n = 4 * b + j
            if n >= N:
                break
            for c in range(ranks[n]):
                sel = digits[n] == c
                if not sel.any():
                    continue
                w, C = cols[n][c]
                u = mulhi64(words[j][sel], np.uint64(C[-1]))
                idx[n, sel] = np.searchsorted(C, u, side="right")
    P = ridge_mixture_probabilities(tuple_tab, cols, ranks, idx)
    weight = 1.0 / (float(s) * P)
    if d_eff_lower is None:
        return idx, weight
    dims = [len(colt[0][1]) for colt in cols]
    d = int(np.prod(ranks))
    D, Cw = coin_weights(d, d_eff_lower, q_bits)
    words = philox4x64(t, np.uint64(counter), np.uint64(problem), np.uint64(AUG_BLOCK), seed, 0)
    ridge = mulhi64(words[0], np.uint64(D + Cw)) >= np.uint64(D)
    k = mulhi64(words[1], np.uint64(d)).astype(np.int64)
    for n in range(N - 1, -1, -1):
        idx[n] = np.where(ridge, dims[n] + k % ranks[n], idx[n]).astype(np.int32)
        k //= ranks[n]
    w_ridge = ((np.float64(D + Cw) / np.float64(Cw)) * np.float64(d)) / np.float64(s) if Cw else 0.0
    weight = np.where(ridge, w_ridge, weight * (float(D + Cw) / float(D)))
    return idx, weight


# --------------------------------------------------------------------------
# Sketched core update (Alg. 3 -> Alg. 1, normal equations as in the proof
# of Thm 4.2; ridge handled as Gram + lam I)
# --------------------------------------------------------------------------

def sampled_entries(X, idx, mask=None):
    """x_t = X[idx_t] and the observed flag of each sample."""
    X = np.asarray(X)
    flat = flat_index(idx, X.shape)
    x = X.reshape(-1)[flat].astype(np.float64)
    obs = np.ones(flat.shape, dtype=bool) if mask is None else mask_lookup(mask, flat)
    return x, obs


def sketched_normal_equations(X, factors, idx, weight, mask=None, chunk=8192):
    """Sketched Gram sum_t w_t k_t k_t^T and right side sum_t w_t x_t k_t.

    Samples that hit a missing entry contribute nothing (they keep their
    weight, so both sums stay unbiased for the observed-only design).
    """
    x, obs = sampled_entries(X, idx, mask)
    idx = np.asarray(idx)
    weight = np.asarray(weight, dtype=np.float64)
    d = int(np.prod([A.shape[1] for A in factors]))
    gram = np.zeros((d, d))
    rhs = np.zeros(d)
    s = idx.shape[1]
    for a in range(0, s, chunk):
        b = min(s, a + chunk)
        keep = obs[a:b]
        rows = kron_rows(factors, idx[:, a:b][:, keep])
        wk = weight[a:b][keep]
        gram += (rows * wk[:, None]).T @ rows
        rhs += rows.T @ (wk * x[a:b][keep])
    return gram, rhs


def core_update_sketched(X, factors, lam, idx, weight, mask=None):
    """Sketched ridge solve (Gram + lam I) g = rhs by Cholesky; returns G (R1..RN)."""
    gram, rhs = sketched_normal_equations(X, factors, idx, weight, mask)
    d = gram.shape[0]
    L = np.linalg.cholesky(gram + lam * np.eye(d))
    g = np.linalg.solve(L.T, np.linalg.solve(L, rhs))
    return g.reshape([A.shape[1] for A in factors])


def augmented_rows(X, factors, lam, idx, mask=None):
    """Rows of the augmented design [K; sqrt(lam) I] and response [vec X; 0] at
    the draws idx of ``sample_augmented`` (Alg. 1 line Abar, bbar): data draws
    give (k_t, x_t), with x_t = 0 and k_t = 0 on unobserved entries (they
    contribute nothing); ridge draws give (sqrt(lam) e_k, 0)."""
    X = np.asarray(X)
    idx = np.asarray(idx)
    dims = X.shape
    ranks = [A.shape[1] for A in factors]
    d = int(np.prod(ranks))
    s = idx.shape[1]
    ridge = idx[0] >= dims[0]
    rows = np.zeros((s, d))
    x = np.zeros(s)
    data = np.nonzero(~ridge)[0]
    if len(data):
        xd, obs = sampled_entries(X, idx[:, data], mask)
        rows[data] = kron_rows(factors, idx[:, data]) * obs[:, None]
        x[data] = xd * obs
    rid = np.nonzero(ridge)[0]
    if len(rid):
        k = np.zeros(len(rid), dtype=np.int64)
        for n in range(len(dims)):
            k = k * ranks[n] + (idx[n, rid].astype(np.int64) - dims[n])
        rows[rid, k] = math.sqrt(lam)
    return rows, x


def core_update_sketched_augmented(X, factors, lam, idx, weight, mask=None):
    """Alg. 1's solve on augmented draws: argmin_g ||S Abar g - S bbar||^2 by its
    normal equations (sum_t w_t abar_t abar_t^T) g = sum_t w_t bbar_t abar_t
    (Cholesky); the ridge enters only through the sampled rows sqrt(lam) e_k."""
    rows, x = augmented_rows(X, factors, lam, idx, mask)
    w = np.asarray(weight, dtype=np.float64)
    gram = (rows * w[:, None]).T @ rows
    rhs = rows.T @ (w * x)
    L = np.linalg.cholesky(gram)
    g = np.linalg.solve(L.T, np.linalg.solve(L, rhs))
    return g.reshape([A.shape[1] for A in factors])


def fast_core_tensor_update_augmented(X, factors, lam, s, seed, counter, d_eff_lower=0.0,
                                      mask=None, problem=0, q_bits=Q_BITS):
    """Alg. 3 with Alg. 1 taken literally: factor leverage scores as the
    overestimate, draws from the augmented distribution, solve on S Abar."""
    tables = [cdf_table(leverage_scores(A), q_bits) for A in factors]
    ranks = [A.shape[1] for A in factors]
    idx, weight = sample_augmented(tables, ranks, s, seed, counter, d_eff_lower, problem, q_bits)
    G = core_update_sketched_augmented(X, factors, lam, idx, weight, mask)
    return G, idx, weight, tables


def fast_core_tensor_update(X, factors, lam, s, seed, counter, mask=None, problem=0,
                            q_bits=Q_BITS):
    """Alg. 3 end to end: factor leverage scores, product sampler, sketched solve
    (sampling tables with q_bits fixed-point bits)."""
    tables = [cdf_table(leverage_scores(A), q_bits) for A in factors]
    idx, weight = sample(tables, s, seed, counter, problem)
    G = core_update_sketched(X, factors, lam, idx, weight, mask)
    return G, idx, weight, tables


def sketched_objective_excess(g, g_star, factors, lam):
    """(g - g*)^T (K^T K + lam I) (g - g*), computed through the Kronecker Gram.

    For a ridge problem f(g) - f(g*) equals exactly this quadratic form, so the
    (1+eps) bound of Thm 3.4 can be checked without cancellation.
    """
    e = np.asarray(g, dtype=np.float64) - np.asarray(g_star, dtype=np.float64)
    Ce = e
    for n, A in enumerate(factors):
        A = np.asarray(A, dtype=np.float64)
        Ce = mode_product(Ce, A.T @ A, n)
    return float(np.sum(e * Ce) + lam * np.sum(e * e))


def ridge_objective(X, G, factors, lam, mask=None):
    """||K vec G - vec X||^2 (observed entries) + lam ||G||^2 (Alg. 2 core step)."""
    R = np.asarray(X, dtype=np.float64) - reconstruct(G, factors)
    if mask is not None:
        R = R * unpack_mask(mask, R.shape)
    return float(np.sum(R * R) + lam * np.sum(np.asarray(G, dtype=np.float64) ** 2))


# --------------------------------------------------------------------------
# Exact core update (Alg. 2 core step), eigen form from the proof of Lemma 4.1:
#   K^T K + lam I = (x V_n) ((x) Lambda_n + lam I) (x V_n)^T
# --------------------------------------------------------------------------

def _kron_eigs(factors):
    evals, vecs = [], []
    for A in factors:
        A = np.asarray(A, dtype=np.float64)
        e, V = np.linalg.eigh(A.T @ A)
        evals.append(e)
        vecs.append(V)
    D = np.ones(())
    for e in evals:
        D = np.multiply.outer(D, e)
    return D, vecs


def apply_inverse_kron_gram(T, factors, lam):
    """(K^T K + lam I)^{-1} applied to a core-shaped tensor T."""
    D, vecs = _kron_eigs(factors)
    B = np.asarray(T, dtype=np.float64)
    for n, V in enumerate(vecs):
        B = mode_product(B, V.T, n)
    B = B / (D + lam)
    for n, V in enumerate(vecs):
        B = mode_product(B, V, n)
    return B


def core_update_exact(X, factors, lam):
    """argmin_G ||K vec G - vec X||^2 + lam ||G||^2 for a fully observed X."""
    B = np.asarray(X, dtype=np.float64)
    for n, A in enumerate(factors):
        B = mode_product(B, np.asarray(A, dtype=np.float64).T, n)  # K^T vec X
    return apply_inverse_kron_gram(B, factors, lam)


def core_update_exact_masked(X, factors, lam, mask, tol=1e-12, maxit=1000):
    """Exact core update over observed entries only.

    The paper's experiments are fully observed; for a masked tensor this solves
    (K~^T K~ + lam I) g = K~^T x~ by conjugate gradients with the matrix-free
    product v -> K^T (M o (K v)) + lam v, preconditioned by the unmasked
    (K^T K + lam I)^{-1}.
    """
    Mk = unpack_mask(mask, np.asarray(X).shape).astype(np.float64)
    Xm = np.asarray(X, dtype=np.float64) * Mk

    def KT(T):
        for n, A in enumerate(factors):
            T = mode_product(T, np.asarray(A, dtype=np.float64).T, n)
        return T

    def op(v):
        return KT(reconstruct(v, factors) * Mk) + lam * v

    b = KT(Xm)
    x = apply_inverse_kron_gram(b, factors, lam)
    r = b - op(x)
    z = apply_inverse_kron_gram(r, factors, lam)
    p = z.copy()
    rz = np.sum(r * z)
    bn = np.linalg.norm(b)
    for _ in range(maxit):
        if np.linalg.norm(r) <= tol * bn:
            break
        Ap = op(p)
        alpha = rz / np.sum(p * Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = apply_inverse_kron_gram(r, factors, lam)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


# --------------------------------------------------------------------------
# Factor update (Alg. 2 inner loop): row-wise ridge with
#   K_n = G_(n) (x_{m != n} A(m))^T,   A(n) = X_(n) K_n^T (K_n K_n^T + lam I)^{-1}
# --------------------------------------------------------------------------

def factor_update(X, G, factors, n, lam):
    """New A(n) for a fully observed X; X_(n) K_n^T and K_n K_n^T via mode products."""
    W = np.asarray(X, dtype=np.float64)
    C = np.ones((1, 1))
    for m, A in enumerate(factors):
        if m == n:
            continue
        A = np.asarray(A, dtype=np.float64)
        W = mode_product(W, A.T, m)
        C = np.kron(C, A.T @ A)
    Gn = unfold(np.asarray(G, dtype=np.float64), n)
    rhs = unfold(W, n) @ Gn.T              # X_(n) K_n^T  (I_n x R_n)
    KKt = Gn @ C @ Gn.T                    # K_n K_n^T    (R_n x R_n)
    Rn = KKt.shape[0]
    return np.linalg.solve(KKt + lam * np.eye(Rn), rhs.T).T


def factor_update_masked(X, G, factors, n, lam, mask, rows=None):
    """New A(n) over the observed entries only: row i solves
        a_i = argmin_y sum_{j observed in row i} (x_(n),ij - y . k_j)^2 + lam ||y||^2,
    k_j the column j of K_n = G_(n) ((x)_{m != n} A(m))^T (Alg. 2 factor step,
    restricted to the observed entries as in the tensor completion setting of
    Sec. 4.2).  K_n is formed as the mode-n unfolding of G multiplied by every
    factor but A(n).  ``rows`` (optional) limits the result to those rows (the
    other rows of the returned matrix are NaN).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(G, dtype=np.float64)
    for m, A in enumerate(factors):
        if m != n:
            Y = mode_product(Y, np.asarray(A, dtype=np.float64), m)
    Kn = unfold(Y, n)                       # R_n x prod_{m != n} I_m
    B = unfold(X, n)
    obs = unfold(unpack_mask(mask, X.shape), n)
    Rn = Kn.shape[0]
    out = np.full((X.shape[n], Rn), np.nan)
    for i in (range(X.shape[n]) if rows is None else rows):
        Ko = Kn[:, obs[i]]
        out[i] = np.linalg.solve(Ko @ Ko.T + lam * np.eye(Rn), Ko @ B[i, obs[i]])
    return out


# --------------------------------------------------------------------------
# Loss (Sec. 2) and RMSE
# --------------------------------------------------------------------------

def loss(X, G, factors, lam, mask=None):
    """(L, rmse): L = ||X - Xhat||_F^2 + lam(||G||^2 + sum ||A(n)||^2); rmse over observed entries."""
    R = np.asarray(X, dtype=np.float64) - reconstruct(G, factors)
    count = R.size
    if mask is not None:
        Mk = unpack_mask(mask, R.shape)
        R = R * Mk
        count = int(Mk.sum())
    sq = float(np.sum(R * R))
    reg = float(np.sum(np.asarray(G, dtype=np.float64) ** 2))
    reg += sum(float(np.sum(np.asarray(A, dtype=np.float64) ** 2)) for A in factors)
    return sq + lam * reg, math.sqrt(sq / max(count, 1))


# --------------------------------------------------------------------------
# ALS (Alg. 2), exact or with the sampled core update of Alg. 3
# --------------------------------------------------------------------------

def als(X, G0, factors0, lam, iters, core="exact", s=None, seed=0, record=None):
    """Alg. 2 from a given initial state; ``core`` is "exact" or "sketched".

    Per iteration: update A(1)..A(N) in order, then the core.  The sketched core
    update of iteration k uses sampling counter k.  Returns (G, factors, history)
    where history holds (loss, rmse) after every core update.
    """
    G = np.asarray(G0, dtype=np.float64).copy()
    factors = [np.asarray(A, dtype=np.float64).copy() for A in factors0]
    hist = []
    for it in range(iters):
        for n in range(len(factors)):
            factors[n] = factor_update(X, G, factors, n, lam)
            if record is not None:
                record.append(("factor", it, n, loss(X, G, factors, lam)))
        if core == "exact":
            G = core_update_exact(X, factors, lam)
        else:
            G, _, _, _ = fast_core_tensor_update(X, factors, lam, s, seed, it)
        hist.append(loss(X, G, factors, lam))
        if record is not None:
            record.append(("core", it, -1, hist[-1]))
    return G, factors, hist


# --------------------------------------------------------------------------
# Adjoint of the sketched solve with the sample set frozen (not in the paper)
# --------------------------------------------------------------------------

def sketched_adjoint(X, factors, lam, idx, weight, g_bar, mask=None):
    """Gradients of <g_bar, g> w.r.t. the factors and the tensor entries.

    g solves (sum_t w_t k_t k_t^T + lam I) g = sum_t w_t x_t k_t with (idx, w)
    held fixed (the sketch is treated as a constant operator).  With
    v = M^{-1} g_bar:
      d/dx_t = w_t (k_t . v)                       (observed samples, summed over duplicates)
      d/dk_t = w_t [ (x_t - k_t . g) v - (k_t . v) g ]
    and d/dA(n)[i_n, :] collects d/dk_t contracted with the other modes' rows.
    Returns (factor_bars, X_bar dense, g).
    """
    X = np.asarray(X)
    gram, rhs = sketched_normal_equations(X, factors, idx, weight, mask)
    d = gram.shape[0]
    M = gram + lam * np.eye(d)
    g = np.linalg.solve(M, rhs)
    v = np.linalg.solve(M, np.asarray(g_bar, dtype=np.float64).reshape(-1))
    x, obs = sampled_entries(X, idx, mask)
    idx = np.asarray(idx)
    rows_all = kron_rows(factors, idx)
    w = np.asarray(weight, dtype=np.float64) * obs
    kv = rows_all @ v
    kg = rows_all @ g
    Xbar = np.zeros(X.size)
    np.add.at(Xbar, flat_index(idx, X.shape), w * kv)
    kbar = w[:, None] * ((x - kg)[:, None] * v[None, :] - kv[:, None] * g[None, :])
    ranks = [A.shape[1] for A in factors]
    T = kbar.reshape([idx.shape[1]] + ranks)
    rows = [np.asarray(A, dtype=np.float64)[idx[m]] for m, A in enumerate(factors)]
    bars = []
    for n, A in enumerate(factors):
        Tn = T
        # contract modes m != n, highest first, so lower axis numbers are unchanged
        for m in reversed(range(len(factors))):
            if m == n:
                continue
            Tn = np.einsum("t...r,tr->t...", np.moveaxis(Tn, 1 + m, -1), rows[m])
        # Tn now has shape (s, R_n)
        Ab = np.zeros(np.asarray(A).shape)
        np.add.at(Ab, idx[n], Tn)
        bars.append(Ab)
    return bars, Xbar.reshape(X.shape), g.reshape(ranks)


def exact_adjoint(X, factors, lam, g_bar):
    """Gradients of <g_bar, g*> for the exact solve g* = (K^T K + lam I)^{-1} K^T x.

    With v = (K^T K + lam I)^{-1} g_bar:  X_bar = K v (a full tensor) and
    A_bar(n) = X_(n) (x_{m!=n} A(m)) V_(n)^T
               - A(n) [G_(n) (x_{m!=n} C_m) V_(n)^T + V_(n) (x_{m!=n} C_m) G_(n)^T],
    C_m = A(m)^T A(m), G = g*, V = v as core-shaped tensors.
    """
    X = np.asarray(X, dtype=np.float64)
    G = core_update_exact(X, factors, lam)
    V = apply_inverse_kron_gram(np.asarray(g_bar, dtype=np.float64).reshape(G.shape), factors, lam)
    Xbar = reconstruct(V, factors)
    bars = []
    for n, A in enumerate(factors):
        A = np.asarray(A, dtype=np.float64)
        W = X
        C = np.ones((1, 1))
        for m, B in enumerate(factors):
            if m == n:
                continue
            B = np.asarray(B, dtype=np.float64)
            W = mode_product(W, B.T, m)
            C = np.kron(C, B.T @ B)
        Gn, Vn = unfold(G, n), unfold(V, n)
        bars.append(unfold(W, n) @ Vn.T - A @ (Gn @ C @ Vn.T + Vn @ C @ Gn.T))
    return bars, Xbar, G


def normal_equation_residual(X, factors, lam, idx, weight, G, mask=None, chunk=4096):
    """Relative residual ||sum_t w_t k_t (x_t - k_t.g) - lam g|| / ||sum_t w_t x_t k_t||.

    Zero exactly when G solves the sketched ridge normal equations of the given
    samples; computed matrix-free in chunks, so it scales to large d and s.
    """
    x, obs = sampled_entries(X, idx, mask)
    idx = np.asarray(idx)
    w = np.asarray(weight, dtype=np.float64) * obs
    g = np.asarray(G, dtype=np.float64).reshape(-1)
    r = -lam * g
    b = np.zeros_like(g)
    for a in range(0, idx.shape[1], chunk):
        e = min(idx.shape[1], a + chunk)
        rows = kron_rows(factors, idx[:, a:e])
        b += rows.T @ (w[a:e] * x[a:e])
        r += rows.T @ (w[a:e] * (x[a:e] - rows @ g))
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def normal_equation_residual_augmented(X, factors, lam, idx, weight, G, mask=None, chunk=4096):
    """Relative residual ||sum_t w_t abar_t (bbar_t - abar_t . g)|| / ||sum_t w_t bbar_t abar_t||
    of Alg. 1's normal equations on augmented draws (rows from ``augmented_rows``);
    zero exactly when G solves them.  Computed in chunks of draws."""
    idx = np.asarray(idx)
    w = np.asarray(weight, dtype=np.float64)
    g = np.asarray(G, dtype=np.float64).reshape(-1)
    r = np.zeros_like(g)
    b = np.zeros_like(g)
    for a in range(0, idx.shape[1], chunk):
        e = min(idx.shape[1], a + chunk)
        rows, x = augmented_rows(X, factors, lam, idx[:, a:e], mask)
        b += rows.T @ (w[a:e] * x)
        r += rows.T @ (w[a:e] * (x - rows @ g))
    return float(np.linalg.norm(r) / np.linalg.norm(b))

