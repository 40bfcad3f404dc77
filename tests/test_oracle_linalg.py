"""Pins for the oracle's leverage scores, solves, factor update, loss and ALS.

Each pin checks the oracle against a fact the paper or the mathematics fixes,
through a route that does not reuse the oracle's own formula:
* scores sum to the rank and lie in [0, 1] (Sec. 2, eq. d_eff_def and the SVD form);
* definition (pseudo-inverse) equals the SVD form (eq. ridge_leverage_score_svd_def)
  and QR leverage;
* Lemma 3.1: ridge scores of A equal leverage scores of the augmented matrix;
* Lemma 4.1: leverage (and cross) scores of an explicit np.kron product equal the
  product of factor scores; the ridge version equals its factor-SVD formula;
* Lemma 4.4 (sum of squared cross scores), Thm 4.3 and Cor. B.1 bounds;
* sketched solve equals least squares on the explicitly built sketch [S K; sqrt(lam) I];
* exact core update (eigen form of the proof of Lemma 4.1) equals a dense solve
  with explicit K; masked PCG equals the dense masked solve;
* factor update equals row-by-row least squares with explicit K_n (Alg. 2);
* Tucker reconstruction equals the elementwise sum (eq. tucker_decomposition_elementwise)
  and K vec(G);
* exact ALS never increases the loss (each step minimises it over one block);
* the Sec. 5 generator fitted at its true rank reaches the 0.10 RMSE noise floor;
* the (1+eps) cost bound of Thm 3.4 holds empirically at the Alg. 1 sample count.
"""
import itertools

import math

import numpy as np
import pytest

import oracle
import workloads


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ---------------------------------------------------------------- scores

@pytest.mark.parametrize("shape", [(30, 4), (7, 7), (100, 12), (13, 1)])
def test_scores_sum_to_rank_and_bounds(shape):
    A = rand(shape, 1)
    l = oracle.leverage_scores(A)
    assert abs(l.sum() - shape[1]) < 1e-11
    assert l.min() > -1e-14 and l.max() < 1 + 1e-12
    Q, _ = np.linalg.qr(A)
    np.testing.assert_allclose(l, (Q ** 2).sum(1), atol=1e-13)


def test_rank_deficient_scores_sum_to_rank():
    A = rand((25, 4), 2)
    A[:, 3] = A[:, 1]
    assert oracle.is_rank_deficient(A)
    l = oracle.leverage_scores(A)
    assert abs(l.sum() - 3) < 1e-10
    assert not oracle.is_rank_deficient(rand((25, 4), 3))


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.5, 10.0])
def test_ridge_definition_equals_svd_form(lam):
    A = rand((40, 6), 4) * np.array([10, 3, 1, 0.3, 0.1, 0.01])
    np.testing.assert_allclose(oracle.ridge_leverage_scores(A, lam),
                               oracle.ridge_scores_svd(A, lam), rtol=1e-9, atol=1e-13)
    l0 = oracle.leverage_scores(A)
    llam = oracle.ridge_leverage_scores(A, lam)
    assert (llam <= l0 + 1e-12).all() and (llam >= -1e-14).all()
    deff = oracle.effective_dimension(A, lam)
    assert deff <= 6 + 1e-9
    if lam == 0.0:
        assert abs(deff - 6) < 1e-9


@pytest.mark.parametrize("lam", [1e-3, 0.7])
def test_lemma_3_1_augmented_design(lam):
    A = rand((20, 5), 5)
    Abar = np.vstack([A, np.sqrt(lam) * np.eye(5)])
    Q, _ = np.linalg.qr(Abar)
    np.testing.assert_allclose(oracle.ridge_leverage_scores(A, lam), (Q ** 2).sum(1)[:20],
                               atol=1e-13)


def test_lemma_4_1_kronecker_product_law():
    factors = [rand((6, 2), 6), rand((5, 3), 7), rand((4, 2), 8)]
    K = oracle.kron_matrix(factors)
    Q, _ = np.linalg.qr(K)
    lK = (Q ** 2).sum(1)
    prod = np.ones(())
    for A in factors:
        prod = np.multiply.outer(prod, oracle.leverage_scores(A))
    np.testing.assert_allclose(lK, prod.reshape(-1), atol=1e-13)
    # cross scores factor as well
    LK = Q @ Q.T
    Lf = [oracle.cross_ridge_scores(A) for A in factors]
    rng = np.random.default_rng(0)
    for _ in range(50):
        i = [rng.integers(A.shape[0]) for A in factors]
        j = [rng.integers(A.shape[0]) for A in factors]
        fi = np.ravel_multi_index(i, [A.shape[0] for A in factors])
        fj = np.ravel_multi_index(j, [A.shape[0] for A in factors])
        assert abs(LK[fi, fj] - np.prod([L[a, b] for L, a, b in zip(Lf, i, j)])) < 1e-13
    # the kron_rows query structure reproduces rows of K
    idx = np.array([[0, 5, 3], [4, 1, 2], [3, 0, 1]])
    flat = np.ravel_multi_index(tuple(idx), [6, 5, 4])
    np.testing.assert_allclose(oracle.kron_rows(factors, idx), K[flat], atol=0)


def test_lemma_4_1_ridge_scores_of_kronecker():
    lam = 0.05
    factors = [rand((5, 2), 9), rand((4, 3), 10)]
    K = oracle.kron_matrix(factors)
    LK = oracle.cross_ridge_scores(K, lam)
    svds = [np.linalg.svd(A, full_matrices=False) for A in factors]
    # sum over singular tuples of prod sigma^2 / (prod sigma^2 + lam) * prod u_i u_j
    F = np.zeros_like(LK)
    for t in itertools.product(*[range(len(s)) for _, s, _ in svds]):
        s2 = np.prod([svds[n][1][t[n]] ** 2 for n in range(2)])
        u = np.kron(svds[0][0][:, t[0]], svds[1][0][:, t[1]])
        F += s2 / (s2 + lam) * np.outer(u, u)
    np.testing.assert_allclose(LK, F, atol=1e-12)


@pytest.mark.parametrize("lam", [0.0, 1e-2, 1.0])
def test_lemma_4_4_sum_of_squared_cross_scores(lam):
    A = rand((15, 4), 11)
    L = oracle.cross_ridge_scores(A, lam)
    l = np.diag(L)
    sq = (L ** 2).sum(1)
    if lam == 0.0:
        np.testing.assert_allclose(sq, l, atol=1e-12)
    else:
        assert (sq < l).all()


def test_thm_4_3_and_cor_b1_removed_rows():
    lam = 0.1
    factors = [rand((5, 2), 12), rand((6, 2), 13)]
    K = oracle.kron_matrix(factors)
    L = oracle.cross_ridge_scores(K, lam)
    l = np.diag(L)
    rng = np.random.default_rng(3)
    bound_b1 = 1 + np.prod([np.linalg.norm(A, 2) ** 2 for A in factors]) / lam
    for _ in range(20):
        keep = rng.random(K.shape[0]) > 0.3
        S, Sb = np.where(keep)[0], np.where(~keep)[0]
        lt = oracle.ridge_leverage_scores(K[S], lam)
        lmax = np.linalg.eigvalsh(L[np.ix_(Sb, Sb)]).max()
        c = 1.0 / (1.0 - lmax)
        assert c <= bound_b1 + 1e-9
        for a, i in enumerate(S):
            ub = l[i] + c * np.sum(L[i, Sb] ** 2)
            assert lt[a] <= ub + 1e-10
            # exact update formula from the proof (Woodbury)
            v = L[i, Sb]
            exact = l[i] + v @ np.linalg.solve(np.eye(len(Sb)) - L[np.ix_(Sb, Sb)], v)
            assert abs(lt[a] - exact) < 1e-9


# ---------------------------------------------------------------- solves

def _tiny_problem(seed, dims=(6, 5, 4), ranks=(2, 3, 2), dtype="f64"):
    return workloads.tucker_tensor(dims, ranks, seed, dtype, factor="gaussian",
                                   noise=("sigma", 0.3))


def test_sketched_solve_equals_explicit_sketch_lstsq():
    p = _tiny_problem(20)
    X, F, lam = p["X"], p["factors_true"], 0.05
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tables, 300, seed=4, counter=2)
    G = oracle.core_update_sketched(X, F, lam, idx, w)
    # explicit S (s x n) with entries 1/sqrt(s P(j)), stacked with sqrt(lam) I
    K = oracle.kron_matrix(F)
    n, d = K.shape
    flat = np.ravel_multi_index(tuple(idx), X.shape)
    p_row = oracle.sampling_probabilities(tables, idx)
    S = np.zeros((idx.shape[1], n))
    S[np.arange(idx.shape[1]), flat] = 1.0 / np.sqrt(idx.shape[1] * p_row)
    Abar = np.vstack([S @ K, np.sqrt(lam) * np.eye(d)])
    bbar = np.concatenate([S @ X.reshape(-1), np.zeros(d)])
    ref = np.linalg.lstsq(Abar, bbar, rcond=None)[0]
    np.testing.assert_allclose(G.reshape(-1), ref, rtol=1e-9, atol=1e-11)


def test_masked_sketched_solve_equals_explicit():
    p = workloads.tucker_tensor((6, 5, 4), (2, 3, 2), 21, "f64", factor="gaussian",
                                noise=("sigma", 0.3), missing=0.3)
    X, F, lam, mask = p["X"], p["factors_true"], 0.05, p["mask"]
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tables, 400, seed=4, counter=2)
    G = oracle.core_update_sketched(X, F, lam, idx, w, mask)
    flat = np.ravel_multi_index(tuple(idx), X.shape)
    obs = oracle.unpack_mask(mask, X.shape).reshape(-1)[flat]
    K = oracle.kron_matrix(F)
    rows = K[flat[obs]] * np.sqrt(w[obs])[:, None]
    Abar = np.vstack([rows, np.sqrt(lam) * np.eye(K.shape[1])])
    bbar = np.concatenate([X.reshape(-1)[flat[obs]] * np.sqrt(w[obs]), np.zeros(K.shape[1])])
    ref = np.linalg.lstsq(Abar, bbar, rcond=None)[0]
    np.testing.assert_allclose(G.reshape(-1), ref, rtol=1e-9, atol=1e-11)
    assert (~obs).sum() > 50


def test_exact_core_equals_dense_solve():
    for seed, lam in [(30, 1e-3), (31, 0.5)]:
        p = _tiny_problem(seed)
        X, F = p["X"], p["factors_true"]
        K = oracle.kron_matrix(F)
        ref = np.linalg.solve(K.T @ K + lam * np.eye(K.shape[1]), K.T @ X.reshape(-1))
        np.testing.assert_allclose(oracle.core_update_exact(X, F, lam).reshape(-1), ref,
                                   rtol=1e-11, atol=1e-12)


def test_masked_exact_core_pcg():
    p = workloads.tucker_tensor((6, 5, 4), (2, 3, 2), 32, "f64", factor="gaussian",
                                noise=("sigma", 0.3), missing=0.25)
    X, F, mask, lam = p["X"], p["factors_true"], p["mask"], 1e-2
    K = oracle.kron_matrix(F)
    obs = oracle.unpack_mask(mask, X.shape).reshape(-1)
    Ko = K[obs]
    ref = np.linalg.solve(Ko.T @ Ko + lam * np.eye(K.shape[1]), Ko.T @ X.reshape(-1)[obs])
    got = oracle.core_update_exact_masked(X, F, lam, mask)
    np.testing.assert_allclose(got.reshape(-1), ref, rtol=1e-9, atol=1e-10)
    full = workloads.pack_mask(np.ones(X.shape, bool))
    np.testing.assert_allclose(oracle.core_update_exact_masked(X, F, lam, full),
                               oracle.core_update_exact(X, F, lam), rtol=1e-10, atol=1e-11)


def test_factor_update_equals_rowwise_lstsq():
    p = _tiny_problem(40, dims=(5, 6, 4), ranks=(2, 3, 2))
    X, F, lam = p["X"], p["factors_true"], 0.1
    G = rand((2, 3, 2), 41)
    for n in range(3):
        others = [F[m] for m in range(3) if m != n]
        Kn = oracle.unfold(G, n) @ oracle.kron_matrix(others).T     # R_n x prod_{m!=n} I_m
        B = oracle.unfold(X, n)
        Rn = Kn.shape[0]
        ref = np.zeros((X.shape[n], Rn))
        for i in range(X.shape[n]):
            M = np.vstack([Kn.T, np.sqrt(lam) * np.eye(Rn)])
            rhs = np.concatenate([B[i], np.zeros(Rn)])
            ref[i] = np.linalg.lstsq(M, rhs, rcond=None)[0]
        np.testing.assert_allclose(oracle.factor_update(X, G, F, n, lam), ref, rtol=1e-10,
                                   atol=1e-12)


def test_reconstruction_elementwise_and_kron():
    F = [rand((3, 2), 50), rand((4, 2), 51), rand((2, 3), 52)]
    G = rand((2, 2, 3), 53)
    Xh = oracle.reconstruct(G, F)
    for i in itertools.product(range(3), range(4), range(2)):
        v = 0.0
        for r in itertools.product(range(2), range(2), range(3)):
            v += G[r] * F[0][i[0], r[0]] * F[1][i[1], r[1]] * F[2][i[2], r[2]]
        assert abs(Xh[i] - v) < 1e-13
    np.testing.assert_allclose(oracle.kron_matrix(F) @ G.reshape(-1), Xh.reshape(-1), atol=1e-13)


def test_loss_at_truth_and_masked_count():
    p = workloads.tucker_tensor((7, 6, 5), (2, 2, 2), 60, "f64", factor="gaussian",
                                noise=("none",), missing=0.2)
    G, F, X, lam = p["G_true"], p["factors_true"], p["X"], 0.3
    L, rmse = oracle.loss(X, G, F, lam)
    reg = np.sum(G ** 2) + sum(np.sum(A ** 2) for A in F)
    assert abs(L - lam * reg) < 1e-9 and rmse < 1e-12
    Y = X + 1.0
    L2, rmse2 = oracle.loss(Y, G, F, 0.0, p["mask"])
    nobs = oracle.unpack_mask(p["mask"], X.shape).sum()
    assert abs(L2 - nobs) < 1e-9 and abs(rmse2 - 1.0) < 1e-12


def test_exact_als_loss_never_increases():
    p = _tiny_problem(70, dims=(8, 7, 6), ranks=(3, 2, 2))
    G0, F0 = workloads.als_init((8, 7, 6), (2, 2, 2), 1070)
    rec = []
    oracle.als(p["X"], G0, F0, 1e-2, 6, core="exact", record=rec)
    losses = [r[3][0] for r in rec]
    assert all(b <= a * (1 + 1e-12) + 1e-12 for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.5 * losses[0]


def test_table1_noise_floor():
    """Sec. 5: N(0,1) noise on 1 % of the entries puts the RMSE floor near 0.10."""
    p = workloads.table1_problem((48, 48, 48), seed=3, dtype="f64")
    G0, F0 = workloads.als_init((48, 48, 48), (8, 8, 8), 1003)
    _, _, hist = oracle.als(p["X"], G0, F0, 1e-3, 40, core="exact")
    rmse = hist[-1][1]
    # fitting a few noise directions puts the fit slightly below the floor
    assert 0.09 < rmse < 0.1005, rmse


def test_one_plus_eps_bound_thm_3_4():
    """At the Alg. 1 sample count, f(g~) <= (1+eps) f(g*) for at least 1-delta of the seeds."""
    eps = delta = 0.1
    p = workloads.tucker_tensor((10, 9, 8), (2, 2, 2), 80, "f64", factor="gaussian",
                                noise=("sigma", 1.0))
    X, F, lam = p["X"], p["factors_true"], 1e-3
    d = 8
    s = oracle.s_theory(d, eps, delta)
    g_star = oracle.core_update_exact(X, F, lam)
    f_star = oracle.ridge_objective(X, g_star, F, lam)
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    ok = 0
    ratios = []
    trials = 20
    for seed in range(trials):
        idx, w = oracle.sample(tables, s, seed=seed, counter=0)
        g = oracle.core_update_sketched(X, F, lam, idx, w)
        excess = oracle.sketched_objective_excess(g, g_star, F, lam)
        ratios.append(excess / f_star)
        ok += excess <= eps * f_star
    assert ok >= (1 - delta) * trials, ratios
    # the excess must shrink with more samples (a wrong weight would not)
    idx, w = oracle.sample(tables, 64, seed=0, counter=0)
    g = oracle.core_update_sketched(X, F, lam, idx, w)
    assert oracle.sketched_objective_excess(g, g_star, F, lam) > 10 * np.median(ratios) * f_star


def test_normal_equation_residual_pin():
    """Zero at the solution of the sketched normal equations, equal to the explicit
    ||(Gram + lam I) g - rhs|| / ||rhs|| elsewhere."""
    p = _tiny_problem(90)
    X, F, lam = p["X"], p["factors_true"], 0.02
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tables, 400, seed=3, counter=0)
    G = oracle.core_update_sketched(X, F, lam, idx, w)
    assert oracle.normal_equation_residual(X, F, lam, idx, w, G, chunk=97) < 1e-12
    Gp = G + 0.01 * np.random.default_rng(0).standard_normal(G.shape)
    rows = oracle.kron_matrix(F)[np.ravel_multi_index(tuple(idx), X.shape)]
    gram = (rows * w[:, None]).T @ rows + lam * np.eye(rows.shape[1])
    rhs = rows.T @ (w * X.reshape(-1)[np.ravel_multi_index(tuple(idx), X.shape)])
    ref = np.linalg.norm(gram @ Gp.reshape(-1) - rhs) / np.linalg.norm(rhs)
    assert abs(oracle.normal_equation_residual(X, F, lam, idx, w, Gp, chunk=97) - ref) < 1e-12


def test_table1_workload_sample_count_is_alg1():
    """The t1 / t1big workloads use Alg. 1's sample count for eps = delta = 0.1 at d = 4^3."""
    for name in ("t1", "t1big"):
        cfg = workloads.CONFIGS[name]
        d = int(np.prod(cfg["ranks"]))
        assert cfg["samples"] == oracle.s_theory(d, 0.1, 0.1), name


# ---------------------------------------------------------------- objective and mask pins

def test_ridge_objective_equals_explicit_kronecker_form():
    """ridge_objective is ||K vec G - vec X||^2 + lam ||G||^2 (Alg. 2 core step), with K
    built here by np.kron of the factors in mode order; with a mask the sum runs over
    the observed rows of K only (Sec. 4.2: missing entries remove rows of K)."""
    p = workloads.tucker_tensor((5, 4, 6), (2, 3, 2), 91, "f64", factor="gaussian",
                                noise=("sigma", 0.5), missing=0.3)
    X, F = p["X"], p["factors_true"]
    G = rand((2, 3, 2), 92)
    lam = 0.7
    K = np.kron(np.kron(F[0], F[1]), F[2])
    r = K @ G.reshape(-1) - X.reshape(-1)
    ref = float(r @ r + lam * np.sum(G * G))
    assert abs(oracle.ridge_objective(X, G, F, lam) - ref) <= 1e-12 * ref
    obs = np.zeros(X.size, dtype=bool)
    words = p["mask"]
    for e in range(X.size):  # bit e & 31 of word e >> 5, written out per entry
        obs[e] = (int(words[e // 32]) >> (e % 32)) & 1 == 1
    ro = r[obs]
    ref_m = float(ro @ ro + lam * np.sum(G * G))
    assert 0 < obs.sum() < X.size
    assert abs(oracle.ridge_objective(X, G, F, lam, mask=words) - ref_m) <= 1e-12 * ref_m


@pytest.mark.parametrize("lam", [0.0, 0.5, 3.0])
def test_objective_excess_equals_objective_difference(lam):
    """For the exact ridge minimiser g*, f(g) - f(g*) = (g - g*)^T (K^T K + lam I)(g - g*)
    exactly (a quadratic expanded at its minimiser), so sketched_objective_excess
    must equal the difference of two ridge_objective values; a dropped lam term,
    a missing factor or a transposed Gram shows up at these lam values."""
    p = _tiny_problem(93, dims=(6, 7, 5), ranks=(2, 3, 2))
    X, F = p["X"], p["factors_true"]
    g_star = oracle.core_update_exact(X, F, lam)
    f_star = oracle.ridge_objective(X, g_star, F, lam)
    for k in range(3):
        g = g_star + 0.3 * rand(g_star.shape, 94 + k)
        diff = oracle.ridge_objective(X, g, F, lam) - f_star
        exc = oracle.sketched_objective_excess(g, g_star, F, lam)
        assert diff > 0
        assert abs(exc - diff) <= 1e-9 * diff, (lam, exc, diff)


def test_mask_bit_order_and_pack_roundtrip():
    """Masks are LSB-first uint32 words: entry e is bit (e & 31) of word e >> 5.
    Hand-built words pin the bit order; a random mask with a ragged last word
    round-trips through the workload packer and the oracle's unpacker."""
    words = np.array([0b1011, 1 << 31, 0x1], dtype=np.uint32)
    flat = np.arange(65, dtype=np.int64)
    got = oracle.mask_lookup(words, flat)
    want = np.zeros(65, dtype=bool)
    want[[0, 1, 3, 63, 64]] = True
    assert np.array_equal(got, want)
    assert np.array_equal(workloads.pack_mask(want), words)
    rng = np.random.default_rng(95)
    for dims in [(5, 7, 3), (33,), (4, 4, 2)]:
        M = rng.random(dims) < 0.6
        packed = workloads.pack_mask(M)
        assert packed.size == (M.size + 31) // 32
        assert np.array_equal(oracle.unpack_mask(packed, dims), M)


# ---------------------------------------------------------------- masked factor update
def _row_design_by_reconstruction(G, F, n, i):
    """Design of row i of A(n) built from the model itself: column r is the
    slice i of the reconstruction with A(n) replaced by the unit matrix e_i e_r^T
    (independent of any unfolding or Kronecker ordering)."""
    cols = []
    for r in range(F[n].shape[1]):
        E = np.zeros_like(F[n])
        E[i, r] = 1.0
        Fe = [E if m == n else A for m, A in enumerate(F)]
        cols.append(np.take(oracle.reconstruct(G, Fe), i, axis=n).reshape(-1))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("dims,ranks", [((6, 5, 4), (2, 3, 2)), ((4, 5, 3, 3), (2, 2, 3, 2)),
                                        ((7, 6), (3, 2))])
def test_masked_factor_update_equals_rowwise_ridge_over_observed(dims, ranks):
    p = workloads.tucker_tensor(dims, ranks, 60, "f64", factor="gaussian", noise=("sigma", 0.3),
                                missing=0.3)
    X, F, lam, mask = p["X"], p["factors_true"], 0.07, p["mask"]
    G = rand(ranks, 61)
    obs = oracle.unpack_mask(mask, dims)
    for n in range(len(dims)):
        got = oracle.factor_update_masked(X, G, F, n, lam, mask)
        for i in range(dims[n]):
            D = _row_design_by_reconstruction(G, F, n, i)
            o = np.take(obs, i, axis=n).reshape(-1)
            x = np.take(X, i, axis=n).reshape(-1)
            M = np.vstack([D[o], np.sqrt(lam) * np.eye(ranks[n])])
            rhs = np.concatenate([x[o], np.zeros(ranks[n])])
            ref = np.linalg.lstsq(M, rhs, rcond=None)[0]
            np.testing.assert_allclose(got[i], ref, rtol=1e-9, atol=1e-11)


def test_masked_factor_update_special_cases():
    p = _tiny_problem(62, dims=(6, 5, 4), ranks=(2, 3, 2))
    X, F, lam = p["X"], p["factors_true"], 0.05
    G = rand((2, 3, 2), 63)
    full = workloads.pack_mask(np.ones(X.shape, bool))
    for n in range(3):
        np.testing.assert_allclose(oracle.factor_update_masked(X, G, F, n, lam, full),
                                   oracle.factor_update(X, G, F, n, lam), rtol=1e-10, atol=1e-12)
    # a row with no observed entry is pulled to zero by the ridge term alone
    obs = np.ones(X.shape, bool)
    obs[:, 2, :] = False
    A1 = oracle.factor_update_masked(X, G, F, 1, lam, workloads.pack_mask(obs))
    assert np.all(A1[2] == 0.0)
    # the update minimises the masked objective over A(n): moving any row off it
    # raises the loss
    obs = np.random.default_rng(64).random(X.shape) > 0.25
    mk = workloads.pack_mask(obs)
    A0 = oracle.factor_update_masked(X, G, F, 0, lam, mk)
    Fa = [A0, F[1], F[2]]
    base = oracle.loss(X, G, Fa, lam, mk)[0]
    rng = np.random.default_rng(65)
    for _ in range(5):
        Fb = [A0 + 1e-3 * rng.standard_normal(A0.shape), F[1], F[2]]
        assert oracle.loss(X, G, Fb, lam, mk)[0] > base


# ---------------------------------------------------------------- missing-data sample count
def test_masked_overestimate_chain():
    """Cor. B.1's bound dominates the exact 1/beta of Thm 4.3 for any mask; the
    exact value makes the K scores a beta-overestimate of the K~ ridge scores
    (each K~ score <= its K score / beta); for semi-orthogonal factors the bound
    is exactly 2 + 1/lam (the remark after Lemma 4.4)."""
    lam = 0.2
    F = [rand((5, 2), 91), rand((4, 2), 92), rand((3, 2), 93)]
    K = oracle.kron_matrix(F)
    lK = oracle.ridge_leverage_scores(K, lam)
    bound = oracle.masked_inverse_beta_bound(F, lam)
    rng = np.random.default_rng(94)
    for _ in range(10):
        obs = rng.random((5, 4, 3)) > 0.3
        mk = workloads.pack_mask(obs)
        ib = oracle.masked_inverse_beta(F, lam, mk)
        assert 2.0 <= ib <= bound + 1e-9
        keep = obs.reshape(-1)
        lt = oracle.ridge_leverage_scores(K[keep], lam)
        assert np.all(lt <= lK[keep] * ib + 1e-12)
    Q = [np.linalg.qr(rand((6, 3), 95 + n))[0] for n in range(3)]
    assert abs(oracle.masked_inverse_beta_bound(Q, 0.01) - (2.0 + 1.0 / 0.01)) < 1e-9


def test_masked_sample_count():
    a = max(420.0 * math.log(4.0 * 64 / 0.1), 1.0 / (0.1 * 0.1))
    assert oracle.s_theory_masked(64, 0.1, 0.1, 2.0) == math.ceil(4.0 * 64 * 2.0 * 2.0 * a)
    # inv_beta = 1 with c = 1 recovers the plain count
    assert oracle.s_theory_masked(64, 0.1, 0.1, 1.0) == oracle.s_theory(64, 0.1, 0.1)
