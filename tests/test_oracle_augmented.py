"""Pins for the oracle's literal Alg. 1: draws from the augmented distribution
D(l, d'_eff) of Sec. 3 and the solve on the sampled rows of [K; sqrt(lam) I].

Pins (each would catch a plausible mistake in the oracle):
* the branch probability equals its definition c / (1 + c), c = min{1, d - d'_eff},
  to the 2^-24 quantisation of the integer coin;
* draw frequencies: ridge fraction (binomial), ridge rows uniform over the d
  rows (chi-square), data rows following the product law (chi-square);
* every weight is 1 / (s P(j)) with P(j) recomputed independently from the
  tables and the coin weights (this plus the law of the draws makes the sketch
  unbiased: E[(S Abar)^T S Abar] = K^T K + lam I, also checked by Monte Carlo);
* the solve equals least squares on the explicit sketched matrix S Abar built
  from the Kronecker matrix (no normal equations);
* c = 0 reduces to the plain product sampler bit for bit;
* Thm 3.4's (1 + eps) bound holds at Alg. 1's sample count for this beta';
* the sample count reduces to the plain count at d'_eff = 0.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def _tables(dims, ranks, seed):
    F = workloads.random_factors(dims, ranks, seed, kind="gaussian")
    return F, [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]


@pytest.mark.parametrize("d,deff", [(8, 0.0), (8, 7.5), (8, 7.9), (64, 63.2), (4096, 4095.99),
                                    (8, 8.0), (8, 9.0)])
def test_branch_probability_matches_definition(d, deff):
    c = min(1.0, d - deff) if d - deff > 0 else 0.0
    D, C = oracle.coin_weights(d, deff)
    assert D == 2 ** 24
    assert abs(C / (D + C) - c / (1.0 + c)) <= 2.0 ** -24
    if deff == 0.0:
        assert C == D  # c = 1: each branch has probability 1/2 exactly


def test_augmented_draw_frequencies():
    dims, ranks = (5, 4, 3), (2, 2, 1)
    F, tabs = _tables(dims, ranks, 3)
    d = 4
    deff = 3.6  # c = 0.4
    s = 200_000
    idx, w = oracle.sample_augmented(tabs, ranks, s, seed=11, counter=2, d_eff_lower=deff)
    D, C = oracle.coin_weights(d, deff)
    ridge = idx[0] >= dims[0]
    p = C / (D + C)
    z = (ridge.sum() - s * p) / math.sqrt(s * p * (1 - p))
    assert abs(z) < 5, z
    # ridge rows: digits in range, uniform over the d rows
    for n in range(3):
        assert np.all((idx[n][ridge] >= dims[n]) & (idx[n][ridge] < dims[n] + ranks[n]))
    k = np.zeros(int(ridge.sum()), dtype=np.int64)
    for n in range(3):
        k = k * ranks[n] + (idx[n][ridge] - dims[n])
    counts = np.bincount(k, minlength=d)
    assert stats.chisquare(counts).pvalue > 1e-4
    # data rows: joint cells against the product law q = prod w / W
    data = ~ridge
    assert np.all(idx[:, data] < np.array(dims)[:, None])
    flat = np.ravel_multi_index(tuple(idx[:, data]), dims)
    obs = np.bincount(flat, minlength=int(np.prod(dims)))
    q = np.ones(1)
    for w_n, C_n in tabs:
        q = np.kron(q, w_n.astype(np.float64) / float(C_n[-1]))
    exp = q * data.sum()
    keep = exp > 5
    assert stats.chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum()).pvalue > 1e-4


@pytest.mark.parametrize("deff", [0.0, 7.3])
def test_augmented_weights_are_inverse_probabilities(deff):
    dims, ranks = (9, 7, 6), (2, 2, 2)
    F, tabs = _tables(dims, ranks, 5)
    d, s = 8, 3000
    idx, w = oracle.sample_augmented(tabs, ranks, s, seed=4, counter=9, d_eff_lower=deff)
    D, C = oracle.coin_weights(d, deff)
    ridge = idx[0] >= dims[0]
    P = np.empty(s)
    P[ridge] = (C / (D + C)) / d
    q = np.ones(int((~ridge).sum()))
    for n, (w_n, C_n) in enumerate(tabs):
        q *= w_n[idx[n][~ridge]].astype(np.float64) / float(C_n[-1])
    P[~ridge] = (D / (D + C)) * q
    np.testing.assert_allclose(w * s * P, 1.0, rtol=1e-14)


def test_augmented_sketch_unbiased():
    dims, ranks = (6, 5, 4), (2, 2, 2)
    p = workloads.tucker_tensor(dims, ranks, 7, "f64", factor="gaussian", noise=("sigma", 0.2))
    X, F, lam = p["X"], p["factors_true"], 0.3
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    K = oracle.kron_matrix(F)
    target = K.T @ K + lam * np.eye(8)
    acc = np.zeros((8, 8))
    trials, s = 400, 200
    for seed in range(trials):
        idx, w = oracle.sample_augmented(tabs, ranks, s, seed=seed, counter=0, d_eff_lower=0.0)
        rows, _ = oracle.augmented_rows(X, F, lam, idx)
        acc += (rows * w[:, None]).T @ rows
    acc /= trials
    assert np.abs(acc - target).max() <= 0.05 * np.abs(target).max()


def test_augmented_solve_equals_explicit_sketch_lstsq():
    dims, ranks = (6, 5, 4), (2, 3, 2)
    p = workloads.tucker_tensor(dims, ranks, 21, "f64", factor="gaussian", noise=("sigma", 0.3),
                                missing=0.2)
    X, F, lam, mask = p["X"], p["factors_true"], 0.05, p["mask"]
    d = 12
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample_augmented(tabs, ranks, 700, seed=8, counter=1, d_eff_lower=11.5)
    got = oracle.core_update_sketched_augmented(X, F, lam, idx, w, mask)
    # explicit Abar = [K; sqrt(lam) I] with unobserved rows of K zeroed, bbar = [x; 0]
    K = oracle.kron_matrix(F) * oracle.unpack_mask(mask, dims).reshape(-1)[:, None]
    Abar = np.vstack([K, math.sqrt(lam) * np.eye(d)])
    bbar = np.concatenate([X.reshape(-1) * oracle.unpack_mask(mask, dims).reshape(-1),
                           np.zeros(d)])
    n = K.shape[0]
    ridge = idx[0] >= dims[0]
    rowid = np.empty(idx.shape[1], dtype=np.int64)
    rowid[~ridge] = np.ravel_multi_index(tuple(idx[:, ~ridge]), dims)
    kk = np.zeros(int(ridge.sum()), dtype=np.int64)
    for m in range(3):
        kk = kk * ranks[m] + (idx[m][ridge] - dims[m])
    rowid[ridge] = n + kk
    SA = np.sqrt(w)[:, None] * Abar[rowid]
    Sb = np.sqrt(w) * bbar[rowid]
    ref = np.linalg.lstsq(SA, Sb, rcond=None)[0]
    np.testing.assert_allclose(got.reshape(-1), ref, rtol=1e-9, atol=1e-11)


def test_c_zero_is_the_plain_sampler():
    dims, ranks = (9, 7, 6), (2, 2, 2)
    F, tabs = _tables(dims, ranks, 5)
    ia, wa = oracle.sample_augmented(tabs, ranks, 5000, seed=3, counter=4, d_eff_lower=8.0)
    ip, wp = oracle.sample(tabs, 5000, seed=3, counter=4)
    assert np.array_equal(ia, ip)
    assert np.array_equal(wa, wp)


def test_sample_count_augmented():
    for d in (1, 8, 64, 4096):
        assert oracle.s_theory_augmented(d, 0.1, 0.1, 0.0) == oracle.s_theory(d, 0.1, 0.1)
    # c = 1/2: 4 d (1 + 1/2) max{...}
    a = max(420.0 * math.log(4.0 * 8 / 0.1), 1.0 / (0.1 * 0.1))
    assert oracle.s_theory_augmented(8, 0.1, 0.1, 7.5) == math.ceil(4.0 * 8 * 1.5 * a)


def test_one_plus_eps_bound_augmented():
    """At Alg. 1's count for beta' = 1/(1 + c), the literal Alg. 1 solve satisfies
    f(g~) <= (1 + eps) f(g*) for at least 1 - delta of the seeds (Thm 3.4)."""
    eps = delta = 0.1
    p = workloads.tucker_tensor((10, 9, 8), (2, 2, 2), 80, "f64", factor="gaussian",
                                noise=("sigma", 1.0))
    X, F, lam = p["X"], p["factors_true"], 1e-1
    ranks = (2, 2, 2)
    s = oracle.s_theory_augmented(8, eps, delta, 0.0)
    g_star = oracle.core_update_exact(X, F, lam)
    f_star = oracle.ridge_objective(X, g_star, F, lam)
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    trials, ok = 10, 0
    ratios = []
    for seed in range(trials):
        idx, w = oracle.sample_augmented(tabs, ranks, s, seed=seed, counter=0)
        g = oracle.core_update_sketched_augmented(X, F, lam, idx, w)
        excess = oracle.sketched_objective_excess(g, g_star, F, lam)
        ratios.append(excess / f_star)
        ok += excess <= eps * f_star
    assert ok >= (1 - delta) * trials, ratios
    # far fewer samples give a visibly larger excess (a wrong weight would not
    # converge at all)
    idx, w = oracle.sample_augmented(tabs, ranks, 64, seed=0, counter=0)
    g = oracle.core_update_sketched_augmented(X, F, lam, idx, w)
    assert oracle.sketched_objective_excess(g, g_star, F, lam) > 10 * np.median(ratios) * f_star


def test_augmented_normal_equation_residual_pin():
    """Zero at Alg. 1's solve, equal to the explicit ||Gram g - rhs|| / ||rhs||
    of the sampled augmented rows elsewhere (chunking does not matter)."""
    dims, ranks = (6, 5, 4), (2, 3, 2)
    p = workloads.tucker_tensor(dims, ranks, 23, "f64", factor="gaussian", noise=("sigma", 0.3))
    X, F, lam = p["X"], p["factors_true"], 0.05
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample_augmented(tabs, ranks, 500, seed=2, counter=0, d_eff_lower=0.0)
    G = oracle.core_update_sketched_augmented(X, F, lam, idx, w)
    assert oracle.normal_equation_residual_augmented(X, F, lam, idx, w, G, chunk=77) < 1e-12
    Gp = G + 0.01 * np.random.default_rng(1).standard_normal(G.shape)
    rows, x = oracle.augmented_rows(X, F, lam, idx)
    gram = (rows * w[:, None]).T @ rows
    rhs = rows.T @ (w * x)
    ref = np.linalg.norm(gram @ Gp.reshape(-1) - rhs) / np.linalg.norm(rhs)
    got = oracle.normal_equation_residual_augmented(X, F, lam, idx, w, Gp, chunk=77)
    assert abs(got - ref) < 1e-12
