"""Pins for the oracle's sampler of the true lambda-ridge leverage scores of K
(the non-product mixture over singular-value tuples).

Pins (each would catch a plausible mistake in the oracle):
* the tables reproduce K's ridge scores: the quantised mixture probability of
  every row equals l^lam(K)_i / d_eff(K), computed from the explicit Kronecker
  matrix by the definition a_i (K^T K + lam I)^+ a_i^T, to the quantisation
  of the integer tables; d_eff equals the definition's trace;
* lam = 0 gives the statistical leverage distribution, the product of the
  factor score distributions (Lemma 4.1);
* draw frequencies match the mixture (chi-square), weights are 1 / (s P),
  and the rescaled sketch is unbiased for K^T K (Monte Carlo);
* a larger lam concentrates the draws on the tuples with large singular
  values (d_eff < d) -- the reason to sample from these scores.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def _factors(dims, ranks, seed, spread=True):
    rng = np.random.default_rng(seed)
    F = []
    for I, R in zip(dims, ranks):
        Q, _ = np.linalg.qr(rng.standard_normal((I, R)))
        s = np.geomspace(3.0, 0.3, R) if spread else np.ones(R)
        F.append(Q * s[None, :] @ np.linalg.qr(rng.standard_normal((R, R)))[0])
    return F


@pytest.mark.parametrize("lam", [0.0, 1e-2, 0.5])
def test_mixture_reproduces_ridge_scores_of_K(lam):
    dims, ranks = (7, 6, 5), (3, 2, 3)
    F = _factors(dims, ranks, 1)
    K = oracle.kron_matrix(F)
    lK = oracle.ridge_leverage_scores(K, lam)
    deff = float(lK.sum())
    tt, cols, deff_t = oracle.ridge_tables(F, lam)
    assert abs(deff_t - deff) <= 1e-10 * deff
    allidx = np.array(np.unravel_index(np.arange(K.shape[0]), dims))
    P = oracle.ridge_mixture_probabilities(tt, cols, ranks, allidx)
    # each of the N + 1 quantised factors is off by at most ~2^-24 in absolute
    # terms: ~1e-7 relative on the large entries, up to ~1e-5 on entries whose
    # factors are ~1e-3 -- far below the error of a wrong column or tuple
    np.testing.assert_allclose(P, lK / deff, rtol=1e-4, atol=1e-8)
    assert abs(P.sum() - 1.0) <= 1e-5


def test_lambda_zero_is_the_product_law():
    dims, ranks = (8, 6, 5), (2, 3, 2)
    F = _factors(dims, ranks, 2)
    tt, cols, _ = oracle.ridge_tables(F, 0.0)
    allidx = np.array(np.unravel_index(np.arange(int(np.prod(dims))), dims))
    P = oracle.ridge_mixture_probabilities(tt, cols, ranks, allidx)
    q = np.ones(1)
    for A in F:
        q = np.kron(q, oracle.leverage_scores(A) / A.shape[1])
    np.testing.assert_allclose(P, q, rtol=1e-4, atol=1e-8)


def test_ridge_draws_frequencies_weights_and_unbiasedness():
    dims, ranks = (6, 5, 4), (2, 2, 2)
    F = _factors(dims, ranks, 3)
    lam = 0.3
    tt, cols, _ = oracle.ridge_tables(F, lam)
    s = 120_000
    idx, w = oracle.sample_ridge(tt, cols, ranks, s, seed=5, counter=1)
    assert np.all(idx < np.array(dims)[:, None])
    allidx = np.array(np.unravel_index(np.arange(int(np.prod(dims))), dims))
    P = oracle.ridge_mixture_probabilities(tt, cols, ranks, allidx)
    flat = np.ravel_multi_index(tuple(idx), dims)
    obs = np.bincount(flat, minlength=P.size)
    keep = P * s > 5
    assert stats.chisquare(obs[keep], P[keep] * obs[keep].sum() / P[keep].sum()).pvalue > 1e-4
    np.testing.assert_allclose(w * s * P[flat], 1.0, rtol=1e-13)
    K = oracle.kron_matrix(F)
    acc = np.zeros((8, 8))
    trials = 300
    for seed in range(trials):
        i2, w2 = oracle.sample_ridge(tt, cols, ranks, 100, seed=seed, counter=0)
        rows = oracle.kron_rows(F, i2)
        acc += (rows * w2[:, None]).T @ rows
    acc /= trials
    target = K.T @ K
    assert np.abs(acc - target).max() <= 0.06 * np.abs(target).max()


def test_large_lambda_concentrates_on_large_singular_values():
    dims, ranks = (9, 8, 7), (3, 3, 3)
    F = _factors(dims, ranks, 4)
    tt_small, _, deff_small = oracle.ridge_tables(F, 1e-6)
    tt_big, _, deff_big = oracle.ridge_tables(F, 1.0)
    assert deff_small > 26.9 and deff_big < 0.5 * 27
    wt_b = tt_big[0].astype(float) / float(tt_big[1][-1])
    # the tuple with the largest singular values carries the most mass
    assert np.argmax(wt_b) == 0


def test_ridge_draws_with_the_branch_coin():
    """The augmented coin over ridge-score draws: ridge rows exactly where
    sample_augmented puts them (same words), data rows those of the plain
    ridge draws with weights times (D + C) / D; c = 0 changes nothing."""
    dims, ranks = (6, 5, 4), (2, 2, 2)
    F = _factors(dims, ranks, 6)
    tt, cols, _ = oracle.ridge_tables(F, 0.2)
    lev = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    ip, wp = oracle.sample_ridge(tt, cols, ranks, 4000, seed=2, counter=7)
    ia, wa = oracle.sample_ridge(tt, cols, ranks, 4000, seed=2, counter=7, d_eff_lower=7.6)
    il, wl = oracle.sample_augmented(lev, ranks, 4000, 2, 7, 7.6)
    ridge = ia[0] >= dims[0]
    assert np.array_equal(ridge, il[0] >= dims[0])
    assert np.array_equal(ia[:, ridge], il[:, ridge]) and np.array_equal(wa[ridge], wl[ridge])
    D, C = oracle.coin_weights(8, 7.6)
    assert np.array_equal(ia[:, ~ridge], ip[:, ~ridge])
    np.testing.assert_allclose(wa[~ridge], wp[~ridge] * (D + C) / D, rtol=1e-15)
    i0, w0 = oracle.sample_ridge(tt, cols, ranks, 4000, seed=2, counter=7, d_eff_lower=8.0)
    assert np.array_equal(i0, ip) and np.array_equal(w0, wp)
