"""Pins for the oracle's counter-based generator, CDF tables and product sampler.

Pins (each would catch a plausible mistake in the oracle):
* Philox4x64-10 equals numpy's independent ``Philox`` bit generator and the
  published known-answer vectors (tests/golden/philox4x64_10_kat.txt).
* The vectorised 128-bit product equals Python's exact integer product.
* Inverse-CDF search equals a brute-force scan of the definition min{j : C_j > u}.
* Draw frequencies match q = w / W per mode (chi-square), modes are independent
  (contingency chi-square), and rows with zero weight are never drawn
  (Lemma 4.1 product law and the factored sampler of Alg. 3).
* The rescaled sketch is unbiased: E[(SK)^T SK] = K^T K (Thm A.3, unbiasedness).
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import philox as ph
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    assert len(rows) == 3
    for r in rows:
        ctr, key, out = r[:4], r[4:6], r[6:]
        assert ph.philox4x64_scalar(ctr, key) == out
        vec = ph.philox4x64(*[np.uint64(c) for c in ctr], key[0], key[1])
        assert [int(v) for v in vec] == out


def test_philox_matches_numpy_bitgenerator():
    rng = np.random.default_rng(123)
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(1, 2 ** 63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
        # numpy's Philox increments word 0 of the counter before each block
        bg = np.random.Philox(counter=np.array([ctr[0] - 1] + ctr[1:], dtype=np.uint64),
                              key=np.array(key, dtype=np.uint64))
        ref = [int(v) for v in bg.random_raw(4)]
        assert ph.philox4x64_scalar(ctr, key) == ref
        vec = ph.philox4x64(np.uint64(ctr[0]), np.uint64(ctr[1]), np.uint64(ctr[2]),
                            np.uint64(ctr[3]), key[0], key[1])
        assert [int(v) for v in vec] == ref


def test_mulhilo64_exact():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2 ** 64, size=1000, dtype=np.uint64)
    b = rng.integers(0, 2 ** 64, size=1000, dtype=np.uint64)
    a[:3] = [0, 2 ** 64 - 1, 2 ** 63]
    b[:3] = [2 ** 64 - 1, 2 ** 64 - 1, 3]
    hi, lo = ph.mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & ph.MASK64


def test_cdf_table_and_search_bruteforce():
    scores = np.array([0.25, 0.0, 1e-9, 0.5, 0.999, 0.0, 0.3])
    w, C = oracle.cdf_table(scores)
    assert w.dtype == np.uint64 and C.dtype == np.uint64
    for sc, wi in zip(scores, w):
        assert int(wi) == int(np.ceil(sc * 2 ** 24))
        assert (sc > 0) == (wi > 0)
    W = int(C[-1])
    assert W == sum(int(v) for v in w)
    rng = np.random.default_rng(1)
    us = list(rng.integers(0, W, size=200)) + [0, W - 1] + [int(c) for c in C[:-1]]
    for u in us:
        brute = next(j for j in range(len(C)) if int(C[j]) > u)
        assert int(np.searchsorted(C, np.uint64(u), side="right")) == brute


def _tables(factors):
    return [oracle.cdf_table(oracle.leverage_scores(A)) for A in factors]


def test_sampler_frequencies_and_independence():
    factors = workloads.random_factors((23, 17, 11), (3, 4, 2), seed=11, kind="gaussian")
    tables = _tables(factors)
    s = 200_000
    idx, weight = oracle.sample(tables, s, seed=99, counter=3)
    assert idx.dtype == np.int32 and idx.shape == (3, s)
    for n, (w, C) in enumerate(tables):
        q = w.astype(np.float64) / float(C[-1])
        counts = np.bincount(idx[n], minlength=len(w))
        res = stats.chisquare(counts, q * s)
        assert res.pvalue > 1e-4, (n, res)
    # independence of modes 0 and 1
    ct = np.zeros((len(tables[0][0]), len(tables[1][0])))
    np.add.at(ct, (idx[0], idx[1]), 1)
    res = stats.chi2_contingency(ct[ct.sum(1) > 0][:, ct.sum(0) > 0])
    assert res.pvalue > 1e-4
    # weights are 1 / (s P(row))
    p = oracle.sampling_probabilities(tables, idx)
    np.testing.assert_allclose(weight, 1.0 / (s * p), rtol=1e-14)


def test_zero_weight_rows_never_drawn():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 3))
    A[[0, 7, 39]] = 0.0  # rows with zero leverage
    B = rng.standard_normal((9, 2))
    tables = _tables([A, B])
    idx, _ = oracle.sample(tables, 50_000, seed=1, counter=0)
    assert not np.isin(idx[0], [0, 7, 39]).any()
    assert idx[0].max() < 40 and idx[1].max() < 9


def test_more_than_four_modes_use_second_block():
    factors = workloads.random_factors((5, 6, 4, 7, 5, 3), (2, 2, 2, 2, 2, 2), seed=3)
    tables = _tables(factors)
    idx, _ = oracle.sample(tables, 4096, seed=5, counter=1)
    # mode 4 is driven by word 0 of block 1, mode 0 by word 0 of block 0
    t = np.arange(4096, dtype=np.uint64)
    w1 = ph.philox4x64(t, np.uint64(1), np.uint64(0), np.uint64(1), 5, 0)
    u = ph.mulhi64(w1[0], np.uint64(tables[4][1][-1]))
    np.testing.assert_array_equal(idx[4], np.searchsorted(tables[4][1], u, side="right"))
    for n in range(6):
        counts = np.bincount(idx[n], minlength=len(tables[n][0]))
        q = tables[n][0].astype(float) / float(tables[n][1][-1])
        assert stats.chisquare(counts, q * 4096).pvalue > 1e-4


def test_sketched_gram_unbiased():
    """E[sum_t w_t k_t k_t^T] = K^T K (Thm A.3); checked by many independent draws."""
    factors = workloads.random_factors((9, 7, 5), (2, 3, 2), seed=21, kind="gaussian")
    tables = _tables(factors)
    K = oracle.kron_matrix(factors)
    KtK = K.T @ K
    reps, s = 400, 256
    acc = np.zeros_like(KtK)
    acc2 = np.zeros_like(KtK)
    for r in range(reps):
        idx, w = oracle.sample(tables, s, seed=1234, counter=r)
        rows = oracle.kron_rows(factors, idx)
        Gs = (rows * w[:, None]).T @ rows
        acc += Gs
        acc2 += Gs * Gs
    mean = acc / reps
    var = acc2 / reps - mean ** 2
    se = np.sqrt(np.maximum(var, 0) / reps) + 1e-12
    z = np.abs(mean - KtK) / se
    assert z.max() < 5.5, z.max()
    # a dropped weight (e.g. forgetting the 1/s) would be off by orders of magnitude
    assert np.abs(mean - KtK).max() < 0.2 * np.abs(KtK).max()


@pytest.mark.parametrize("d,expected", [(8, 155053), (16, 347369), (32, 769265), (64, 1687583)])
def test_s_theory(d, expected):
    # Alg. 1 sample count with beta' = 1/2 (Cor. 3.3), eps = delta = 0.1 (Sec. 5 settings)
    assert oracle.s_theory(d, 0.1, 0.1) == expected
