"""Pins for the oracle's adjoints (differentiation form; not in the paper).

* The sketched-solve adjoint (sample set frozen) equals central finite
  differences of the oracle's own forward solve in float64 (h = 1e-4).
* The exact-solve adjoint equals central finite differences of the exact solve.
* With many samples the sketched gradient approaches the exact-solve gradient
  along smooth (low-rank) directions.
"""
import numpy as np

import oracle
import workloads


def _setup(seed=3, missing=None):
    p = workloads.tucker_tensor((7, 6, 5), (2, 3, 2), seed, "f64", factor="gaussian",
                                noise=("sigma", 0.3), missing=missing)
    F = p["factors_true"]
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tables, 500, seed=8, counter=1)
    gbar = np.random.default_rng(seed + 100).standard_normal((2, 3, 2))
    return p, F, idx, w, gbar


def _fd_sketched(p, F, idx, w, gbar, lam, which, direction, h=1e-4):
    def f(eps):
        Fs = [A.copy() for A in F]
        X = p["X"].copy()
        if which == "X":
            X = X + eps * direction
        else:
            Fs[which] = Fs[which] + eps * direction
        return np.sum(gbar * oracle.core_update_sketched(X, Fs, lam, idx, w, p["mask"]))
    return (f(h) - f(-h)) / (2 * h)


def test_sketched_adjoint_matches_finite_differences():
    for missing in (None, 0.3):
        p, F, idx, w, gbar = _setup(missing=missing)
        lam = 0.05
        bars, Xbar, g = oracle.sketched_adjoint(p["X"], F, lam, idx, w, gbar, p["mask"])
        np.testing.assert_allclose(g, oracle.core_update_sketched(p["X"], F, lam, idx, w,
                                                                  p["mask"]), rtol=1e-10, atol=1e-13)
        rng = np.random.default_rng(0)
        for which in [0, 1, 2, "X"]:
            for _ in range(4):
                shape = p["X"].shape if which == "X" else F[which].shape
                D = rng.standard_normal(shape)
                fd = _fd_sketched(p, F, idx, w, gbar, lam, which, D)
                an = np.sum((Xbar if which == "X" else bars[which]) * D)
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)
        if missing:
            # gradient is zero at unobserved entries
            obs = oracle.unpack_mask(p["mask"], p["X"].shape)
            assert np.all(Xbar[~obs] == 0)


def test_exact_adjoint_matches_finite_differences():
    p, F, _, _, gbar = _setup(seed=5)
    lam = 0.05
    bars, Xbar, _ = oracle.exact_adjoint(p["X"], F, lam, gbar)
    rng = np.random.default_rng(1)
    h = 1e-4
    for which in [0, 1, 2, "X"]:
        shape = p["X"].shape if which == "X" else F[which].shape
        D = rng.standard_normal(shape)

        def f(eps):
            Fs = [A.copy() for A in F]
            X = p["X"]
            if which == "X":
                X = X + eps * D
            else:
                Fs[which] = Fs[which] + eps * D
            return np.sum(gbar * oracle.core_update_exact(X, Fs, lam))
        fd = (f(h) - f(-h)) / (2 * h)
        an = np.sum((Xbar if which == "X" else bars[which]) * D)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)


def test_sketched_gradient_approaches_exact_gradient():
    p = workloads.tucker_tensor((9, 8, 7), (2, 2, 2), 9, "f64", factor="qr",
                                noise=("sigma", 0.05))
    F, lam = p["factors_true"], 1e-2
    gbar = np.random.default_rng(2).standard_normal((2, 2, 2))
    ebars, eXbar, gstar = oracle.exact_adjoint(p["X"], F, lam, gbar)
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tables, 200_000, seed=1, counter=0)
    sbars, sXbar, g = oracle.sketched_adjoint(p["X"], F, lam, idx, w, gbar)
    gap = np.linalg.norm(g - gstar) / np.linalg.norm(gstar)
    rng = np.random.default_rng(4)
    for n in range(3):
        D = rng.standard_normal(F[n].shape)
        a, b = np.sum(sbars[n] * D), np.sum(ebars[n] * D)
        assert abs(a - b) <= max(50 * gap, 0.05) * max(1.0, abs(b)), (n, a, b, gap)
    # tensor direction: smooth low-rank direction
    Dt = oracle.reconstruct(rng.standard_normal((2, 2, 2)), F)
    a, b = np.sum(sXbar * Dt), np.sum(eXbar * Dt)
    assert abs(a - b) <= max(50 * gap, 0.05) * max(1.0, abs(b)), (a, b, gap)
