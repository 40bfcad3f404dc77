"""Sampling from the true lambda-ridge leverage scores of K on the GPU
(tucker_ridge_tables, tucker_sample_ridge, sampling = 1 in the sampled update)
against the FP64 oracle, through the C ABI.

The tables hold one choice of singular vectors; degenerate singular values
leave that choice open, so the GPU's Jacobi tables and the oracle's SVD tables
are compared through what is unique:
* the mixture's row probabilities against K's ridge scores from the explicit
  Kronecker matrix: within the integer tables' quantisation (rtol 1e-4,
  atol 1e-8; each factor is off by at most ~2^-24 absolute);
* d_eff within 1e-12 relative.
Given the GPU's tables, the oracle's sampler reproduces the draws: indices
bit-exact; weights within 1e-12 relative (P is a sum over all d tuples taken
in a different order).  The sampled update on these draws matches the oracle's
solve of the same sampled system: 1e-10 (FP64 Gram), 1e-9 (BF16 + refinement).
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_10654_amd as tk_mod
    return tk_mod


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def elem_err(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _factors(dims, ranks, seed, lo=0.3):
    rng = np.random.default_rng(seed)
    F = []
    for I, R in zip(dims, ranks):
        Q, _ = np.linalg.qr(rng.standard_normal((I, R)))
        s = np.geomspace(3.0, lo, R)
        F.append(Q * s[None, :] @ np.linalg.qr(rng.standard_normal((R, R)))[0])
    return F


def _host_tables(tcdf, ccdf, dims, ranks):
    """The GPU's tables in the oracle's (w, C) form."""
    Ct = tcdf.cpu().numpy().view(np.uint64)
    wt = np.diff(np.concatenate([[np.uint64(0)], Ct])).astype(np.uint64)
    cc = ccdf.cpu().numpy().view(np.uint64)
    cols, off = [], 0
    for I, R in zip(dims, ranks):
        colt = []
        for c in range(R):
            C = cc[off + c * I: off + (c + 1) * I]
            colt.append((np.diff(np.concatenate([[np.uint64(0)], C])).astype(np.uint64), C))
        cols.append(colt)
        off += I * R
    return (wt, Ct), cols


@pytest.mark.parametrize("dims,ranks,lam", [
    ((7, 6, 5), (3, 2, 3), 1e-2),
    ((7, 6, 5), (3, 2, 3), 0.5),
    ((9, 8), (4, 5), 0.1),
    ((5, 4, 4, 3), (2, 2, 1, 3), 0.05),
])
def test_ridge_tables_reproduce_ridge_scores_of_K(tk, dims, ranks, lam):
    F = _factors(dims, ranks, 11)
    tcdf, ccdf, deff = tk.ridge_tables([T(A) for A in F], lam)
    K = oracle.kron_matrix(F)
    lK = oracle.ridge_leverage_scores(K, lam)
    assert abs(deff - lK.sum()) <= 1e-12 * lK.sum() + 1e-9  # trace form vs eigenvalues
    tt, cols = _host_tables(tcdf, ccdf, dims, ranks)
    allidx = np.array(np.unravel_index(np.arange(K.shape[0]), dims))
    P = oracle.ridge_mixture_probabilities(tt, cols, list(ranks), allidx)
    np.testing.assert_allclose(P, lK / lK.sum(), rtol=1e-4, atol=1e-8)


@pytest.mark.parametrize("dims,ranks,s,aug", [
    ((30, 25, 20), (3, 4, 5), 20000, None),
    ((30, 25, 20), (3, 4, 5), 20000, 58.4),
    ((13, 11, 9, 7, 5), (2, 3, 2, 3, 2), 5001, None),   # order 5: second Philox block
    ((200, 150, 120), (8, 8, 6), 300000, None),         # d = 384, grid-stride passes
    ((60,), (7,), 4000, None),                          # order 1
])
def test_ridge_draws_bit_exact_given_tables(tk, dims, ranks, s, aug):
    F = _factors(dims, ranks, 12)
    tcdf, ccdf, _ = tk.ridge_tables([T(A) for A in F], 0.05)
    print(f"[ridge draws] dims {dims} ranks {ranks} s {s} aug {aug}", flush=True)
    idx, w = tk.sample_ridge(dims, ranks, tcdf, ccdf, s, seed=5, counter=2, problem=1,
                             augmented=aug is not None, d_eff_lower=aug or 0.0)
    tt, cols = _host_tables(tcdf, ccdf, dims, ranks)
    ridx, rw = oracle.sample_ridge(tt, cols, list(ranks), s, 5, 2, problem=1, d_eff_lower=aug)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-12)


@pytest.mark.parametrize("dims,ranks,s,aug", [
    ((23, 19, 17), (3, 4, 5), 6000, None),
    ((40, 36, 30), (8, 8, 6), 15000, None),
    ((23, 19, 17), (3, 4, 5), 6000, 59.5),
])
@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_update_with_ridge_sampling_matches_oracle(tk, dims, ranks, s, aug, precision):
    p = workloads.tucker_tensor(dims, ranks, 13, "f64", factor="gaussian", noise=("sigma", 0.1))
    rng = np.random.default_rng(14)
    F = [A + 0.1 * rng.standard_normal(A.shape) for A in p["factors_true"]]
    lam = 0.5
    X, FF = T(p["X"]), [T(A) for A in F]
    G, idx, w, info = tk.core_update_sketched(X, FF, lam, s, seed=3, counter=1, precision=precision,
                                              refine_max=30, refine_tol=1e-13, sampling="ridge",
                                              augmented=aug is not None, d_eff_lower=aug or 0.0,
                                              return_samples=True, return_info=True)
    # the update's draws are tucker_sample_ridge's on the update's tables
    tcdf, ccdf, _ = tk.ridge_tables(FF, lam)
    i2, w2 = tk.sample_ridge(dims, ranks, tcdf, ccdf, s, seed=3, counter=1,
                             augmented=aug is not None, d_eff_lower=aug or 0.0)
    assert torch.equal(idx, i2) and torch.equal(w, w2)
    ii, ww = idx.cpu().numpy(), w.cpu().numpy()
    if aug is None:
        Gr = oracle.core_update_sketched(p["X"], F, lam, ii, ww)
    else:
        assert (ii[0] >= dims[0]).any()
        Gr = oracle.core_update_sketched_augmented(p["X"], F, lam, ii, ww)
    if precision != "f64":
        assert info[3].item() <= 1e-13, info
    assert elem_err(G.cpu().numpy(), Gr) <= (1e-10 if precision == "f64" else 1e-9)


def test_ridge_sampling_cdf_bits(tk):
    # tables of the ridge mixture with Q = 20: the update solves its own draws
    # (checked against the oracle's solve) and they differ from the default Q's
    dims, ranks, s = (23, 19, 17), (3, 4, 5), 6000
    p = workloads.tucker_tensor(dims, ranks, 13, "f64", factor="gaussian", noise=("sigma", 0.1))
    rng = np.random.default_rng(14)
    F = [A + 0.1 * rng.standard_normal(A.shape) for A in p["factors_true"]]
    lam = 0.5
    X, FF = T(p["X"]), [T(A) for A in F]
    G, idx, w = tk.core_update_sketched(X, FF, lam, s, seed=3, counter=1, precision="f64",
                                        sampling="ridge", return_samples=True, cdf_bits=20)
    _, idx0, w0 = tk.core_update_sketched(X, FF, lam, s, seed=3, counter=1, precision="f64",
                                          sampling="ridge", return_samples=True)
    assert not torch.equal(w, w0)
    ii, ww = idx.cpu().numpy(), w.cpu().numpy()
    assert all((ii[n] >= 0).all() and (ii[n] < dims[n]).all() for n in range(3))
    Gr = oracle.core_update_sketched(p["X"], F, lam, ii, ww)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10
