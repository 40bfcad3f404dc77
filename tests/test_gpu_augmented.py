"""Alg. 1 taken literally on the GPU (augmented draws over [K; sqrt(lam) I])
against the FP64 oracle, through the C ABI.

Bars (written per test):
* draws (indices with the ridge encoding, weights): bit-exact against the
  oracle's augmented sampler given equal tables -- integer work and weights
  formed with the same IEEE operations in the same order;
* FP64 Gram: core element-wise within 1e-10 of the oracle's solve of the same
  sampled system (max |G - G_ref| / max |G_ref|);
* BF16 / FP32 Gram with FP64 refinement: 1e-9 after the refinement reports
  convergence to 1e-13;
* C2 size (512^3 f32, d = 4096, BF16): draws bit-exact and the f32 core solves
  the sampled augmented normal equations to 1e-6 (oracle FP64 residual).
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


def _case(dims, ranks, seed, missing=None):
    p = workloads.tucker_tensor(dims, ranks, seed, "f64", factor="gaussian", noise=("sigma", 0.1),
                                missing=missing)
    rng = np.random.default_rng(seed + 7)
    F = [A + 0.1 * rng.standard_normal(A.shape) for A in p["factors_true"]]
    return p, F


@pytest.mark.parametrize("dims,ranks,s,deff", [
    ((23, 19, 17), (3, 4, 5), 5000, 0.0),            # c = 1
    ((23, 19, 17), (3, 4, 5), 5000, 59.3),           # c = 0.7
    ((13, 11, 9, 7, 5), (2, 3, 2, 3, 2), 3001, 0.0), # order 5: second Philox block
    ((9, 8, 7, 6, 5, 4, 3, 3), (2, 2, 2, 2, 1, 2, 2, 1), 2000, 10.0),  # order 8
    ((50,), (7,), 4099, 6.5),                        # order 1
    ((3000, 2500, 1200), (2, 2, 2), 4000, 0.0),      # tables past the LDS-staged size
    ((23, 19, 17), (3, 4, 5), 1_000_000, 0.0),       # many grid-stride passes
    ((23, 19, 17), (3, 4, 5), 4000, 60.0),           # c = 0: the plain draws
])
def test_augmented_draws_bit_exact(tk, dims, ranks, s, deff):
    F = workloads.random_factors(dims, ranks, 5, kind="gaussian")
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    cdf = T(np.concatenate([C for _, C in tabs]).view(np.int64))
    print(f"[aug draws] dims {dims} ranks {ranks} s {s} d'_eff {deff}", flush=True)
    idx, w = tk.sample_augmented(dims, ranks, cdf, s, seed=17, counter=3, problem=2,
                                 d_eff_lower=deff)
    ridx, rw = oracle.sample_augmented(tabs, ranks, s, 17, 3, deff, problem=2)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)


@pytest.mark.parametrize("dims,ranks,s,missing", [
    ((23, 19, 17), (3, 4, 5), 6000, None),      # d = 60: per-sample residual kernels
    ((41, 37, 29), (5, 6, 7), 9000, None),      # d = 210
    ((40, 36, 30), (8, 8, 6), 15000, 0.2),      # d = 384: fused residual pass, masked
    ((13, 11, 9, 7), (2, 3, 2, 3), 3000, None), # order 4
])
@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_augmented_update_matches_oracle(tk, dims, ranks, s, missing, precision):
    p, F = _case(dims, ranks, 31, missing)
    lam, deff = 2e-2, float(np.prod(ranks)) - 0.6
    mask = T(p["mask"].view(np.int32)) if missing else None
    print(f"[aug update] dims {dims} ranks {ranks} s {s} {precision}", flush=True)
    G, idx, w, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=7,
                                              counter=5, precision=precision, mask=mask,
                                              refine_max=30, refine_tol=1e-13, augmented=True,
                                              d_eff_lower=deff, return_samples=True,
                                              return_info=True)
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    ridx, rw = oracle.sample_augmented(tabs, ranks, s, 7, 5, deff)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    assert (ridx[0] >= dims[0]).sum() > 0  # ridge rows were drawn
    Gr = oracle.core_update_sketched_augmented(p["X"], F, lam, ridx, rw, p.get("mask"))
    if precision != "f64":
        assert info[3].item() <= 1e-13, info
    assert elem_err(G.cpu().numpy(), Gr) <= (1e-10 if precision == "f64" else 1e-9)


def test_augmented_cdf_bits_matches_oracle(tk):
    # the factor tables and the branch coin with Q = 20 fixed-point bits
    dims, ranks, s, q = (41, 37, 29), (5, 6, 7), 9000, 20
    p, F = _case(dims, ranks, 31)
    lam, deff = 2e-2, float(np.prod(ranks)) - 0.6
    G, idx, w = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=7, counter=5,
                                        precision="f64", augmented=True, d_eff_lower=deff,
                                        return_samples=True, cdf_bits=q)
    tabs = [oracle.cdf_table(oracle.leverage_scores(A), q) for A in F]
    ridx, rw = oracle.sample_augmented(tabs, ranks, s, 7, 5, deff, q_bits=q)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    Gr = oracle.core_update_sketched_augmented(p["X"], F, lam, ridx, rw)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10


def test_augmented_frozen_set_and_adjoint_refusal(tk):
    p, F = _case((20, 18, 16), (3, 4, 2), 32)
    lam, s = 5e-2, 2500
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    ridx, rw = oracle.sample_augmented(tabs, (3, 4, 2), s, 9, 0, 0.0)
    X, FF = T(p["X"]), [T(A) for A in F]
    G = tk.core_update_sketched(X, FF, lam, s, idx=T(ridx), weight=T(rw), augmented=True)
    Gr = oracle.core_update_sketched_augmented(p["X"], F, lam, ridx, rw)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10
    # the adjoint is of the Gram + lambda I form: augmented options are refused on
    # the host before anything is enqueued
    import ctypes
    from paper_2107_10654_amd import _lib as L
    pr = tk.make_problem(X, FF, lam)
    o = L.TkSketchOpts()
    o.num_samples = s
    o.augmented = 1
    o.gram_precision = L.TK_F64
    fb = (ctypes.c_void_p * 3)(*[A.data_ptr() for A in FF])
    it, wt = T(ridx), T(rw)
    code = L.load().tucker_core_update_sketched_adjoint(
        ctypes.byref(pr), ctypes.byref(o), it.data_ptr(), wt.data_ptr(), G.data_ptr(),
        G.data_ptr(), fb, None, None, None, X.data_ptr(), 1 << 20, None)
    assert code == 1  # TK_E_ARG


def test_augmented_c2_size(tk):
    prob = workloads.config_problem("c2")
    cfg = prob["cfg"]
    Fn = [np.ascontiguousarray(A.astype(np.float32)) for A in prob["factors_true"]]
    X, F = T(prob["X"]), [T(A) for A in Fn]
    s = cfg["samples"]
    G, idx, w, info = tk.core_update_sketched(X, F, cfg["lam"], s, seed=cfg["seed"], counter=0,
                                              precision="bf16", refine_max=12, refine_tol=1e-13,
                                              augmented=True, return_samples=True,
                                              return_info=True)
    F64 = [A.astype(np.float64) for A in Fn]
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F64]
    ridx, rw = oracle.sample_augmented(tabs, cfg["ranks"], s, cfg["seed"], 0, 0.0)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    assert info[3].item() <= 1e-13
    res = oracle.normal_equation_residual_augmented(prob["X"], F64, cfg["lam"], ridx, rw,
                                                    G.cpu().numpy())
    assert res <= 1e-6, res
