"""GPU adjoint of the sampled core update (C ABI tucker_core_update_sketched_adjoint
and the torch.autograd wrapper), with the sample set held fixed.

Bars (written per test):
* against the FP64 oracle's adjoint on the same frozen samples: relative error
  of every factor gradient and of the tensor gradient <= 1e-9 with the FP64
  Gram, <= 1e-8 with the BF16 Gram + FP64 refinement (the v solve is refined
  to 1e-13 of its right side);
* against central finite differences of the FP64 forward on the same samples
  (h = 1e-4 along unit-norm directions): relative difference <= 1e-6;
* against the exact-solve gradient (oracle, FP64), along directions in the
  factors' column spaces and in range(K), where the sampled residual term
  cancels: the bar is 4x the measured forward gap ||g_sketch - g_exact|| /
  ||g_exact|| (the oracle shows at most 1.4x at a smaller size).
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
    """Element-wise error bound: max_i |a_i - b_i| / max_i |b_i| (every entry of a
    lies within this fraction of the reference's largest entry)."""
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


@pytest.mark.parametrize("dims,ranks,missing", [
    ((20, 18, 16), (3, 4, 2), None),
    ((11, 9, 8, 7), (2, 3, 2, 2), None),
    ((25, 21, 17), (4, 3, 5), 0.2),
    ((40, 30), (5, 6), None),
    ((60,), (6,), None),
])
@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_adjoint_matches_oracle(tk, dims, ranks, missing, precision):
    p, F = _case(dims, ranks, 21, missing)
    lam, s = 1e-3, 3000
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tabs, s, seed=4, counter=3)
    mask = p.get("mask")
    gbar = np.random.default_rng(5).standard_normal(ranks)
    bars_r, xbar_r, g_r = oracle.sketched_adjoint(p["X"], F, lam, idx, w, gbar, mask=mask)
    X, FF = T(p["X"]), [T(A) for A in F]
    mk = T(mask.view(np.int32)) if mask is not None else None
    G = tk.core_update_sketched(X, FF, lam, s, idx=T(idx), weight=T(w), precision=precision,
                                mask=mk, refine_max=30)
    assert elem_err(G.cpu().numpy(), g_r) <= (1e-10 if precision == "f64" else 1e-9)
    fbar, xbar, info = tk.core_update_sketched_adjoint(X, FF, lam, T(idx), T(w), G, T(gbar),
                                                       precision=precision, mask=mk,
                                                       refine_max=30, return_info=True)
    bar = 1e-9 if precision == "f64" else 1e-8
    for n in range(len(F)):
        assert elem_err(fbar[n].cpu().numpy(), bars_r[n]) <= bar, n
    assert elem_err(xbar.cpu().numpy(), xbar_r) <= bar
    if precision != "f64":
        assert info[3].item() <= 1e-13


def test_adjoint_without_tensor_gradient(tk):
    p, F = _case((16, 15, 14), (2, 3, 4), 22)
    lam, s = 1e-2, 900
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tabs, s, seed=1, counter=0)
    gbar = np.random.default_rng(2).standard_normal((2, 3, 4))
    bars_r, _, g_r = oracle.sketched_adjoint(p["X"], F, lam, idx, w, gbar)
    fbar, xbar = tk.core_update_sketched_adjoint(T(p["X"]), [T(A) for A in F], lam, T(idx), T(w),
                                                 T(g_r), T(gbar), want_x=False)
    assert xbar is None
    for n in range(3):
        assert elem_err(fbar[n].cpu().numpy(), bars_r[n]) <= 1e-9


def test_adjoint_f32_problem(tk):
    # f32 storage: the adjoint is computed in FP64 and returned in f32
    p, F = _case((24, 20, 18), (4, 3, 3), 23)
    X32 = p["X"].astype(np.float32)
    F32 = [A.astype(np.float32) for A in F]
    lam, s = 1e-2, 4000
    tabs = [oracle.cdf_table(oracle.leverage_scores(A.astype(np.float64))) for A in F32]
    idx, w = oracle.sample(tabs, s, seed=8, counter=0)
    gbar = np.random.default_rng(3).standard_normal((4, 3, 3))
    bars_r, xbar_r, g_r = oracle.sketched_adjoint(X32.astype(np.float64),
                                                  [A.astype(np.float64) for A in F32], lam, idx, w,
                                                  gbar)
    X, FF = T(X32), [T(A) for A in F32]
    G = tk.core_update_sketched(X, FF, lam, s, idx=T(idx), weight=T(w), precision="bf16")
    fbar, xbar = tk.core_update_sketched_adjoint(X, FF, lam, T(idx), T(w), G,
                                                 T(gbar.astype(np.float32)), precision="bf16")
    # inputs g and gbar are f32-rounded, outputs f32
    for n in range(3):
        assert elem_err(fbar[n].cpu().numpy(), bars_r[n]) <= 1e-5
    assert elem_err(xbar.cpu().numpy(), xbar_r) <= 1e-5


def test_autograd_function(tk):
    p, F = _case((18, 16, 14), (3, 2, 4), 24)
    lam, s = 1e-3, 2500
    X = T(p["X"]).requires_grad_(True)
    FF = [T(A).requires_grad_(True) for A in F]
    gbar = np.random.default_rng(6).standard_normal((3, 2, 4))
    G, idx, w = tk.sketched_core_update(X, FF, lam, s, seed=3, counter=1, return_samples=True)
    (G * T(gbar)).sum().backward()
    bars_r, xbar_r, g_r = oracle.sketched_adjoint(p["X"], F, lam, idx.cpu().numpy(),
                                                  w.cpu().numpy(), gbar)
    assert elem_err(G.detach().cpu().numpy(), g_r) <= 1e-10
    for n in range(3):
        assert elem_err(FF[n].grad.cpu().numpy(), bars_r[n]) <= 1e-9
    assert elem_err(X.grad.cpu().numpy(), xbar_r) <= 1e-9


# ---------------------------------------------------------------- C5-size checks
@pytest.fixture(scope="module")
def c5(tk):
    prob = workloads.config_problem("c5")
    cfg = prob["cfg"]
    X = T(prob["X"].astype(np.float64))
    F = [T(np.ascontiguousarray(A, dtype=np.float64)) for A in prob["factors_true"]]
    rng = np.random.default_rng(6)
    gbar = T(rng.standard_normal(cfg["ranks"]))
    G, idx, w = tk.core_update_sketched(X, F, cfg["lam"], cfg["samples"], seed=cfg["seed"],
                                        precision="f64", return_samples=True)
    fbar, xbar = tk.core_update_sketched_adjoint(X, F, cfg["lam"], idx, w, G, gbar)
    return dict(prob=prob, cfg=cfg, X=X, F=F, gbar=gbar, G=G, idx=idx, w=w, fbar=fbar, xbar=xbar)


def _f(tk, c, X, F):
    """<gbar, g> of the FP64 forward on the frozen samples."""
    G = tk.core_update_sketched(X, F, c["cfg"]["lam"], c["cfg"]["samples"], idx=c["idx"],
                                weight=c["w"], precision="f64")
    return float((G * c["gbar"]).sum().item())


def test_c5_forward_matches_oracle(tk, c5):
    """The full-size C5 forward (FP64 mode) against the oracle: samples bit-exact
    with the oracle's sampler, core within 1e-10 element-wise of the oracle's
    Cholesky solve of the same sketched system."""
    cfg = c5["cfg"]
    Fn = [np.asarray(A, dtype=np.float64) for A in c5["prob"]["factors_true"]]
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in Fn]
    ridx, rw = oracle.sample(tables, cfg["samples"], cfg["seed"], 0)
    assert np.array_equal(c5["idx"].cpu().numpy(), ridx)
    assert np.array_equal(c5["w"].cpu().numpy(), rw)
    Gr = oracle.core_update_sketched(c5["prob"]["X"].astype(np.float64), Fn, cfg["lam"], ridx, rw)
    assert elem_err(c5["G"].cpu().numpy(), Gr) <= 1e-10


def _fd_check(ad, fd, floor):
    # central differences at h = 1e-4 in FP64: truncation ~1e-8 relative, and the
    # forward's rounding noise (~1e-13 of <gbar, g>) divided by 2h gives an
    # absolute floor
    assert abs(ad - fd) <= 1e-6 * abs(fd) + floor, (ad, fd)


def test_c5_adjoint_matches_central_differences(tk, c5):
    """32 random unit directions per factor and for X, and 64 coordinates (16
    per factor: rows that were sampled and rows drawn at random; 16 of X: 8
    sampled entries and 8 random ones, whose gradient is 0 unless sampled)."""
    h = 1e-4
    rng = np.random.default_rng(7)
    F = c5["F"]
    scale = abs(float((c5["G"] * c5["gbar"]).sum().item()))
    floor = 1e-13 * scale / h
    for n in range(3):
        for _ in range(32):
            D = rng.standard_normal(tuple(F[n].shape))
            D /= np.linalg.norm(D)
            Dt = T(D)
            Fp = [A if m != n else A + h * Dt for m, A in enumerate(F)]
            Fm = [A if m != n else A - h * Dt for m, A in enumerate(F)]
            fd = (_f(tk, c5, c5["X"], Fp) - _f(tk, c5, c5["X"], Fm)) / (2 * h)
            ad = float((c5["fbar"][n] * Dt).sum().item())
            _fd_check(ad, fd, floor)
    for _ in range(32):
        D = rng.standard_normal(tuple(c5["X"].shape))
        D /= np.linalg.norm(D)
        Dt = T(D)
        fd = (_f(tk, c5, c5["X"] + h * Dt, F) - _f(tk, c5, c5["X"] - h * Dt, F)) / (2 * h)
        ad = float((c5["xbar"] * Dt).sum().item())
        _fd_check(ad, fd, floor)
    # A single coordinate carries the whole step h (a random unit direction
    # spreads it over thousands of entries), so the O(h^2) truncation of the
    # central difference is larger there: the coordinate checks combine the
    # central differences at h and h/2 (Richardson, error O(h^4)), whose
    # rounding noise is three times that of one difference.
    idx = c5["idx"].cpu().numpy()

    def factor_fd(n, i, r, step):
        Fp = [A.clone() for A in F]
        Fm = [A.clone() for A in F]
        Fp[n][i, r] += step
        Fm[n][i, r] -= step
        return (_f(tk, c5, c5["X"], Fp) - _f(tk, c5, c5["X"], Fm)) / (2 * step)

    def x_fd(c, step):
        Xp, Xm = c5["X"].clone(), c5["X"].clone()
        Xp[c] += step
        Xm[c] -= step
        return (_f(tk, c5, Xp, F) - _f(tk, c5, Xm, F)) / (2 * step)

    for n in range(3):
        I, R = F[n].shape
        rows = list(rng.choice(idx[n], 8)) + list(rng.integers(0, I, 8))
        for i in rows:
            r = int(rng.integers(0, R))
            fd = (4 * factor_fd(n, int(i), r, h / 2) - factor_fd(n, int(i), r, h)) / 3
            _fd_check(float(c5["fbar"][n][int(i), r].item()), fd, 3 * floor)
    cols = rng.choice(idx.shape[1], 8)
    coords = [tuple(int(v) for v in idx[:, t]) for t in cols]
    coords += [tuple(int(rng.integers(0, I)) for I in c5["X"].shape) for _ in range(8)]
    for c in coords:
        fd = (4 * x_fd(c, h / 2) - x_fd(c, h)) / 3
        _fd_check(float(c5["xbar"][c].item()), fd, 3 * floor)


def test_adjoint_repeatable_with_duplicate_samples(tk):
    """Duplicate samples accumulate through atomics in an order that can vary
    from run to run; two runs agree to rounding (1e-13 of the largest entry in
    FP64), and both match the oracle's sequential sums (1e-9)."""
    dims, ranks = (10, 9, 8), (3, 3, 2)
    p, F = _case(dims, ranks, 41)
    lam, s = 1e-3, 20000  # 720 entries, so every entry is drawn many times
    tabs = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    idx, w = oracle.sample(tabs, s, 3, 1)
    assert len(np.unique(oracle.flat_index(idx, dims))) < s // 10
    gbar = np.random.default_rng(42).standard_normal(ranks)
    X, FF = T(p["X"]), [T(A) for A in F]
    G = tk.core_update_sketched(X, FF, lam, s, idx=T(idx), weight=T(w), precision="f64")
    runs = [tk.core_update_sketched_adjoint(X, FF, lam, T(idx), T(w), G, T(gbar))
            for _ in range(2)]
    bars_r, xbar_r, _ = oracle.sketched_adjoint(p["X"], F, lam, idx, w, gbar)
    for n in range(3):
        a, b = runs[0][0][n].cpu().numpy(), runs[1][0][n].cpu().numpy()
        assert elem_err(a, b) <= 1e-13, n
        assert elem_err(a, bars_r[n]) <= 1e-9, n
    assert elem_err(runs[0][1].cpu().numpy(), runs[1][1].cpu().numpy()) <= 1e-13
    assert elem_err(runs[0][1].cpu().numpy(), xbar_r) <= 1e-9


def test_c5_adjoint_against_exact_solve_gradient(tk, c5):
    """Sketched vs exact-solve gradient where the sketch is expected to agree.

    dg = M^{-1} (dK^T r - K^T dK g) with r = x - K g.  Along directions that
    stay in the factors' column spaces (D_n = A_n B for factors, D in range(K)
    for the tensor) the residual term vanishes for both solves up to lambda
    terms (their normal equations make the residual orthogonal to range(K) in
    their own inner products), so the two directional derivatives differ by
    the sketch's error in M: a multiple of the forward gap.  Along generic
    directions the sketched gradient also carries the sampling noise of the
    data residual and no such bar holds.
    """
    cfg = c5["cfg"]
    Xn = c5["prob"]["X"].astype(np.float64)
    Fn = [np.asarray(A, dtype=np.float64) for A in c5["prob"]["factors_true"]]
    gbar = c5["gbar"].cpu().numpy()
    bars_e, xbar_e, g_e = oracle.exact_adjoint(Xn, Fn, cfg["lam"], gbar)
    gap = elem_err(c5["G"].cpu().numpy(), g_e)
    assert 0 < gap < 0.5
    for n in range(3):
        # derivative along every D_n = A_n B at once: <Abar, A_n B> = <A_n^T Abar, B>
        proj_s = Fn[n].T @ c5["fbar"][n].cpu().numpy()
        proj_e = Fn[n].T @ bars_e[n]
        r = elem_err(proj_s, proj_e)
        assert r <= 4 * gap, (n, r, gap)
    rng = np.random.default_rng(8)
    xs = c5["xbar"].cpu().numpy()
    for _ in range(3):
        D = oracle.reconstruct(rng.standard_normal(cfg["ranks"]), Fn)
        a, b = float(np.vdot(xs, D)), float(np.vdot(xbar_e, D))
        assert abs(a - b) <= 4 * gap * abs(b), (a, b, gap)
    # g is linear in X, so <xbar, X> = <gbar, g> for both solves
    ip_s = float((c5["xbar"] * c5["X"]).sum().item())
    assert abs(ip_s - float((c5["G"] * c5["gbar"]).sum().item())) <= 1e-9 * abs(ip_s)
    ip_e = float(np.vdot(xbar_e, Xn))
    assert abs(ip_e - float(np.vdot(g_e, gbar))) <= 1e-9 * abs(ip_e)
    assert abs(ip_s - ip_e) <= 4 * gap * abs(ip_e)
