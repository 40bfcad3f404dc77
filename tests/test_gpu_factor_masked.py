"""The factor update over the observed entries (tucker_factor_update with a
mask) against the FP64 oracle's row-wise ridge solves, through the C ABI.

Bars: FP64 problems element-wise (max |A - A_ref| / max |A_ref|) <= 1e-10 (the
same normal equations accumulated in a different order; the rows' ridge systems
have condition numbers below 6e4 in these cases, so rounding stays near
1e-12); f32 problems <= 1e-5 (f32 output rounding of entries
whose size varies by a few units).  The cases cover orders 2-4, every mode
(the last mode takes the other pass layout), ranks that are not multiples of
4 (zero-padded 4 x 4 tiles), ranks above 16 (fewer rows per workgroup), a rank-1
mode, row blocks and inner tiles with ragged ends, a row with no observed entry,
NaN at unobserved entries (never read) and, at the C3 size, sampled rows.
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


def _case(dims, ranks, seed, dtype="f64", missing=0.3):
    p = workloads.tucker_tensor(dims, ranks, seed, dtype, factor="gaussian", noise=("sigma", 0.1),
                                missing=missing)
    rng = np.random.default_rng(seed + 7)
    t = workloads.NP_DTYPES[dtype]
    F = [(A + 0.1 * rng.standard_normal(A.shape)).astype(t) for A in p["factors_true"]]
    G = rng.standard_normal(ranks).astype(t)
    return p, F, G


CASES = [
    ((23, 19, 17), (3, 4, 5)),
    ((41, 37, 70), (5, 6, 7)),        # inner size 70: ragged 32-wide tiles
    ((13, 11, 9, 7), (2, 3, 2, 3)),   # order 4
    ((30, 20), (1, 9)),               # order 2, a rank-1 mode
    ((90, 33), (6, 4)),               # 90 rows: two row blocks, one ragged
    ((40, 24, 18), (20, 4, 6)),       # rank 20: 5 rank tiles, 32-row blocks
    ((36, 40, 12), (6, 33, 8)),       # rank 33: 9 rank tiles, 16-row blocks
]


@pytest.mark.parametrize("dims,ranks", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_masked_factor_update_matches_oracle(tk, dims, ranks, dtype):
    p, F, G = _case(dims, ranks, 70, dtype)
    lam = 1e-2
    mask = T(p["mask"].view(np.int32))
    F64 = [A.astype(np.float64) for A in F]
    for n in range(len(dims)):
        print(f"[masked factor] dims {dims} ranks {ranks} {dtype} mode {n}", flush=True)
        A = tk.factor_update(T(p["X"]), T(G), [T(B) for B in F], n, lam, mask=mask)
        ref = oracle.factor_update_masked(p["X"], G.astype(np.float64), F64, n, lam, p["mask"])
        assert elem_err(A.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-5), n


def test_masked_factor_update_full_mask_is_the_unmasked_update(tk):
    p, F, G = _case((21, 18, 15), (4, 3, 5), 71, missing=None)
    full = T(workloads.pack_mask(np.ones(p["X"].shape, bool)).view(np.int32))
    for n in range(3):
        Am = tk.factor_update(T(p["X"]), T(G), [T(B) for B in F], n, 1e-2, mask=full)
        Au = tk.factor_update(T(p["X"]), T(G), [T(B) for B in F], n, 1e-2)
        assert elem_err(Am.cpu().numpy(), Au.cpu().numpy()) <= 1e-10, n


def test_masked_factor_update_edge_rows_and_unread_entries(tk):
    p, F, G = _case((16, 14, 12), (3, 4, 2), 72, missing=0.2)
    X = p["X"].copy()
    obs = oracle.unpack_mask(p["mask"], X.shape)
    obs[:, 5, :] = False                       # row 5 of mode 1: nothing observed
    mk = workloads.pack_mask(obs)
    X[~obs] = np.nan                           # unobserved entries are never read
    A = tk.factor_update(T(X), T(G), [T(B) for B in F], 1, 1e-2, mask=T(mk.view(np.int32)))
    A = A.cpu().numpy()
    assert np.all(A[5] == 0.0)
    Xz = np.where(obs, X, 0.0)
    ref = oracle.factor_update_masked(Xz, G, F, 1, 1e-2, mk)
    assert elem_err(A, ref) <= 1e-10
    # lambda = 0 and an empty row: that row's system is singular
    with pytest.raises(tk.TuckerError) as e:
        tk.factor_update(T(X), T(G), [T(B) for B in F], 1, 0.0, mask=T(mk.view(np.int32)))
    assert e.value.code == 5  # TK_E_NOT_SPD


def test_masked_factor_update_c3_size_sampled_rows(tk):
    """C3 (128^4, rank 8^4, 10 % missing, f32): every mode, 6 rows each against
    the oracle's row solves."""
    prob = workloads.config_problem("c3")
    cfg = prob["cfg"]
    Fn = [np.ascontiguousarray(A.astype(np.float32)) for A in prob["factors_true"]]
    rng = np.random.default_rng(73)
    G = rng.standard_normal(cfg["ranks"]).astype(np.float32)
    X, F = T(prob["X"]), [T(A) for A in Fn]
    mask = T(prob["mask"].view(np.int32))
    Xn = prob["X"].astype(np.float64)
    F64 = [A.astype(np.float64) for A in Fn]
    for n in range(4):
        print(f"[masked factor] c3 mode {n}", flush=True)
        A = tk.factor_update(X, T(G), F, n, cfg["lam"], mask=mask).cpu().numpy()
        rows = sorted(rng.choice(128, 6, replace=False))
        ref = oracle.factor_update_masked(Xn, G.astype(np.float64), F64, n, cfg["lam"],
                                          prob["mask"], rows=rows)
        assert elem_err(A[rows], ref[rows]) <= 1e-5, n
