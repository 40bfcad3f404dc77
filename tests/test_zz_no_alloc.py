"""The no-allocation entry point (tucker_core_update_sketched_noalloc) against
tucker_core_update_sketched on the same inputs, through the C ABI.

Both run the same kernels, the first on the library's built-in device array
and the second on a caller workspace, so the bars are those of the sampled
update's parity tests: sample indices and weights bit-exact, the core within
1e-12 of the other call element by element (max |a - b| / max |b|).  Two
calls in a row, the second on a smaller problem, check that the array's
leftover contents from the first call do not leak into the second; the
second is also checked against the FP64 oracle (1e-10, FP64 mode).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2107_10654_amd as tk
from paper_2107_10654_amd import _lib as L

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def elem_err(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _both(p, lam, s, seed, precision):
    X = T(p["X"])
    F = [T(A) for A in p["factors_true"]]
    kw = dict(seed=seed, counter=3, precision=precision, refine_max=30, refine_tol=1e-13,
              return_samples=True, return_info=True)
    print(f"[no-alloc] dims {p['X'].shape} ranks {[A.shape[1] for A in F]} s {s} "
          f"{precision}: no-alloc call", flush=True)
    Gn, idn, wn, infn = tk.core_update_sketched_noalloc(X, F, lam, s, **kw)
    print("[no-alloc] workspace call", flush=True)
    Gw, idw, ww, infw = tk.core_update_sketched(X, F, lam, s, **kw)
    torch.cuda.synchronize()
    assert torch.equal(idn, idw)
    assert torch.equal(wn, ww)
    assert elem_err(Gn.cpu().numpy(), Gw.cpu().numpy()) <= 1e-12
    assert infn[0].item() == infw[0].item() and infn[2].item() == infw[2].item()
    if precision != "f64":
        assert infn[3].item() <= 1e-13
    return Gn, idn, wn


def test_noalloc_matches_workspace_call_twice():
    # first call: d = 384 (fused FP64 residual pass), BF16 Gram + refinement
    big = workloads.tucker_tensor((96, 80, 72), (8, 8, 6), seed=21, dtype="f64",
                                  factor="gaussian", noise=("sigma", 0.1))
    assert L.load().tucker_workspace_bytes is not None
    _both(big, 1e-2, 12000, 5, "bf16")
    # second call, smaller: d = 24, FP64 Gram; also against the oracle
    small = workloads.tucker_tensor((24, 20, 18), (3, 4, 2), seed=1, dtype="f64",
                                    factor="gaussian", noise=("sigma", 0.1))
    G, idx, w = _both(small, 1e-3, 1500, 7, "f64")
    Gr, ridx, rw, _ = oracle.fast_core_tensor_update(small["X"], small["factors_true"], 1e-3,
                                                     1500, 7, 3)
    np.testing.assert_array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10


def test_noalloc_rejects_problems_beyond_its_array():
    p = workloads.tucker_tensor((64, 64, 64), (4, 4, 4), seed=2, dtype="f32",
                                factor="qr", noise=("sigma", 0.01))
    X = T(p["X"])
    F = [T(A.astype(np.float32)) for A in p["factors_true"]]
    s = 4_000_000
    prob = tk.make_problem(X, F, 1e-3)
    o = L.TkSketchOpts()
    o.num_samples = s
    o.gram_precision = L.TK_BF16
    o.refine_max = 8
    o.refine_tol = 1e-13
    import ctypes
    assert L.load().tucker_workspace_bytes(ctypes.byref(prob), ctypes.byref(o),
                                           L.CALL_SKETCHED) > L.NOALLOC_SCRATCH_BYTES
    with pytest.raises(tk.TuckerError) as e:
        tk.core_update_sketched_noalloc(X, F, 1e-3, s, precision="bf16", check=False)
    assert e.value.code == 4  # TK_E_WORKSPACE
