"""Python binding of the gfx950 library (same names as the C ABI, minus the prefix).

PyTorch supplies device memory and the current stream; every computation runs
in the HIP kernels of ``libtucker_hip.so``.  Functions take CUDA (HIP) tensors:
X is row-major with shape (I_1, ..., I_N), factor n is (I_n, R_n), the core is
(R_1, ..., R_N); float64 or float32, all of one dtype.

``check=True`` synchronises the stream after the call and raises
``TuckerError`` when the library reported a data-dependent failure (not
positive definite, rank-deficient factor, refinement not converged).
"""
import ctypes

import torch

from . import _lib as L

_DT = {torch.float64: L.TK_F64, torch.float32: L.TK_F32}
PRECISIONS = {"f64": L.TK_F64, "f32": L.TK_F32, "bf16": L.TK_BF16}


class TuckerError(RuntimeError):
    def __init__(self, code, where):
        self.code = int(code)
        super().__init__(f"{where}: {L.STATUS_NAMES.get(self.code, self.code)}")


def _raise_if(code, where):
    if code != 0:
        raise TuckerError(code, where)


_ws = {}
_status = {}


def _workspace(nbytes, device):
    key = (device.index if device.index is not None else torch.cuda.current_device())
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws[key] = buf
    return buf


def _status_word(device):
    key = (device.index if device.index is not None else torch.cuda.current_device())
    s = _status.get(key)
    if s is None:
        s = torch.zeros(1, dtype=torch.int32, device=device)
        _status[key] = s
    return s


def release_workspace():
    """Free the cached workspace buffers."""
    _ws.clear()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def make_problem(X, factors, lam, mask=None):
    """Fill a TkProblem from tensors (X may be None for leverage scores)."""
    factors = list(factors)
    N = len(factors)
    if not 1 <= N <= L.MAX_ORDER:
        raise ValueError("order must be 1..8")
    dtype = factors[0].dtype
    if dtype not in _DT:
        raise TypeError("factors must be float64 or float32")
    p = L.TkProblem()
    p.order = N
    p.dtype = _DT[dtype]
    p.lam = float(lam)
    for n, A in enumerate(factors):
        _check_tensor(A, f"factor {n}", dtype)
        if A.dim() != 2:
            raise ValueError("factors must be 2-D")
        p.dims[n] = A.shape[0]
        p.ranks[n] = A.shape[1]
        p.factors[n] = A.data_ptr()
    if X is not None:
        _check_tensor(X, "X", dtype)
        if tuple(X.shape) != tuple(A.shape[0] for A in factors):
            raise ValueError(f"X shape {tuple(X.shape)} does not match the factors")
        p.X = X.data_ptr()
    if mask is not None:
        _check_tensor(mask, "mask", torch.int32)
        need = (int(torch.tensor(X.shape).prod()) + 31) // 32
        if mask.numel() < need:
            raise ValueError(f"mask needs {need} words")
        p.mask = mask.data_ptr()
    return p


SAMPLINGS = {"leverage": 0, "ridge": 1}


def _opts(samples, seed, counter, problem, precision, refine_max, refine_tol, eps=0.1, delta=0.1,
          stage_events=None, augmented=False, d_eff_lower=0.0, sampling="leverage", cdf_bits=0):
    o = L.TkSketchOpts()
    o.cdf_bits = int(cdf_bits)
    o.augmented = 1 if augmented else 0
    o.d_eff_lower = float(d_eff_lower)
    o.sampling = SAMPLINGS[sampling]
    o.stage_events = stage_events
    o.num_samples = int(samples) if samples is not None else 0
    o.eps, o.delta = float(eps), float(delta)
    o.seed = int(seed) & ((1 << 64) - 1)
    o.counter = int(counter) & ((1 << 64) - 1)
    o.problem = int(problem) & ((1 << 64) - 1)
    o.gram_precision = PRECISIONS[precision]
    o.refine_max = int(refine_max)
    o.refine_tol = float(refine_tol)
    return o


def _finish(device, status, where, check):
    if check:
        torch.cuda.current_stream(device).synchronize()
        _raise_if(int(status.item()), where)


def sample_count(d, eps, delta):
    """Alg. 1 sample count with beta' = 1/2."""
    return int(L.load().tucker_sample_count(int(d), float(eps), float(delta)))


def sample_count_augmented(d, eps, delta, d_eff_lower=0.0):
    """Alg. 1 sample count for augmented draws: beta' = 1/(1 + c), c = min{1, d - d'_eff}."""
    return int(L.load().tucker_sample_count_augmented(int(d), float(eps), float(delta),
                                                      float(d_eff_lower)))


def masked_sample_bound(factors, lam, eps=0.1, delta=0.1, d_eff_lower=0.0):
    """Cor. B.1's overestimate for missing data and Alg. 1's count with it:
    (1/beta bound, prod_n sigma_max(A(n))^2, beta', s) as floats."""
    lib = L.load()
    p = make_problem(None, factors, lam)
    dev = factors[0].device
    out = torch.empty(4, dtype=torch.float64, device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_MASKED_BOUND)
    ws = _workspace(nb, dev)
    _raise_if(lib.tucker_masked_sample_bound(ctypes.byref(p), float(eps), float(delta),
                                             float(d_eff_lower), _ptr(out), _ptr(ws), ws.numel(),
                                             _stream()), "masked_sample_bound")
    return tuple(out.cpu().tolist())


def leverage_scores(factors, check=True):
    """Per-mode leverage scores (concatenated float64) and integer CDFs (int64 view of uint64)."""
    lib = L.load()
    p = make_problem(None, factors, 0.0)
    dev = factors[0].device
    total = sum(A.shape[0] for A in factors)
    scores = torch.empty(total, dtype=torch.float64, device=dev)
    cdf = torch.empty(total, dtype=torch.int64, device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_LEVERAGE)
    ws = _workspace(nb, dev)
    st = _status_word(dev)
    _raise_if(lib.tucker_leverage_scores(ctypes.byref(p), _ptr(scores), _ptr(cdf), _ptr(st),
                                         _ptr(ws), ws.numel(), _stream()), "leverage_scores")
    _finish(dev, st, "leverage_scores", check)
    return scores, cdf


def sample(dims, cdf, s, seed, counter=0, problem=0):
    """Product-distribution samples: idx (N, s) int32 and weight (s,) float64."""
    lib = L.load()
    _check_tensor(cdf, "cdf", torch.int64)
    dims = [int(v) for v in dims]
    if not 1 <= len(dims) <= L.MAX_ORDER or min(dims) < 1:
        raise ValueError("dims must hold 1..8 sizes, each >= 1")
    if cdf.numel() != sum(dims):
        raise ValueError(f"cdf must hold sum(dims) = {sum(dims)} entries, got {cdf.numel()}")
    if int(s) < 1:
        raise ValueError("s must be >= 1")
    dev = cdf.device
    N = len(dims)
    idx = torch.empty((N, int(s)), dtype=torch.int32, device=dev)
    w = torch.empty(int(s), dtype=torch.float64, device=dev)
    dims_c = (ctypes.c_int64 * N)(*[int(v) for v in dims])
    _raise_if(lib.tucker_sample(N, dims_c, _ptr(cdf), int(s), int(seed) & ((1 << 64) - 1),
                                int(counter), int(problem), _ptr(idx), _ptr(w), _stream()),
              "sample")
    return idx, w


def ridge_tables(factors, lam):
    """Tables of the lambda-ridge leverage scores of K (mixture over singular-value
    tuples): tuple CDF (d,), column CDFs (sum I_n R_n,) as int64 views of uint64,
    and d_eff."""
    lib = L.load()
    p = make_problem(None, factors, lam)
    dev = factors[0].device
    d = 1
    for A in factors:
        d *= A.shape[1]
    tq = sum(A.shape[0] * A.shape[1] for A in factors)
    tcdf = torch.empty(d, dtype=torch.int64, device=dev)
    ccdf = torch.empty(tq, dtype=torch.int64, device=dev)
    deff = torch.empty(1, dtype=torch.float64, device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_RIDGE_TABLES)
    ws = _workspace(nb, dev)
    _raise_if(lib.tucker_ridge_tables(ctypes.byref(p), _ptr(tcdf), _ptr(ccdf), _ptr(deff),
                                      _ptr(ws), ws.numel(), _stream()), "ridge_tables")
    return tcdf, ccdf, float(deff.item())


def sample_ridge(dims, ranks, tuple_cdf, col_cdf, s, seed, counter=0, problem=0, augmented=False,
                 d_eff_lower=0.0):
    """Draws from the ridge-score mixture of K: idx (N, s) int32, weight (s,) float64."""
    lib = L.load()
    _check_tensor(tuple_cdf, "tuple_cdf", torch.int64)
    _check_tensor(col_cdf, "col_cdf", torch.int64)
    dims = [int(v) for v in dims]
    ranks = [int(v) for v in ranks]
    d = 1
    for r in ranks:
        d *= r
    if tuple_cdf.numel() != d or col_cdf.numel() != sum(a * b for a, b in zip(dims, ranks)):
        raise ValueError("table lengths do not match dims and ranks")
    dev = tuple_cdf.device
    N = len(dims)
    idx = torch.empty((N, int(s)), dtype=torch.int32, device=dev)
    w = torch.empty(int(s), dtype=torch.float64, device=dev)
    _raise_if(lib.tucker_sample_ridge(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int32 * N)(*ranks),
                                      _ptr(tuple_cdf), _ptr(col_cdf), int(s),
                                      int(seed) & ((1 << 64) - 1), int(counter), int(problem),
                                      1 if augmented else 0, float(d_eff_lower), _ptr(idx),
                                      _ptr(w), _stream()), "sample_ridge")
    return idx, w


def sample_augmented(dims, ranks, cdf, s, seed, counter=0, problem=0, d_eff_lower=0.0):
    """Draws from Alg. 1's augmented distribution: idx (N, s) int32 (ridge draws
    stored as dims[n] + digit) and weight (s,) float64."""
    lib = L.load()
    _check_tensor(cdf, "cdf", torch.int64)
    dims = [int(v) for v in dims]
    ranks = [int(v) for v in ranks]
    if not 1 <= len(dims) <= L.MAX_ORDER or len(ranks) != len(dims) or min(dims) < 1:
        raise ValueError("dims and ranks must hold 1..8 sizes each")
    if cdf.numel() != sum(dims):
        raise ValueError(f"cdf must hold sum(dims) = {sum(dims)} entries, got {cdf.numel()}")
    if int(s) < 1:
        raise ValueError("s must be >= 1")
    dev = cdf.device
    N = len(dims)
    idx = torch.empty((N, int(s)), dtype=torch.int32, device=dev)
    w = torch.empty(int(s), dtype=torch.float64, device=dev)
    dims_c = (ctypes.c_int64 * N)(*dims)
    ranks_c = (ctypes.c_int32 * N)(*ranks)
    _raise_if(lib.tucker_sample_augmented(N, dims_c, ranks_c, _ptr(cdf), int(s),
                                          int(seed) & ((1 << 64) - 1), int(counter), int(problem),
                                          float(d_eff_lower), _ptr(idx), _ptr(w), _stream()),
              "sample_augmented")
    return idx, w


def core_update_sketched(X, factors, lam, samples, seed=0, counter=0, problem=0, precision="f64",
                         mask=None, idx=None, weight=None, refine_max=20, refine_tol=1e-13,
                         return_samples=False, return_info=False, check=True, out=None,
                         stage_events=None, status=None, augmented=False, d_eff_lower=0.0,
                         sampling="leverage", cdf_bits=0):
    """Sampled core update (Alg. 3 with Alg. 1); returns the core (and optionally samples/info).

    stage_events: optional address of an array of NUM_STAGE_EVENTS hipEvent_t
    handles that the library records at its stage boundaries.
    status: optional int32 device tensor of one element that receives the call's
    status word (default: a per-device word shared by all calls).
    augmented: draw from Alg. 1's augmented distribution (lower bound d_eff_lower
    of the effective dimension) and solve on the sampled rows of [K; sqrt(lam) I].
    sampling: "leverage" (product of the factor leverage scores) or "ridge" (the
    lambda-ridge leverage scores of K, a mixture over singular-value tuples).
    cdf_bits: fixed-point bits Q of the integer sampling weights ceil(l 2^Q)
    (0: the library default, TK_Q_BITS = 24; else 8..40).
    """
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    o = _opts(samples, seed, counter, problem, precision, refine_max, refine_tol,
              stage_events=stage_events, augmented=augmented, d_eff_lower=d_eff_lower,
              sampling=sampling, cdf_bits=cdf_bits)
    dev = X.device
    N = len(factors)
    d = int(torch.tensor([A.shape[1] for A in factors]).prod())
    s = int(samples) if samples else (sample_count_augmented(d, 0.1, 0.1, d_eff_lower)
                                      if augmented else sample_count(d, 0.1, 0.1))
    if idx is not None:
        _check_tensor(idx, "idx", torch.int32)
        _check_tensor(weight, "weight", torch.float64)
        if tuple(idx.shape) != (N, s) or weight.numel() != s:
            raise ValueError("idx must be (N, s) and weight (s,)")
    core = out if out is not None else torch.empty([A.shape[1] for A in factors], dtype=X.dtype,
                                                   device=dev)
    idx_out = w_out = None
    if return_samples and idx is None:
        idx_out = torch.empty((N, s), dtype=torch.int32, device=dev)
        w_out = torch.empty(s, dtype=torch.float64, device=dev)
    info = torch.empty(L.INFO_LEN, dtype=torch.float64, device=dev) if return_info else None
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), ctypes.byref(o), L.CALL_SKETCHED)
    if nb == 0:
        raise ValueError("unsupported problem for the sketched update")
    ws = _workspace(nb, dev)
    if status is not None:
        _check_tensor(status, "status", torch.int32)
        if status.numel() != 1:
            raise ValueError("status must hold one int32 word")
    st = status if status is not None else _status_word(dev)
    _raise_if(lib.tucker_core_update_sketched(ctypes.byref(p), ctypes.byref(o), _ptr(idx),
                                              _ptr(weight), _ptr(idx_out), _ptr(w_out), _ptr(core),
                                              _ptr(st), _ptr(info), _ptr(ws), ws.numel(),
                                              _stream()), "core_update_sketched")
    _finish(dev, st, "core_update_sketched", check)
    res = [core]
    if return_samples:
        res += [idx if idx is not None else idx_out, weight if weight is not None else w_out]
    if return_info:
        res.append(info)
    return res[0] if len(res) == 1 else tuple(res)


def core_update_sketched_noalloc(X, factors, lam, samples, seed=0, counter=0, problem=0,
                                 precision="f64", mask=None, idx=None, weight=None, refine_max=20,
                                 refine_tol=1e-13, return_samples=False, return_info=False,
                                 check=True, out=None, status=None):
    """The sampled core update of core_update_sketched through the library's
    no-allocation entry point: its workspace is a device array built into the
    library (NOALLOC_SCRATCH_BYTES per GPU), so the call allocates nothing in
    the library.  Raises TuckerError(TK_E_WORKSPACE) for problems that need
    more workspace than that.  Calls on one GPU share the array: do not overlap
    them in time."""
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    o = _opts(samples, seed, counter, problem, precision, refine_max, refine_tol)
    dev = X.device
    N = len(factors)
    s = int(samples) if samples else sample_count(
        int(torch.tensor([A.shape[1] for A in factors]).prod()), 0.1, 0.1)
    if idx is not None:
        _check_tensor(idx, "idx", torch.int32)
        _check_tensor(weight, "weight", torch.float64)
        if tuple(idx.shape) != (N, s) or weight.numel() != s:
            raise ValueError("idx must be (N, s) and weight (s,)")
    core = out if out is not None else torch.empty([A.shape[1] for A in factors], dtype=X.dtype,
                                                   device=dev)
    idx_out = w_out = None
    if return_samples and idx is None:
        idx_out = torch.empty((N, s), dtype=torch.int32, device=dev)
        w_out = torch.empty(s, dtype=torch.float64, device=dev)
    info = torch.empty(L.INFO_LEN, dtype=torch.float64, device=dev) if return_info else None
    if status is not None:
        _check_tensor(status, "status", torch.int32)
        if status.numel() != 1:
            raise ValueError("status must hold one int32 word")
    st = status if status is not None else _status_word(dev)
    _raise_if(lib.tucker_core_update_sketched_noalloc(
        ctypes.byref(p), ctypes.byref(o), _ptr(idx), _ptr(weight), _ptr(idx_out), _ptr(w_out),
        _ptr(core), _ptr(st), _ptr(info), _stream()), "core_update_sketched_noalloc")
    _finish(dev, st, "core_update_sketched_noalloc", check)
    res = [core]
    if return_samples:
        res += [idx if idx is not None else idx_out, weight if weight is not None else w_out]
    if return_info:
        res.append(info)
    return res[0] if len(res) == 1 else tuple(res)


def sketched_system(X, factors, lam, idx, weight, precision="f64", mask=None, check=True,
                    augmented=False):
    """The sketched normal equations (M, b) of the sampled update on the samples (idx, weight),
    in the solver's whitened coordinates: M = sum_t w_t q_t q_t^T + lam P (lower triangle
    valid), b = sum_t w_t x_t q_t, q_t the Kronecker row of L_n^{-1} a^(n)_{i_n}."""
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    N = len(factors)
    _check_tensor(idx, "idx", torch.int32)
    _check_tensor(weight, "weight", torch.float64)
    s = idx.shape[1]
    if idx.dim() != 2 or idx.shape[0] != N or weight.numel() != s:
        raise ValueError("idx must be (N, s) and weight (s,)")
    o = _opts(s, 0, 0, 0, precision, 0, 0.0, augmented=augmented)
    dev = X.device
    d = int(torch.tensor([A.shape[1] for A in factors]).prod())
    M = torch.empty((d, d), dtype=torch.float64, device=dev)
    b = torch.empty(d, dtype=torch.float64, device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), ctypes.byref(o), L.CALL_SKETCHED)
    if nb == 0:
        raise ValueError("unsupported problem for the sketched update")
    ws = _workspace(nb, dev)
    st = _status_word(dev)
    _raise_if(lib.tucker_sketched_system(ctypes.byref(p), ctypes.byref(o), _ptr(idx),
                                         _ptr(weight), _ptr(M), _ptr(b), _ptr(st), _ptr(ws),
                                         ws.numel(), _stream()), "sketched_system")
    _finish(dev, st, "sketched_system", check)
    return M, b


def core_update_sketched_adjoint(X, factors, lam, idx, weight, core, core_bar, precision="f64",
                                 mask=None, refine_max=20, refine_tol=1e-13, want_x=True,
                                 return_info=False, check=True):
    """Adjoint of the sampled core update with the sample set (idx, weight) held fixed.

    Returns (factor_bars, x_bar) -- the gradients of <core_bar, g> w.r.t. the
    factors and the tensor entries (x_bar is None when want_x is False).
    """
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    N = len(factors)
    _check_tensor(idx, "idx", torch.int32)
    _check_tensor(weight, "weight", torch.float64)
    s = idx.shape[1]
    if idx.dim() != 2 or idx.shape[0] != N or weight.numel() != s:
        raise ValueError("idx must be (N, s) and weight (s,)")
    _check_tensor(core, "core", X.dtype)
    _check_tensor(core_bar, "core_bar", X.dtype)
    o = _opts(s, 0, 0, 0, precision, refine_max, refine_tol)
    dev = X.device
    fbar = [torch.empty_like(A) for A in factors]
    fptrs = (ctypes.c_void_p * N)(*[t.data_ptr() for t in fbar])
    xbar = torch.empty_like(X) if want_x else None
    info = torch.empty(L.INFO_LEN, dtype=torch.float64, device=dev) if return_info else None
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), ctypes.byref(o), L.CALL_ADJOINT)
    if nb == 0:
        raise ValueError("unsupported problem for the adjoint")
    ws = _workspace(nb, dev)
    st = _status_word(dev)
    _raise_if(lib.tucker_core_update_sketched_adjoint(
        ctypes.byref(p), ctypes.byref(o), _ptr(idx), _ptr(weight), _ptr(core), _ptr(core_bar),
        fptrs, _ptr(xbar), _ptr(st), _ptr(info), _ptr(ws), ws.numel(), _stream()),
        "core_update_sketched_adjoint")
    _finish(dev, st, "core_update_sketched_adjoint", check)
    if return_info:
        return fbar, xbar, info
    return fbar, xbar


def core_update_exact(X, factors, lam, mask=None, check=True, out=None):
    """Exact core update (eigen form of the Kronecker normal equations; with a
    mask, preconditioned conjugate gradients over the observed entries)."""
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    dev = X.device
    core = out if out is not None else torch.empty([A.shape[1] for A in factors], dtype=X.dtype,
                                                   device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_EXACT)
    ws = _workspace(nb, dev)
    st = _status_word(dev)
    _raise_if(lib.tucker_core_update_exact(ctypes.byref(p), _ptr(core), _ptr(st), _ptr(ws),
                                           ws.numel(), _stream()), "core_update_exact")
    _finish(dev, st, "core_update_exact", check)
    return core


def factor_update(X, G, factors, mode, lam, out=None, check=True, mask=None):
    """Row-wise ridge update of factor `mode` (Alg. 2); returns the new factor.
    With ``mask`` (int32 view of the LSB-first bit mask) every row is fitted to
    its observed entries only."""
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    _check_tensor(G, "core", X.dtype)
    dev = X.device
    A = out if out is not None else torch.empty_like(factors[mode])
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_FACTOR)
    ws = _workspace(nb, dev)
    st = _status_word(dev)
    _raise_if(lib.tucker_factor_update(ctypes.byref(p), _ptr(G), int(mode), _ptr(A), _ptr(st),
                                       _ptr(ws), ws.numel(), _stream()), "factor_update")
    _finish(dev, st, "factor_update", check)
    return A


def loss(X, G, factors, lam, mask=None, sync=True):
    """(L, sum of squared residuals, observed count) of the regularised Tucker loss (Sec. 2)."""
    lib = L.load()
    p = make_problem(X, factors, lam, mask)
    _check_tensor(G, "core", X.dtype)
    dev = X.device
    out = torch.empty(3, dtype=torch.float64, device=dev)
    nb = lib.tucker_workspace_bytes(ctypes.byref(p), None, L.CALL_LOSS)
    ws = _workspace(nb, dev)
    _raise_if(lib.tucker_loss(ctypes.byref(p), _ptr(G), _ptr(out), _ptr(ws), ws.numel(), _stream()),
              "loss")
    if not sync:
        return out
    v = out.cpu().tolist()
    return v[0], v[1], v[2]


def als(X, G0, factors0, lam, iters, core="exact", samples=None, seed=0, precision="f64",
        record=None, mask=None):
    """Alg. 2 on the GPU: factor updates 1..N then the core (exact or sampled, counter = iteration).
    With ``mask`` every update fits the observed entries only.

    Returns (G, factors, history) with history[k] = (loss, rmse) after iteration k.
    """
    G = G0.clone()
    F = [A.clone() for A in factors0]
    hist = []
    for it in range(iters):
        for n in range(len(F)):
            F[n] = factor_update(X, G, F, n, lam, mask=mask)
            if record is not None:
                record.append(("factor", it, n, loss(X, G, F, lam, mask=mask)))
        if core == "exact":
            G = core_update_exact(X, F, lam, mask=mask)
        else:
            G = core_update_sketched(X, F, lam, samples, seed=seed, counter=it,
                                     precision=precision, mask=mask)
        Lv, sq, cnt = loss(X, G, F, lam, mask=mask)
        hist.append((Lv, (sq / cnt) ** 0.5))
        if record is not None:
            record.append(("core", it, -1, (Lv, sq, cnt)))
    return G, F, hist


# ---------------------------------------------------------------- batches
def _batch(Xs, factors_list, lams, samples, seeds, counters, problems, precision, refine_max,
           refine_tol, masks):
    count = len(Xs)
    if not 1 <= count <= L.MAX_BATCH:
        raise ValueError(f"batch of 1..{L.MAX_BATCH} problems")

    def per(v, default):
        if v is None:
            return [default] * count
        return list(v) if isinstance(v, (list, tuple)) else [v] * count

    lams, samples = per(lams, 0.0), per(samples, None)
    seeds, counters = per(seeds, 0), per(counters, 0)
    problems = per(problems, None)
    masks = per(masks, None)
    P = (L.TkProblem * count)()
    O = (L.TkSketchOpts * count)()
    for k in range(count):
        P[k] = make_problem(Xs[k], factors_list[k], lams[k], masks[k])
        O[k] = _opts(samples[k], seeds[k], counters[k], k if problems[k] is None else problems[k],
                     precision, refine_max, refine_tol)
    return P, O


def _config(config):
    if config is None:
        return None
    c = L.TkBatchConfig()
    c.tile, c.wg_per_cu = int(config["tile"]), int(config["wg_per_cu"])
    return c


def tune_batched(Xs, factors_list, lams, samples, seeds=None, counters=None, problems=None,
                 precision="bf16", masks=None):
    """Time every candidate Gram configuration of the batched call; returns (best, times_ms)."""
    lib = L.load()
    P, O = _batch(Xs, factors_list, lams, samples, seeds, counters, problems, precision, 0, 0.0,
                  masks)
    count = len(Xs)
    nb = lib.tucker_workspace_bytes_batched(P, O, count, None)
    if nb == 0:
        raise ValueError("unsupported batch")
    dev = Xs[0].device
    ws = _workspace(nb, dev)
    best = L.TkBatchConfig()
    times = (ctypes.c_double * 16)()
    n = ctypes.c_int32(0)
    _raise_if(lib.tucker_tune_batched(P, O, count, _ptr(ws), ws.numel(), _stream(),
                                      ctypes.byref(best), times, ctypes.byref(n)), "tune_batched")
    return {"tile": best.tile, "wg_per_cu": best.wg_per_cu}, list(times[:n.value])


def core_update_sketched_batched(Xs, factors_list, lams, samples, seeds=None, counters=None,
                                 problems=None, precision="bf16", config=None, refine_max=12,
                                 refine_tol=1e-13, masks=None, out=None, return_info=False,
                                 check=True, workspace=None, status=None, info=None):
    """Sampled core updates of a batch of problems with one persistent Gram launch.

    problems[k] (default k) is the sampler's problem field of problem k, so
    problem k draws the samples of core_update_sketched(..., problem=k).
    Returns the list of cores (and the (count, INFO_LEN) info tensor).  `info`
    (optional, (count, INFO_LEN) float64 on the device) receives the per-problem
    info rows; it is returned when return_info is set.
    """
    lib = L.load()
    P, O = _batch(Xs, factors_list, lams, samples, seeds, counters, problems, precision,
                  refine_max, refine_tol, masks)
    count = len(Xs)
    cfg = _config(config)
    dev = Xs[0].device
    cores = out if out is not None else [
        torch.empty([A.shape[1] for A in F], dtype=X.dtype, device=dev)
        for X, F in zip(Xs, factors_list)]
    ptrs = (ctypes.c_void_p * count)(*[c.data_ptr() for c in cores])
    st = status if status is not None else torch.zeros(count, dtype=torch.int32, device=dev)
    if info is None and return_info:
        info = torch.empty((count, L.INFO_LEN), dtype=torch.float64, device=dev)
    if info is not None and (tuple(info.shape) != (count, L.INFO_LEN) or
                             info.dtype != torch.float64 or not info.is_contiguous()):
        raise ValueError("info must be a contiguous (count, INFO_LEN) float64 tensor")
    nb = lib.tucker_workspace_bytes_batched(P, O, count, ctypes.byref(cfg) if cfg else None)
    if nb == 0:
        raise ValueError("unsupported batch")
    ws = workspace if workspace is not None else _workspace(nb, dev)
    if ws.numel() < nb:
        raise ValueError(f"workspace needs {nb} bytes")
    _raise_if(lib.tucker_core_update_sketched_batched(
        P, O, count, ctypes.byref(cfg) if cfg else None, ptrs, _ptr(st), _ptr(info), _ptr(ws),
        ws.numel(), _stream()), "core_update_sketched_batched")
    if check:
        torch.cuda.current_stream(dev).synchronize()
        bad = st.cpu().tolist()
        for k, code in enumerate(bad):
            _raise_if(code, f"core_update_sketched_batched[{k}]")
    if return_info:
        return cores, info
    return cores


class BatchedSketchedUpdate:
    """A batched sampled update captured once in a CUDA (HIP) graph.

    The inputs are read at every replay (their contents may change between
    replays; shapes and addresses may not); the sampler's seed, counter and
    problem fields are fixed at capture.  replay() returns the list of cores.
    """

    def __init__(self, Xs, factors_list, lams, samples, seeds=None, counters=None, problems=None,
                 precision="bf16", config=None, refine_max=12, refine_tol=1e-13, masks=None):
        lib = L.load()
        self._args = (Xs, factors_list, lams, samples, seeds, counters, problems, precision)
        P, O = _batch(Xs, factors_list, lams, samples, seeds, counters, problems, precision,
                      refine_max, refine_tol, masks)
        cfg = _config(config)
        dev = Xs[0].device
        nb = lib.tucker_workspace_bytes_batched(P, O, len(Xs), ctypes.byref(cfg) if cfg else None)
        if nb == 0:
            raise ValueError("unsupported batch")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.status = torch.zeros(len(Xs), dtype=torch.int32, device=dev)
        self.info = torch.empty((len(Xs), L.INFO_LEN), dtype=torch.float64, device=dev)
        self.cores = [torch.empty([A.shape[1] for A in F], dtype=X.dtype, device=dev)
                      for X, F in zip(Xs, factors_list)]
        kw = dict(seeds=seeds, counters=counters, problems=problems, precision=precision,
                  config=config, refine_max=refine_max, refine_tol=refine_tol, masks=masks,
                  out=self.cores, workspace=self.workspace, status=self.status, info=self.info)
        # eager run first (checks the status words), then capture
        core_update_sketched_batched(Xs, factors_list, lams, samples, check=True, **kw)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            core_update_sketched_batched(Xs, factors_list, lams, samples, check=False, **kw)

    def replay(self):
        self.graph.replay()
        return self.cores
