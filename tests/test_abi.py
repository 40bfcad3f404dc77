"""CPU-side checks of the C ABI: the library loads, exports every function that
include/tucker.h declares, and validates arguments on the host (no GPU needed:
these paths return before anything is enqueued)."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
from paper_2107_10654_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tucker.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tucker_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return L.load()


def test_header_declares_binding_functions():
    assert header_functions() == L.exported_symbols()


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (tucker_\w+)", out))
    missing = [f for f in header_functions() if f not in exported]
    assert not missing, missing
    for f in header_functions():
        assert getattr(lib, f) is not None


def test_struct_layouts_match_header(lib):
    # tk_problem: int32 order, int64 dims[8], int32 ranks[8], enum dtype, 2 pointers,
    # 8 pointers, double -> natural alignment
    assert ctypes.sizeof(L.TkProblem) == 4 + 4 + 64 + 32 + 4 + 4 + 8 + 8 + 64 + 8
    # ... int32 gram_precision, int32 refine_max, double, pointer, int32 augmented
    # (+4 padding), double d_eff_lower, int32 sampling, int32 cdf_bits
    assert ctypes.sizeof(L.TkSketchOpts) == 8 * 6 + 4 + 4 + 8 + 8 + 8 + 8 + 8
    assert L.TkSketchOpts.sampling.offset == 88 and L.TkSketchOpts.cdf_bits.offset == 92


def _problem(dims, ranks, dtype=L.TK_F32, lam=1e-2):
    p = L.TkProblem()
    p.order = len(dims)
    for n, (I, R) in enumerate(zip(dims, ranks)):
        p.dims[n] = I
        p.ranks[n] = R
        p.factors[n] = 0x1000  # never dereferenced on the host paths tested here
    p.dtype = dtype
    p.X = 0x1000
    p.lam = lam
    return p


def _opts(s=1024, prec=L.TK_BF16):
    o = L.TkSketchOpts()
    o.num_samples = s
    o.gram_precision = prec
    o.refine_max = 10
    o.refine_tol = 1e-13
    return o


def test_sample_count_matches_oracle(lib):
    for d in (1, 8, 64, 4096, 13824):
        for eps, delta in ((0.1, 0.1), (0.05, 0.2)):
            assert lib.tucker_sample_count(d, eps, delta) == oracle.s_theory(d, eps, delta)
    assert lib.tucker_sample_count(0, 0.1, 0.1) == 0
    assert lib.tucker_sample_count(8, 0.1, 1.5) == 0
    for d in (1, 8, 64, 4096):
        for deff in (0.0, d - 0.25, d - 0.5, float(d), d + 3.0):
            assert lib.tucker_sample_count_augmented(d, 0.1, 0.1, deff) == \
                oracle.s_theory_augmented(d, 0.1, 0.1, deff), (d, deff)


def test_workspace_sizes(lib):
    p = _problem((512, 512, 512), (16, 16, 16))
    o = _opts(131072)
    for call in range(6):
        n = lib.tucker_workspace_bytes(ctypes.byref(p), ctypes.byref(o), call)
        assert n > 0, call
    # unsupported shapes give 0
    bad = _problem((8, 8), (9, 2))            # rank above the dimension
    assert lib.tucker_workspace_bytes(ctypes.byref(bad), ctypes.byref(o), 1) == 0
    bad = _problem((100,) * 3, (65, 1, 1))    # rank above 64
    assert lib.tucker_workspace_bytes(ctypes.byref(bad), ctypes.byref(o), 1) == 0
    bad = _problem((100,) * 3, (40, 40, 40))  # d above 16384
    assert lib.tucker_workspace_bytes(ctypes.byref(bad), ctypes.byref(o), 1) == 0


def test_host_argument_errors(lib):
    p = _problem((64, 64, 64), (4, 4, 4))
    o = _opts()
    ws = ctypes.create_string_buffer(16)
    st = ctypes.c_void_p(0)
    core = ctypes.c_void_p(0x2000)
    f = lib.tucker_core_update_sketched
    # workspace too small
    assert f(ctypes.byref(p), ctypes.byref(o), None, None, None, None, core, None, None,
             ws, 16, st) == 4
    # bad precision
    o2 = _opts(prec=7)
    assert f(ctypes.byref(p), ctypes.byref(o2), None, None, None, None, core, None, None,
             ws, 16, st) == 3
    # idx without weights
    assert f(ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(0x10), None, None, None, core,
             None, None, ws, 16, st) == 1
    # fixed-point bits of the sampling weights outside 8..40 (0 selects the default)
    for q in (7, 41, -1):
        oq = _opts()
        oq.cdf_bits = q
        assert f(ctypes.byref(p), ctypes.byref(oq), None, None, None, None, core, None, None,
                 ws, 16, st) == 1
    # bad order / dtype / lambda
    bad = _problem((64, 64, 64), (4, 4, 4))
    bad.order = 0
    assert f(ctypes.byref(bad), ctypes.byref(o), None, None, None, None, core, None, None, ws, 16,
             st) == 2
    bad = _problem((64, 64, 64), (4, 4, 4), dtype=2)
    assert f(ctypes.byref(bad), ctypes.byref(o), None, None, None, None, core, None, None, ws, 16,
             st) == 3
    bad = _problem((64, 64, 64), (4, 4, 4), lam=-1.0)
    assert f(ctypes.byref(bad), ctypes.byref(o), None, None, None, None, core, None, None, ws, 16,
             st) == 1
    # factor update: bad mode; a masked order-1 problem; too small a workspace
    assert lib.tucker_factor_update(ctypes.byref(p), core, 3, core, core, ws, 16, st) == 1
    pm = _problem((64,), (4,))
    pm.mask = 0x3000
    assert lib.tucker_factor_update(ctypes.byref(pm), core, 0, core, core, ws, 16, st) == 2
    pm = _problem((64, 64, 64), (4, 4, 4))
    pm.mask = 0x3000
    assert lib.tucker_factor_update(ctypes.byref(pm), core, 0, core, core, ws, 16, st) == 4
    # adjoint: frozen samples, core and cotangent are required
    fb = (ctypes.c_void_p * 3)(0x10, 0x10, 0x10)
    adj = lib.tucker_core_update_sketched_adjoint
    assert adj(ctypes.byref(p), ctypes.byref(o), None, None, core, core, fb, None, None, None, ws,
               16, st) == 1
    assert adj(ctypes.byref(p), ctypes.byref(o), core, core, core, core, None, None, None, None,
               ws, 16, st) == 1
    assert adj(ctypes.byref(p), ctypes.byref(o), core, core, core, core, fb, None, None, None, ws,
               16, st) == 4
    # sampler arguments
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.tucker_sample(0, dims, core, 10, 0, 0, 0, core, core, st) == 1
    assert lib.tucker_sample(3, dims, core, 0, 0, 0, 0, core, core, st) == 1


def test_batched_host_checks(lib):
    n = 3
    P = (L.TkProblem * n)(*[_problem((40 + k, 30, 20), (4, 3, 2)) for k in range(n)])
    O = (L.TkSketchOpts * n)(*[_opts(500) for _ in range(n)])
    nb = lib.tucker_workspace_bytes_batched(P, O, n, None)
    cfg = L.TkBatchConfig(64, 4)
    nb64 = lib.tucker_workspace_bytes_batched(P, O, n, ctypes.byref(cfg))
    assert nb >= nb64 > 0
    assert lib.tucker_workspace_bytes_batched(P, O, 0, None) == 0
    bad = L.TkBatchConfig(96, 3)
    assert lib.tucker_workspace_bytes_batched(P, O, n, ctypes.byref(bad)) == 0
    ws = ctypes.create_string_buffer(16)
    outs = (ctypes.c_void_p * n)(0x10, 0x10, 0x10)
    st = ctypes.c_void_p(0x10)
    f = lib.tucker_core_update_sketched_batched
    assert f(P, O, n, None, outs, st, None, ws, 16, None) == 4  # workspace too small
    assert f(P, O, 0, None, outs, st, None, ws, 16, None) == 1
    assert f(P, O, n, ctypes.byref(bad), outs, st, None, ws, nb, None) == 1
    O64 = (L.TkSketchOpts * n)(*[_opts(500, prec=L.TK_F64) for _ in range(n)])
    assert f(P, O64, n, None, outs, st, None, ws, 16, None) == 3  # batches use FP32 / BF16 Grams
    mixed = (L.TkSketchOpts * n)(_opts(500), _opts(500, prec=L.TK_F32), _opts(500))
    assert f(P, mixed, n, None, outs, st, None, ws, 16, None) == 3
    best = L.TkBatchConfig()
    assert lib.tucker_tune_batched(P, O, n, ws, 16, None, ctypes.byref(best), None, None) == 4


def test_status_strings(lib):
    for code, name in L.STATUS_NAMES.items():
        assert lib.tucker_status_string(code)
    assert lib.tucker_abi_version() >= 1
