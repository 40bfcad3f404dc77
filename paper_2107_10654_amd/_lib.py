"""ctypes view of the C ABI in ``include/tucker.h`` (libtucker_hip.so).

Only argument marshalling lives here; every step of the computation runs in
the HIP library.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

MAX_ORDER = 8
MAX_RANK = 64
Q_BITS = 24
INFO_LEN = 8
NUM_STAGE_EVENTS = 10
NOALLOC_SCRATCH_BYTES = 128 << 20

TK_F64, TK_F32, TK_BF16 = 0, 1, 2
(CALL_LEVERAGE, CALL_SKETCHED, CALL_EXACT, CALL_FACTOR, CALL_LOSS, CALL_ADJOINT,
 CALL_MASKED_BOUND, CALL_RIDGE_TABLES) = range(8)

STATUS_NAMES = {
    0: "TK_OK", 1: "TK_E_ARG", 2: "TK_E_SHAPE", 3: "TK_E_DTYPE", 4: "TK_E_WORKSPACE",
    5: "TK_E_NOT_SPD", 6: "TK_E_RANK_DEFICIENT", 7: "TK_E_NO_CONVERGE", 8: "TK_E_HIP",
}

LIB_PATH = os.environ.get("TK_LIBRARY_PATH") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libtucker_hip.so")


class TkProblem(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("ranks", ctypes.c_int32 * MAX_ORDER),
        ("dtype", ctypes.c_int32),
        ("X", ctypes.c_void_p),
        ("mask", ctypes.c_void_p),
        ("factors", ctypes.c_void_p * MAX_ORDER),
        ("lam", ctypes.c_double),
    ]


class TkSketchOpts(ctypes.Structure):
    _fields_ = [
        ("num_samples", ctypes.c_int64),
        ("eps", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("counter", ctypes.c_uint64),
        ("problem", ctypes.c_uint64),
        ("gram_precision", ctypes.c_int32),
        ("refine_max", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("stage_events", ctypes.c_void_p),
        ("augmented", ctypes.c_int32),
        ("d_eff_lower", ctypes.c_double),
        ("sampling", ctypes.c_int32),
        ("cdf_bits", ctypes.c_int32),
    ]


class TkBatchConfig(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]


MAX_BATCH = 64

_P = ctypes.POINTER
_vp = ctypes.c_void_p
_SIGNATURES = {
    "tucker_abi_version": (ctypes.c_int32, []),
    "tucker_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "tucker_sample_count": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_double, ctypes.c_double]),
    "tucker_sample_count_augmented": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_double,
                                                       ctypes.c_double, ctypes.c_double]),
    "tucker_sample_augmented": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64),
                                                 _P(ctypes.c_int32), _vp, ctypes.c_int64,
                                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                 ctypes.c_double, _vp, _vp, _vp]),
    "tucker_workspace_bytes": (ctypes.c_size_t, [_P(TkProblem), _P(TkSketchOpts), ctypes.c_int32]),
    "tucker_masked_sample_bound": (ctypes.c_int32, [_P(TkProblem), ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_double, _vp, _vp,
                                                    ctypes.c_size_t, _vp]),
    "tucker_ridge_tables": (ctypes.c_int32, [_P(TkProblem), _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                             _vp]),
    "tucker_sample_ridge": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int32),
                                             _vp, _vp, ctypes.c_int64, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                             ctypes.c_double, _vp, _vp, _vp]),
    "tucker_leverage_scores": (ctypes.c_int32, [_P(TkProblem), _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                                _vp]),
    "tucker_sample": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64), _vp, ctypes.c_int64,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp,
                                       _vp]),
    "tucker_core_update_sketched": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts), _vp, _vp, _vp,
                                                     _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                                     _vp]),
    "tucker_core_update_sketched_noalloc": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts), _vp,
                                                             _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tucker_core_update_sketched_adjoint": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts), _vp,
                                                             _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                             _vp, ctypes.c_size_t, _vp]),
    "tucker_sketched_system": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts), _vp, _vp, _vp,
                                                _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "tucker_workspace_bytes_batched": (ctypes.c_size_t, [_P(TkProblem), _P(TkSketchOpts),
                                                         ctypes.c_int32, _P(TkBatchConfig)]),
    "tucker_core_update_sketched_batched": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts),
                                                             ctypes.c_int32, _P(TkBatchConfig),
                                                             _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                                             _vp]),
    "tucker_tune_batched": (ctypes.c_int32, [_P(TkProblem), _P(TkSketchOpts), ctypes.c_int32, _vp,
                                             ctypes.c_size_t, _vp, _P(TkBatchConfig),
                                             _P(ctypes.c_double), _P(ctypes.c_int32)]),
    "tucker_core_update_exact": (ctypes.c_int32, [_P(TkProblem), _vp, _vp, _vp, ctypes.c_size_t,
                                                  _vp]),
    "tucker_factor_update": (ctypes.c_int32, [_P(TkProblem), _vp, ctypes.c_int32, _vp, _vp, _vp,
                                              ctypes.c_size_t, _vp]),
    "tucker_loss": (ctypes.c_int32, [_P(TkProblem), _vp, _vp, _vp, ctypes.c_size_t, _vp]),
}

_lib = None


def load():
    """Load libtucker_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2107_10654_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    """Names of the C-ABI functions this binding expects the library to export."""
    return sorted(_SIGNATURES)
