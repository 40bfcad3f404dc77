"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Bars (written per test):
* integer work (CDF tables, sample indices) and the sample weights: bit-exact;
* FP64 mode: element-wise error of the core, max|G - G_ref| / max|G_ref|, <= 1e-10 (solutions of the same
  sketched system computed in a different order; the system's condition
  number here is < 1e3, so 1e-10 leaves ample room above rounding);
* FP32 / BF16 Gram with FP64 refinement: element-wise error <= 1e-9 after the
  refinement reports convergence to 1e-13.
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


def T(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def tables_of(factors):
    return [oracle.cdf_table(oracle.leverage_scores(A)) for A in factors]


def elem_err(a, b):
    """Element-wise error bound: max_i |a_i - b_i| / max_i |b_i| (every entry of a
    lies within this fraction of the reference's largest entry)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SHAPES = [
    ((23, 19, 17), (3, 4, 5)),        # d = 60, one ragged tile
    ((41, 37, 29), (5, 6, 7)),        # d = 210, several tiles and a ragged tail
    ((13, 11, 9, 7), (2, 3, 2, 3)),   # order 4
    ((50,), (7,)),                    # order 1
    ((30, 20), (1, 9)),               # a rank-1 mode
    ((12, 10, 11), (4, 5, 1)),        # last rank 1
]


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_leverage_scores_and_tables(tk, dims, ranks, dtype):
    F = workloads.random_factors(dims, ranks, seed=1, kind="gaussian", dtype=dtype)
    scores, cdf = tk.leverage_scores([T(A) for A in F])
    scores, cdf = scores.cpu().numpy(), cdf.cpu().numpy().view(np.uint64)
    off = 0
    for A in F:
        I = A.shape[0]
        ref = oracle.leverage_scores(A.astype(np.float64))
        np.testing.assert_allclose(scores[off:off + I], ref, rtol=1e-11, atol=1e-13)
        _, C = oracle.cdf_table(ref)
        mism = int((cdf[off:off + I] != C).sum())
        assert mism == 0, f"{mism} CDF entries differ"
        off += I


# (7000, 9): tables too long for the sampler's LDS copy (global binary searches)
@pytest.mark.parametrize("dims", [(23, 19, 17), (41, 37, 29, 5), (7, 5, 6, 4, 3, 5), (300,),
                                  (7000, 9)])
@pytest.mark.parametrize("s", [1, 17, 4099])
def test_sampler_bit_exact(tk, dims, s):
    ranks = tuple(min(3, I) for I in dims)
    F = workloads.random_factors(dims, ranks, seed=2, kind="gaussian")
    tabs = tables_of(F)
    cdf = T(np.concatenate([C for _, C in tabs]).view(np.int64))
    for seed, counter, problem in [(0, 0, 0), (12345, 7, 3), (2 ** 63 + 5, 2 ** 40, 1)]:
        idx, w = tk.sample(dims, cdf, s, seed, counter, problem)
        ridx, rw = oracle.sample(tabs, s, seed, counter, problem)
        np.testing.assert_array_equal(idx.cpu().numpy(), ridx)
        assert np.array_equal(w.cpu().numpy().view(np.uint64), rw.view(np.uint64)), "weights differ"


def _sketch_case(dims, ranks, seed, dtype="f64", missing=None, factor="gaussian"):
    p = workloads.tucker_tensor(dims, ranks, seed, dtype, factor=factor, noise=("sigma", 0.1),
                                missing=missing)
    F = [A.astype(workloads.NP_DTYPES[dtype]) for A in p["factors_true"]]
    # move away from the generating factors so the fit is not trivial
    rng = np.random.default_rng(seed + 7)
    F = [(A + 0.1 * rng.standard_normal(A.shape)).astype(A.dtype) for A in F]
    return p, F


# FP64 shapes with d >= 256 take the Gram grouped by the last mode of rank >= 2
# The right side and residual are grouped the same way (up to three modes
# before L): on MFMA when prod_{n<L-1} R_n <= 64 and R_{L-1} <= 64 (each wave
# on its own samples when that V2 has at most four 16 x 16 blocks), else on
# the vector units; with four or more modes before L they stay per sample.
GROUPED_SHAPES = [
    ((40, 36, 30), (8, 8, 8)),          # d = 512, 30 groups
    ((30, 28, 26, 9), (8, 6, 6, 1)),    # d = 288, trailing rank-1 mode, d' = 48
    ((40, 16, 8), (24, 12, 1)),         # L = 1: one mode before L, d' = 24
    ((12, 10, 10, 10), (4, 4, 4, 4)),   # three modes before L, d' = 64
    ((12, 10, 4, 5), (9, 8, 2, 4)),     # R_0 R_1 = 72 > 64: vector-unit residual
    ((8, 6, 6, 5, 6), (4, 3, 3, 2, 4)),  # four modes before L: per-sample vectors
    ((44, 20, 5), (40, 17, 2)),         # d = 1360: V2 of 3 x 2 blocks (32-sample MFMA form)
    ((40, 6, 30), (32, 2, 8)),          # two modes before L, 528 x 3 pairs: lower-triangle B_k
    ((20, 14, 10), (16, 12, 4)),        # pair form, 136 x 78 pairs: full and ragged tiles
]


@pytest.mark.parametrize("dims,ranks", SHAPES + GROUPED_SHAPES)
def test_sketched_f64_matches_oracle(tk, dims, ranks):
    p, F = _sketch_case(dims, ranks, 3)
    lam, s = 1e-3, 3001
    G, idx, w = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=11, counter=2,
                                        precision="f64", return_samples=True)
    Gr, ridx, rw, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 11, 2)
    np.testing.assert_array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10


# d = 6144, a multiple of 64 with more tiles per workgroup than stay on chip:
# the CG kernel streams its tiles from memory every iteration.  The core must
# solve its normal equations (the oracle's matrix-free residual on the same
# samples) with CG converged and no factorisation run.
def test_sketched_f64_cg_streamed_tiles(tk):
    dims, ranks = (24, 24, 30), (16, 16, 24)
    p, F = _sketch_case(dims, ranks, 8)
    lam, d = 1e-3, 16 * 16 * 24
    s = 8 * d
    print(f"[cg streamed] dims {dims} ranks {ranks} s {s}", flush=True)
    G, idx, w, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=17,
                                              counter=3, precision="f64", return_samples=True,
                                              return_info=True)
    info = info.cpu().numpy()
    assert 1 <= info[2] < 64 and info[4] == 0.0 and info[3] <= 1e-12, info
    res = oracle.normal_equation_residual(p["X"], F, lam, idx.cpu().numpy(), w.cpu().numpy(),
                                          G.cpu().numpy())
    assert res <= 1e-10, res


# tk_sketch_opts.cdf_bits: the integer sampling weights ceil(l 2^Q) with another
# Q; the draws must stay bit-exact with the oracle's tables of the same Q (and
# differ from the default Q's, so the option reaches the sampler).
@pytest.mark.parametrize("q", [12, 32])
def test_sketched_cdf_bits_matches_oracle(tk, q):
    dims, ranks = (41, 37, 29), (5, 6, 7)
    p, F = _sketch_case(dims, ranks, 3)
    lam, s = 1e-3, 3001
    G, idx, w = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=11, counter=2,
                                        precision="f64", return_samples=True, cdf_bits=q)
    Gr, ridx, rw, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 11, 2, q_bits=q)
    np.testing.assert_array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10
    _, ridx24, rw24, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 11, 2)
    assert not np.array_equal(rw24, rw)


# FP64 with d >= 1024 and s >= 8 d solves by conjugate gradients (one
# persistent launch; the Cholesky runs only when they do not converge).
# info[2] = iterations, info[4] = 0 (no factorisation ran), info[3] the
# matrix-free FP64 residual check.  Shapes: d = 1024 (16 x 16 tiles), and
# d = 1287 with a ragged last 64-block; both with the grouped Gram.
CG_SHAPES = [
    ((40, 36, 30), (16, 16, 4), 9000),
    ((30, 28, 26), (13, 11, 9), 12000),
]


@pytest.mark.parametrize("dims,ranks,s", CG_SHAPES)
def test_sketched_f64_cg_matches_oracle(tk, dims, ranks, s):
    p, F = _sketch_case(dims, ranks, 6)
    lam = 1e-3
    print(f"[cg] dims {dims} ranks {ranks} s {s}", flush=True)
    G, idx, w, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=13,
                                              counter=1, precision="f64", return_samples=True,
                                              return_info=True)
    Gr, ridx, rw, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 13, 1)
    np.testing.assert_array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(w.cpu().numpy(), rw)
    info = info.cpu().numpy()
    assert 1 <= info[2] < 64 and info[4] == 0.0, info
    assert info[3] <= 1e-12, info
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10


def test_sketched_f64_cg_falls_back_to_cholesky(tk):
    # a frozen sample set with weights over six decades and a tiny lambda: the
    # system's condition number (~1e6) keeps conjugate gradients from reaching
    # 1e-14 in their 64 iterations, so the factorisation and its solves run.
    # Bars: the Cholesky ran (positive pivot reported); the core solves its
    # normal equations (oracle FP64 residual <= 1e-9); against the oracle's
    # own Cholesky solve within 1e-6 (both carry cond * 1e-16 error).
    dims, ranks, s = (40, 36, 30), (16, 16, 4), 9000
    p, F = _sketch_case(dims, ranks, 8)
    lam = 1e-6
    rng = np.random.default_rng(21)
    idx = np.stack([rng.integers(0, I, s) for I in dims]).astype(np.int32)
    w = 10.0 ** rng.uniform(-6.0, 0.0, s) / s
    G, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, idx=T(idx),
                                      weight=T(w), precision="f64", return_info=True)
    info = info.cpu().numpy()
    assert info[2] == 64 and info[4] > 0.0, info
    G = G.cpu().numpy()
    res = oracle.normal_equation_residual(p["X"], F, lam, idx, w, G)
    assert res <= 1e-9, res
    assert elem_err(G, oracle.core_update_sketched(p["X"], F, lam, idx, w)) <= 1e-6


@pytest.mark.parametrize("precision", ["f32", "bf16"])
@pytest.mark.parametrize("dims,ranks", [((41, 37, 29), (5, 6, 7)), ((30, 28, 26), (8, 8, 4))])
def test_sketched_low_precision_refined(tk, precision, dims, ranks):
    p, F = _sketch_case(dims, ranks, 4, dtype="f32")
    lam, s = 1e-2, 20000
    X, FF = T(p["X"]), [T(A) for A in F]
    G, info = tk.core_update_sketched(X, FF, lam, s, seed=5, precision=precision,
                                      refine_max=30, refine_tol=1e-13, return_info=True)
    info = info.cpu().numpy()
    Gr, _, _, _ = oracle.fast_core_tensor_update(p["X"].astype(np.float64),
                                                 [A.astype(np.float64) for A in F], lam, s, 5, 0)
    assert info[3] <= 1e-13, info
    # the core is returned in the problem dtype (f32): compare at f32 rounding
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-6
    # the FP64 whitened solution before the cast: re-run in f64 problem dtype
    X64, F64 = T(p["X"].astype(np.float64)), [T(A.astype(np.float64)) for A in F]
    G64 = tk.core_update_sketched(X64, F64, lam, s, seed=5, precision=precision, refine_max=30,
                                  refine_tol=1e-13)
    assert elem_err(G64.cpu().numpy(), Gr) <= 1e-9


# Every rank <= RM (a power of two <= 8) with RM^N <= 64: the refinement's
# residual keeps Kronecker rows in registers (a sample shared by RM lanes,
# ranks zero-padded to RM); ragged ranks, a rank-1 mode, orders 1 to 5, and a
# sample count far below one pass of the grid.
@pytest.mark.parametrize("precision", ["bf16", "f32"])
@pytest.mark.parametrize("dims,ranks,s", [
    ((40, 36, 30), (4, 4, 4), 20000),
    ((33, 29, 27), (3, 2, 4), 20000),
    ((12, 11, 10, 9, 8), (2, 2, 2, 2, 2), 20000),
    ((60, 50), (8, 5), 20000),
    ((45, 40, 35), (2, 1, 2), 7001),
    ((70,), (8,), 5000),
    ((40, 36, 30), (4, 4, 4), 300),
])
def test_sketched_refined_register_rows(tk, precision, dims, ranks, s):
    p, F = _sketch_case(dims, ranks, 15)
    lam = 1e-2
    G, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=7, counter=1,
                                      precision=precision, refine_max=40, refine_tol=1e-13,
                                      return_info=True)
    info = info.cpu().numpy()
    Gr, _, _, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 7, 1)
    assert info[3] <= 1e-13, info
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-9


# d > 256 with a rank sum above 64: the large-d refinement kernels with their
# long prefetch (rows staged through LDS sized by the rank sum).
@pytest.mark.parametrize("precision", ["bf16", "f32"])
def test_sketched_refined_wide_rank_sum(tk, precision):
    p, F = _sketch_case((80, 70), (40, 30), 18)
    lam = 1e-2
    G, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, 6000, seed=3,
                                      precision=precision, refine_max=40, refine_tol=1e-13,
                                      return_info=True)
    info = info.cpu().numpy()
    Gr, _, _, _ = oracle.fast_core_tensor_update(p["X"], F, lam, 6000, 3, 0)
    assert info[3] <= 1e-13, info
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-9


# 256 < d <= 4096 with at most 512 outer indices, R_L <= 32 and a rank sum
# <= 64: the residual is one fused pass (FP64 MFMA in blocks of 16 outer
# indices, 1 to 8 blocks per wave, one or two 16-wide last-mode blocks).
# Shapes: (d, R_L, outer indices) = (512, 8, 64), (2880, 24, 120),
# (2048, 8, 256), (4080, 17, 240), (2688, 7, 384) order 4, (640, 32, 20)
# order 2, (378, 9, 42) masked; s = 700 leaves fewer chunks than workgroups
# and a ragged last chunk.
@pytest.mark.parametrize("precision", ["bf16", "f32"])
@pytest.mark.parametrize("dims,ranks,s,missing", [
    ((30, 28, 26), (8, 8, 8), 2000, None),
    ((40, 36, 30), (12, 10, 24), 9000, None),
    ((40, 36, 30), (16, 16, 8), 6500, None),
    ((40, 36, 30), (16, 15, 17), 12000, None),
    ((12, 11, 10, 9), (8, 8, 6, 7), 8500, None),
    ((80, 70), (20, 32), 2500, None),
    ((31, 27, 25), (6, 7, 9), 1500, 0.2),
    ((30, 28, 26), (8, 8, 8), 700, None),
])
def test_sketched_refined_fused_residual(tk, precision, dims, ranks, s, missing):
    p, F = _sketch_case(dims, ranks, 19, missing=missing)
    lam = 1e-2
    mask = T(p["mask"].view(np.int32)) if missing else None
    G, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=13, counter=4,
                                      precision=precision, refine_max=40, refine_tol=1e-13,
                                      mask=mask, return_info=True)
    info = info.cpu().numpy()
    Gr, _, _, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 13, 4, mask=p["mask"])
    assert info[3] <= 1e-13, info
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-9


def test_sketched_masked_matches_oracle(tk):
    dims, ranks = (31, 27, 25), (4, 5, 3)
    p, F = _sketch_case(dims, ranks, 6, missing=0.2)
    lam, s = 1e-3, 5000
    G, info = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, s, seed=3,
                                      mask=T(p["mask"].view(np.int32)), return_info=True)
    Gr, idx, w, _ = oracle.fast_core_tensor_update(p["X"], F, lam, s, 3, 0, mask=p["mask"])
    assert elem_err(G.cpu().numpy(), Gr) <= 1e-10
    _, obs = oracle.sampled_entries(p["X"], idx, p["mask"])
    assert int(info[1].item()) == int((~obs).sum())


def test_frozen_sample_set(tk):
    p, F = _sketch_case((20, 18, 16), (3, 3, 3), 8)
    lam = 0.05
    tabs = tables_of(F)
    idx, w = oracle.sample(tabs, 700, seed=9, counter=1)
    G = tk.core_update_sketched(T(p["X"]), [T(A) for A in F], lam, 700, idx=T(idx), weight=T(w))
    assert elem_err(G.cpu().numpy(), oracle.core_update_sketched(p["X"], F, lam, idx, w)) <= 1e-10


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_core_matches_oracle(tk, dims, ranks, dtype):
    p, F = _sketch_case(dims, ranks, 9, dtype=dtype)
    lam = 1e-3
    G = tk.core_update_exact(T(p["X"]), [T(A) for A in F], lam)
    ref = oracle.core_update_exact(p["X"].astype(np.float64), [A.astype(np.float64) for A in F],
                                   lam)
    assert elem_err(G.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_core_masked_matches_oracle(tk, dims, ranks, dtype):
    # PCG on both sides to 1e-10 (GPU) / 1e-12 (oracle) relative residual; the
    # preconditioned system is well conditioned (20 % missing), so the
    # solutions agree to ~1e-9
    p, F = _sketch_case(dims, ranks, 10, dtype=dtype, missing=0.2)
    lam = 1e-3
    G = tk.core_update_exact(T(p["X"]), [T(A) for A in F], lam, mask=T(p["mask"].view(np.int32)))
    ref = oracle.core_update_exact_masked(p["X"].astype(np.float64),
                                          [A.astype(np.float64) for A in F], lam, p["mask"])
    assert elem_err(G.cpu().numpy(), ref) <= (1e-8 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("dims,ranks,dtype", [
    ((129, 130, 37), (4, 5, 6), "f64"),   # >= 16384 rows per last-mode fibre: MFMA contraction,
    ((130, 128, 64), (6, 3, 16), "f32"),  # ragged (37) and vector-aligned (64) fibre lengths
    ((128, 129, 33), (2, 2, 33), "f64"),  # last rank above 16 (three 16-wide output blocks)
])
def test_exact_core_long_fibres_matches_oracle(tk, dims, ranks, dtype):
    p, F = _sketch_case(dims, ranks, 12, dtype=dtype)
    lam = 1e-3
    G = tk.core_update_exact(T(p["X"]), [T(A) for A in F], lam)
    ref = oracle.core_update_exact(p["X"].astype(np.float64), [A.astype(np.float64) for A in F],
                                   lam)
    assert elem_err(G.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-6)


# Last-mode contractions with J in {1, 2, 4, 8} outputs and I J <= 4096 stream
# rows with per-lane weights in registers: J = 4 over 1024 columns, J = 8 with a
# ragged last vector of columns, J = 1 with an odd number of rows.
# Rows longer than one wave's registers (I J > 4096) are split over a
# workgroup's four waves: J = 4 over 2600 columns, J = 2 over 3000 (odd rows).
@pytest.mark.parametrize("dims,ranks,dtype", [
    ((70, 65, 1024), (3, 2, 4), "f32"),
    ((90, 50, 252), (2, 3, 8), "f64"),
    ((101, 41, 100), (2, 2, 1), "f32"),
    ((4100, 2600), (3, 4), "f32"),
    ((4097, 3000), (5, 2), "f64"),
])
def test_exact_core_skinny_last_mode(tk, dims, ranks, dtype):
    p, F = _sketch_case(dims, ranks, 16, dtype=dtype)
    lam = 1e-3
    G = tk.core_update_exact(T(p["X"]), [T(A) for A in F], lam)
    ref = oracle.core_update_exact(p["X"].astype(np.float64), [A.astype(np.float64) for A in F],
                                   lam)
    assert elem_err(G.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-6)


def test_exact_core_all_observed_mask_equals_unmasked(tk):
    p, F = _sketch_case((19, 17, 15), (3, 4, 5), 11)
    X, FF = T(p["X"]), [T(A) for A in F]
    ones = workloads.pack_mask(np.ones(p["X"].shape, dtype=bool))
    Gm = tk.core_update_exact(X, FF, 1e-3, mask=T(ones.view(np.int32)))
    Gu = tk.core_update_exact(X, FF, 1e-3)
    assert elem_err(Gm.cpu().numpy(), Gu.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_factor_update_matches_oracle(tk, dims, ranks):
    p, F = _sketch_case(dims, ranks, 10)
    lam = 1e-2
    G = np.random.default_rng(1).standard_normal(ranks)
    for n in range(len(dims)):
        A = tk.factor_update(T(p["X"]), T(G), [T(B) for B in F], n, lam)
        ref = oracle.factor_update(p["X"], G, F, n, lam)
        assert elem_err(A.cpu().numpy(), ref) <= 1e-10, n


@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_loss_matches_oracle(tk, dims, ranks):
    for missing in (None, 0.3):
        p, F = _sketch_case(dims, ranks, 12, missing=missing)
        G = np.random.default_rng(2).standard_normal(ranks)
        mask = T(p["mask"].view(np.int32)) if missing else None
        Lv, sq, cnt = tk.loss(T(p["X"]), T(G), [T(A) for A in F], 0.1, mask=mask)
        rL, rrmse = oracle.loss(p["X"], G, F, 0.1, p["mask"])
        assert abs(Lv - rL) <= 1e-10 * abs(rL)
        assert abs((sq / cnt) ** 0.5 - rrmse) <= 1e-10 * rrmse


# Middle-mode contractions with many (p, q) fibres run as per-p MFMA products
# (a wave per 64 q, J in blocks of 16): ragged q tails, a partial i chunk and
# J = 4, 20 and 64 (one, two and four j blocks).  The rank-64 mode's own update
# is left out: its system has condition number ~3e8 (rank 6 core unfolding).
@pytest.mark.parametrize("dims,ranks,dtype,modes", [
    ((520, 9, 70), (3, 4, 5), "f64", (0, 1, 2)),
    ((530, 33, 66), (4, 20, 6), "f32", (0, 1, 2)),
    ((520, 70, 64), (2, 64, 3), "f64", (0, 2)),
])
def test_factor_update_mid_mode_contraction(tk, dims, ranks, dtype, modes):
    p, F = _sketch_case(dims, ranks, 13, dtype=dtype)
    lam = 1e-2
    G = np.random.default_rng(3).standard_normal(ranks)
    Xf = p["X"].astype(np.float64)
    Ff = [A.astype(np.float64) for A in F]
    for n in modes:
        A = tk.factor_update(T(p["X"]), T(G.astype(p["X"].dtype)), [T(B) for B in F], n, lam)
        Gr = G.astype(p["X"].dtype).astype(np.float64)
        ref = oracle.factor_update(Xf, Gr, Ff, n, lam)
        assert elem_err(A.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-5), n


# Middle-mode contractions with J in {1, 2, 4, 8} and long q runs stream along
# q without padding J: J = 4 (f32), J = 8 and J = 2 (f64, ragged q runs).
@pytest.mark.parametrize("dims,ranks,dtype", [
    ((300, 20, 512), (2, 4, 3), "f32"),
    ((280, 9, 260), (3, 8, 2), "f64"),
    ((270, 13, 258), (2, 2, 3), "f64"),
])
def test_factor_update_mid_mode_skinny(tk, dims, ranks, dtype):
    p, F = _sketch_case(dims, ranks, 17, dtype=dtype)
    lam = 1e-2
    G = np.random.default_rng(5).standard_normal(ranks)
    Xf = p["X"].astype(np.float64)
    Ff = [A.astype(np.float64) for A in F]
    Gt = G.astype(p["X"].dtype)
    A = tk.factor_update(T(p["X"]), T(Gt), [T(B) for B in F], 2, lam)
    ref = oracle.factor_update(Xf, Gt.astype(np.float64), Ff, 2, lam)
    assert elem_err(A.cpu().numpy(), ref) <= (1e-10 if dtype == "f64" else 1e-5)


# The loss expands the last mode on MFMA in k-steps of 4 ranks (1, 2, 4, 8 or 16
# steps) with A_N staged in LDS in column chunks: R_N = 20 and 33 give 8 and 16
# steps, the latter with eleven 64-column chunks; ragged last chunks.
@pytest.mark.parametrize("dims,ranks", [
    ((50, 37, 300), (2, 3, 20)),
    ((40, 30, 700), (3, 4, 33)),
    ((33, 1029), (5, 4)),
])
def test_loss_wide_last_mode(tk, dims, ranks):
    for missing in (None, 0.25):
        p, F = _sketch_case(dims, ranks, 14, missing=missing)
        G = np.random.default_rng(4).standard_normal(ranks)
        mask = T(p["mask"].view(np.int32)) if missing else None
        Lv, sq, cnt = tk.loss(T(p["X"]), T(G), [T(A) for A in F], 0.1, mask=mask)
        rL, rrmse = oracle.loss(p["X"], G, F, 0.1, p["mask"])
        assert abs(Lv - rL) <= 1e-10 * abs(rL)
        assert abs((sq / cnt) ** 0.5 - rrmse) <= 1e-10 * rrmse


def test_als_c1_exact_and_sketched(tk):
    """C1 workload: 5 ALS iterations, exact and sketched cores, from the same U[0,1) start."""
    prob = workloads.config_problem("c1")
    cfg = prob["cfg"]
    X = prob["X"]
    G0, F0 = workloads.als_init(cfg["dims"], cfg["ranks"], 1000)
    for core in ("exact", "sketched"):
        Gg, Fg, hg = tk.als(T(X), T(G0), [T(A) for A in F0], cfg["lam"], cfg["als_iters"],
                            core=core, samples=cfg["samples"], seed=0)
        Gr, Fr, hr = oracle.als(X, G0, F0, cfg["lam"], cfg["als_iters"], core=core,
                                s=cfg["samples"], seed=0)
        for (a, ra), (b, rb) in zip(hg, hr):
            assert abs(a - b) <= 1e-6 * abs(b), (core, hg, hr)
        assert elem_err(Gg.cpu().numpy(), Gr) <= 1e-6


def test_status_errors(tk):
    from paper_2107_10654_amd import TuckerError
    rng = np.random.default_rng(0)
    A = rng.standard_normal((20, 4))
    A[:, 3] = A[:, 0]
    F = [T(A), T(rng.standard_normal((15, 3)))]
    with pytest.raises(TuckerError, match="RANK_DEFICIENT"):
        tk.leverage_scores(F)
    X = T(rng.standard_normal((20, 15)))
    good = [T(rng.standard_normal((20, 4))), F[1]]
    idx = T(np.array([[0, 25], [1, 2]], dtype=np.int32))  # 25 is out of range
    w = T(np.array([1.0, 1.0]))
    with pytest.raises(TuckerError, match="E_ARG"):
        tk.core_update_sketched(X, good, 0.1, 2, idx=idx, weight=w)
    # a following good call clears the status word
    tk.core_update_sketched(X, good, 0.1, 64)


# A tiny trailing mode (the video-shaped case): the exact update contracts the
# longest mode first, and a product whose fibres hold at most 4 trailing entries
# reads X as long rows against M (x) I_Q.  f32 data: bars 1e-5 element-wise.
def test_exact_and_factor_update_tiny_last_mode(tk):
    dims, ranks = (20, 850, 1000, 3), (2, 3, 4, 2)
    p = workloads.tucker_tensor(dims, ranks, 61, "f32", factor="gaussian", noise=("sigma", 0.1))
    F = [A.astype(np.float32) for A in p["factors_true"]]
    X, FF = T(p["X"]), [T(A) for A in F]
    X64, F64 = p["X"].astype(np.float64), [A.astype(np.float64) for A in F]
    lam = 1e-2
    G = tk.core_update_exact(X, FF, lam)
    ref = oracle.core_update_exact(X64, F64, lam)
    assert elem_err(G.cpu().numpy(), ref) <= 1e-5
    Gc = np.random.default_rng(62).standard_normal(ranks).astype(np.float32)
    for n in range(4):
        A = tk.factor_update(X, T(Gc), FF, n, lam)
        ref = oracle.factor_update(X64, Gc.astype(np.float64), F64, n, lam)
        assert elem_err(A.cpu().numpy(), ref) <= 1e-5, n
