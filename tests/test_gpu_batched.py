"""Batched sampled core updates (one persistent stream-K Gram launch for all
problems), the tuner and HIP-graph capture.

Bars (written per test):
* every problem of a batch equals the single-problem call on the same samples
  (problem field k): both are refined in FP64 to 1e-13 of the right side, so
  FP64 outputs agree to 1e-10 and f32 outputs to 1e-5;
* against the FP64 oracle on the same samples: 1e-9 (FP64 outputs);
* tiles 64, 128 and 256 give the same solution (1e-10);
* graph replays are bit-identical to the eager batched call, with eager work
  and synchronisation between the replays.
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


def _small_batch(dtype="f64", count=10):
    probs = workloads.batch_problems(seed=31, count=count, side=(12, 48), rank=(2, 6),
                                     dtype=dtype)
    Xs = [T(p["X"]) for p in probs]
    Fs = [[T(np.ascontiguousarray(A.astype(p["X"].dtype))) for A in p["factors_true"]]
          for p in probs]
    return probs, Xs, Fs


@pytest.mark.parametrize("config", [None, {"tile": 64, "wg_per_cu": 4},
                                    {"tile": 128, "wg_per_cu": 2}, {"tile": 256, "wg_per_cu": 1}])
def test_batched_equals_single_calls_and_oracle(tk, config):
    probs, Xs, Fs = _small_batch()
    lam = 1e-3
    ss = [p["samples"] for p in probs]
    cores, info = tk.core_update_sketched_batched(Xs, Fs, lam, ss, seeds=9, counters=2,
                                                  precision="bf16", config=config,
                                                  refine_max=30, return_info=True)
    info = info.cpu().numpy()
    for k, p in enumerate(probs):
        assert info[k, 3] <= 1e-13, (k, info[k])
        G1 = tk.core_update_sketched(Xs[k], Fs[k], lam, ss[k], seed=9, counter=2, problem=k,
                                     precision="bf16", refine_max=30)
        assert elem_err(cores[k].cpu().numpy(), G1.cpu().numpy()) <= 1e-10, k
        Gr, _, _, _ = oracle.fast_core_tensor_update(p["X"], p["factors_true"], lam, ss[k], 9, 2,
                                                     problem=k)
        assert elem_err(cores[k].cpu().numpy(), Gr) <= 1e-9, k


def test_batched_f32_precision_and_f32_problems(tk):
    probs, Xs, Fs = _small_batch(dtype="f32", count=7)
    lam = 1e-2
    ss = [p["samples"] for p in probs]
    cores = tk.core_update_sketched_batched(Xs, Fs, lam, ss, seeds=4, precision="f32")
    for k in range(len(probs)):
        G1 = tk.core_update_sketched(Xs[k], Fs[k], lam, ss[k], seed=4, problem=k,
                                     precision="f32")
        assert elem_err(cores[k].cpu().numpy(), G1.cpu().numpy()) <= 1e-5, k


def test_tuner_returns_a_candidate(tk):
    probs, Xs, Fs = _small_batch(count=6)
    best, times = tk.tune_batched(Xs, Fs, 1e-3, [p["samples"] for p in probs], seeds=1)
    assert best["tile"] in (64, 128, 256) and 1 <= best["wg_per_cu"] <= 8
    assert len(times) == 6 and all(t > 0 for t in times)


def test_graph_replays_match_eager(tk):
    probs, Xs, Fs = _small_batch(count=8)
    lam = 1e-3
    ss = [p["samples"] for p in probs]
    eager = [c.clone() for c in tk.core_update_sketched_batched(Xs, Fs, lam, ss, seeds=5,
                                                                precision="bf16")]
    upd = tk.BatchedSketchedUpdate(Xs, Fs, lam, ss, seeds=5, precision="bf16")
    for rep in range(3):
        # eager work of the program between replays
        tk.core_update_sketched(Xs[0], Fs[0], lam, ss[0], seed=77, precision="bf16")
        torch.cuda.synchronize()
        for c in upd.cores:
            c.zero_()
        out = upd.replay()
        torch.cuda.synchronize()
        for k in range(len(probs)):
            assert torch.equal(out[k], eager[k]), (rep, k)
        assert int(upd.status.abs().sum().item()) == 0
        # the captured call writes its info rows: sample count, refinement residual
        info = upd.info.cpu().numpy()
        assert np.array_equal(info[:, 0], [float(p["samples"]) for p in probs]), info[:, 0]
        assert (info[:, 3] <= 1e-13).all(), info[:, 3]


def test_graph_replay_reads_new_inputs(tk):
    probs, Xs, Fs = _small_batch(count=4)
    lam = 1e-3
    ss = [p["samples"] for p in probs]
    upd = tk.BatchedSketchedUpdate(Xs, Fs, lam, ss, seeds=6, precision="bf16")
    before = [c.clone() for c in upd.replay()]
    torch.cuda.synchronize()
    Xs[2].mul_(2.0)  # the core is linear in X
    after = upd.replay()
    torch.cuda.synchronize()
    assert elem_err(after[2].cpu().numpy(), 2.0 * before[2].cpu().numpy()) <= 1e-10
    assert torch.equal(after[1], before[1])


# ---------------------------------------------------------------- the 64-problem batch
@pytest.fixture(scope="module")
def c4(tk):
    probs = workloads.batch_problems(seed=4, count=64)
    Xs = [T(p["X"]) for p in probs]
    Fs = [[T(np.ascontiguousarray(A.astype(np.float32))) for A in p["factors_true"]]
          for p in probs]
    return probs, Xs, Fs


def test_c4_batch_matches_single_calls(tk, c4):
    probs, Xs, Fs = c4
    lam = 1e-3
    ss = [p["samples"] for p in probs]
    best, _ = tk.tune_batched(Xs, Fs, lam, ss, seeds=4)
    cores, info = tk.core_update_sketched_batched(Xs, Fs, lam, ss, seeds=4, precision="bf16",
                                                  config=best, return_info=True)
    info = info.cpu().numpy()
    assert (info[:, 3] <= 1e-13).all(), info[:, 3].max()
    order = np.argsort([int(p["G_true"].size) for p in probs])
    for k in list(order[:4]) + list(order[-2:]):  # smallest and largest cores
        G1, idx1, w1 = tk.core_update_sketched(Xs[k], Fs[k], lam, ss[k], seed=4, problem=int(k),
                                               precision="bf16", return_samples=True)
        assert elem_err(cores[k].cpu().numpy(), G1.cpu().numpy()) <= 1e-5, k
        if k in order[-2:]:
            # the largest problems against the oracle: the batch draws the single
            # call's samples (bit-exact with the oracle's sampler), and the batched
            # core solves the sketched normal equations of those samples to the
            # f32 output's rounding (oracle FP64 residual)
            p = probs[k]
            F64 = [A.astype(np.float32).astype(np.float64) for A in p["factors_true"]]
            tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F64]
            ridx, rw = oracle.sample(tables, ss[k], 4, 0, problem=int(k))
            assert np.array_equal(idx1.cpu().numpy(), ridx), k
            assert np.array_equal(w1.cpu().numpy(), rw), k
            res = oracle.normal_equation_residual(p["X"].astype(np.float64), F64, lam, ridx, rw,
                                                  cores[k].cpu().numpy())
            assert res <= 1e-6, (k, res)
    for k in order[:3]:  # the oracle solves the small ones end to end
        p = probs[k]
        Gr, _, _, _ = oracle.fast_core_tensor_update(
            p["X"].astype(np.float64), [A.astype(np.float32).astype(np.float64)
                                        for A in p["factors_true"]], lam, ss[k], 4, 0,
            problem=int(k))
        assert elem_err(cores[k].cpu().numpy(), Gr) <= 1e-5, k
