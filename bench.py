#!/usr/bin/env python3
"""Sampled Tucker core updates per second on one MI355X (gfx950).

Workload (default ``c2``): 512 x 512 x 512 float32 tensor, Tucker rank
16 x 16 x 16 (core dimension d = 4096), Gaussian-then-QR factors, noise at
20 dB SNR, lambda = 1e-2, 131072 leverage samples per core update, seed 2.

One step = one sampled core update, every step of the hot path: factor
leverage scores and integer CDFs, product-distribution sampling, gather of the
sampled entries, the sketched Gram plus lambda P and the FP64 right side, the
solve and its FP64 residual check, and the map back from whitened
coordinates.  The default precision is FP64: the Gram grouped by the last
mode's sample index on FP64 MFMA, solved by conjugate gradients (Cholesky as
fallback).  --precision bf16 / f32 times the stream-K Gram on MFMA with FP32
accumulation, FP64 Cholesky and FP64 refinement.  Inputs are resident in HBM
before the timed region.  Beside the headline number the
script times the exact core update and one ALS iteration (exact factor
updates plus either core update) on the same data, and the loss each core
update reaches.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}
WORKLOADS = {
    "c2": "512x512x512 f32 Tucker tensor, rank 16x16x16 (d=4096), Gaussian-then-QR factors, "
          "20 dB SNR noise, lambda=1e-2, 131072 samples per core update",
    "c5": "256x256x256 f32 Tucker tensor, rank 12x12x12 (d=1728), lambda=1e-2, 32768 samples",
    "c1": "64x64x64 f64 Tucker tensor, rank 4x4x4 (d=64), lambda=1e-3, 2048 samples",
    "c3": "128x128x128x128 f32 Tucker tensor, rank 8x8x8x8 (d=4096), 10% entries missing, "
          "lambda=1e-3, 65536 samples per core update",
    "t1big": "2560x2560x2560 f32 tensor (67 GB, generated on the GPU) of the Sec. 5 synthetic "
             "protocol, fitted at rank 4x4x4 (d=64) from a U[0,1] initial state, lambda=1e-3, "
             "1687583 samples (Alg. 1 count, eps=delta=0.1)",
    "t1": "1024x1024x1024 f32 tensor of the Sec. 5 synthetic protocol (true core 8x8x8, U[0,1] "
          "core and factors, N(0,1) noise on 1% of entries), fitted at rank 4x4x4 (d=64) from a "
          "U[0,1] initial state, lambda=1e-3, 1687583 samples (Alg. 1 count, eps=delta=0.1)",
    "c4": "batch of 64 order-3 f32 Tucker tensors, sides U{32..384}, ranks U{4..24}, 1% noise, "
          "lambda=1e-3, 16*prod(ranks) samples each; one persistent batched Gram launch, "
          "autotuned tiles, replayed as a HIP graph",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime that torch already loaded."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            if self.lib.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            arr[i] = h
        return arr

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.lib.hipEventElapsedTime(ctypes.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def destroy(self, arr):
        for h in arr:
            self.lib.hipEventDestroy(h)


GRAM_SOURCES = {"bf16": ("tk_gram_sk.hip", "tk_mfma.h", "tk_internal.h"),
                "f32": ("tk_gram_sk.hip", "tk_mfma.h", "tk_internal.h"),
                "f64": ("tk_gram_grouped.hip", "tk_mfma.h", "tk_internal.h")}


def kernel_source_hash(prec):
    """Hash of the sources the Gram kernels of precision prec are built from."""
    h = hashlib.sha256()
    for name in GRAM_SOURCES[prec]:
        with open(os.path.join(ROOT, "paper_2107_10654_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def grouped_gram_on(d, s, RL, IL):
    """Whether the library takes the FP64 Gram grouped by the last mode (its
    plan: d >= 256, R_L >= 2, and clearly fewer multiply-adds than per sample)."""
    if d < 256 or RL < 2:
        return False
    dp = d // RL
    pt = -(-dp // 64)
    tiles = pt * (pt + 1) // 2 * 4096.0
    return 3.0 * tiles * (s + IL * RL * RL) <= s * d * d * 0.5


def read_traffic(kernel, workload, prec):
    """HBM bytes per launch from profiles/traffic.txt, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash(prec)
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 5 and not line.startswith("#") and parts[0] == kernel \
                    and parts[1] == workload and parts[2] == src:
                return int(parts[3]) + int(parts[4])
    return None


def host_cpu():
    """CPU model and logical CPU count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    return model, os.cpu_count()


def cpu_baseline(prob, F, lam, s, s_cpu, seed, mask=None):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    Returns the baseline record and, when the sample is the whole workload
    (s_cpu == s), the oracle's core for counter 0, else None."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    model, ncpu = host_cpu()
    X = prob["X"]
    F = [np.asarray(A, dtype=np.float64) for A in F]
    t0 = time.perf_counter()
    tables = [oracle.cdf_table(oracle.leverage_scores(A)) for A in F]
    t1 = time.perf_counter()
    idx, w = oracle.sample(tables, s_cpu, seed, 0)
    t2 = time.perf_counter()
    gram, rhs = oracle.sketched_normal_equations(X, F, idx, w, mask)
    t3 = time.perf_counter()
    d = gram.shape[0]
    Lc = np.linalg.cholesky(gram + lam * np.eye(d))
    g = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rhs))
    t4 = time.perf_counter()
    scale = s / s_cpu
    t_full = (t1 - t0) + (t2 - t1 + t3 - t2) * scale + (t4 - t3)
    omp = os.environ.get("OMP_NUM_THREADS")
    rec = {
        "value": 1.0 / t_full, "unit": "updates/s", "cores": int(cores), "kind": "oracle",
        "host_cpus": ncpu, "cpu_model": model,
        "threads_note": (f"BLAS threads = {cores} (OMP_NUM_THREADS={omp} on this host; "
                         f"{ncpu} logical CPUs visible)"),
        "sample": (f"FP64 NumPy oracle sketched update with {s_cpu} of the {s} samples: sampling and "
                   f"Gram/right side timed on {s_cpu} samples and scaled linearly to {s}; leverage "
                   f"scores and the d={d} Cholesky solve timed in full; measured "
                   f"{t4 - t0:.1f} s of CPU work, extrapolated update time {t_full:.1f} s"),
    }
    return rec, (g if s_cpu == s else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f64", choices=["bf16", "f32", "f64"])
    ap.add_argument("--refine-max", type=int, default=8)
    ap.add_argument("--cpu-samples", type=int, default=131072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip exact/ALS comparison timings")
    ap.add_argument("--protocol", choices=["table1", "movie"], default=None,
                    help="run the paper's ALS vs ALS-RS comparison instead of the headline "
                         "benchmark (one JSON line per point)")
    ap.add_argument("--dims", default=None, help="tensor shape of --protocol table1, e.g. 512,512,512")
    ap.add_argument("--microbench", action="store_true",
                    help="time the sampling and gather steps at Alg. 1's count and the sampler "
                         "alone at 2^24 samples (one JSON line)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain FP32 copy kernel over this many MiB (calibrates the "
                         "HBM byte counters of a profiler run)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampled update's multi-GPU split is a design note, not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2107_10654_amd as tk
    import workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.protocol:
        return bench_protocol(args, tk, workloads, np, torch, dev)
    if args.microbench:
        return bench_microbench(args, tk, workloads, np, torch, dev)
    if args.workload == "c4":
        return bench_batch(args, tk, workloads, np, torch, dev)

    t_gen = time.perf_counter()
    prob = workloads.config_problem(args.workload)
    cfg = prob["cfg"]
    lam, s = cfg["lam"], cfg["samples"]
    np_dt = workloads.NP_DTYPES[cfg["dtype"]]
    on_device = torch.is_tensor(prob["X"])  # generated on the GPU (no host copy)
    X = prob["X"] if on_device else torch.from_numpy(prob["X"]).to(dev)
    F_host = prob.get("factors_fit", prob["factors_true"])
    F = [torch.from_numpy(np.ascontiguousarray(A.astype(np_dt))).to(dev) for A in F_host]
    mask = (torch.from_numpy(prob["mask"].view(np.int32)).to(dev)
            if prob.get("mask") is not None else None)
    torch.cuda.synchronize()
    log(f"[bench] workload {args.workload}: X {tuple(X.shape)} {X.dtype}, d={int(np.prod(cfg['ranks']))}, "
        f"s={s}, generated in {time.perf_counter() - t_gen:.1f} s")
    d = int(np.prod(cfg["ranks"]))

    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: 3 launches reading and writing {nbytes} bytes each")

    hip = HipEvents()
    nst = tk.tucker.L.NUM_STAGE_EVENTS

    def run(k, events=None, check=False, info=False, status=None):
        return tk.core_update_sketched(X, F, lam, s, seed=cfg["seed"], counter=k, mask=mask,
                                       precision=args.precision, refine_max=args.refine_max,
                                       refine_tol=1e-13, check=check, return_info=info,
                                       stage_events=ctypes.addressof(events) if events else None,
                                       status=status)

    # warmup (first call checked); the counter-0 core is compared with the oracle's
    G, info = run(0, check=True, info=True)
    G0 = G.detach().clone()
    for k in range(1, args.warmup):
        run(k)
    torch.cuda.synchronize()
    log(f"[bench] warmup done; refinement steps {info[2].item():.0f}, rel. residual {info[3].item():.2e}")

    ev = [hip.create(nst) for _ in range(args.steps)]
    # one status word per timed step: a data-dependent failure in any of them
    # (not positive definite, refinement not converged, a bounded wait that
    # ran out) is caught after the timed region
    st_words = torch.zeros(args.steps, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        G = run(1000 + k, events=ev[k], status=st_words[k:k + 1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = st_words.cpu().numpy()
    if bad.any():
        log(f"[bench] timed steps reported status words {bad.tolist()}; no result")
        sys.exit(3)
    stage_names = ["leverage", "sample", "gather", "gram", "assemble_rhs", "cholesky", "solve",
                   "refine", "finish"]
    stage_ms = {n: 0.0 for n in stage_names}
    for k in range(args.steps):
        for j, n in enumerate(stage_names):
            stage_ms[n] += hip.elapsed_ms(ev[k][j], ev[k][j + 1]) / args.steps
    for e in ev:
        hip.destroy(e)
    ms = wall * 1e3 / args.steps
    log(f"[bench] {args.steps} sketched updates: {ms:.3f} ms each; stages (ms): "
        + ", ".join(f"{n} {v:.3f}" for n, v in stage_ms.items()))

    # rooflines of the Gram stage and of the solve; the larger stage is "roofline"
    gram_ms = stage_ms["gram"]
    ranks = list(cfg["ranks"])
    dims = list(cfg["dims"])
    L = max(n for n in range(len(ranks)) if ranks[n] >= 2)
    grouped = args.precision == "f64" and grouped_gram_on(d, s, ranks[L], dims[L])
    if grouped:
        # lower triangle: each sample adds d'(d'+1)/2 products to its group's
        # B_k, each group adds d(d+1)/2 to M (one multiply-add = 2 flops)
        dp = d // ranks[L]
        flops = float(s) * dp * (dp + 1) + float(dims[L]) * d * (d + 1)
        kern = ("grouped FP64 Gram (grp_block_split_kernel, in its pair form when two modes "
                "precede the grouping mode, or grp_block_kernel beyond three, and "
                "grp_expand_kernel on FP64 MFMA, with the sort and sorted-row kernels; time of "
                "the Gram stage; flops counted as the algorithm's, not as executed)")
    else:
        flops = float(s) * d * (d + 1)
        kern = (f"gram_sk_kernel (stream-K Gram, {args.precision} operands, fp32 "
                "accumulation; time of the Gram stage, with its slot-index kernel)")
    achieved = flops / (gram_ms * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    traffic = read_traffic(f"gram_{args.precision}", args.workload, args.precision)
    gram_roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                 "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kern,
                 "algorithmic_flops": flops, "kernel_ms": round(gram_ms, 4)}
    solve_roof = None
    cg_iters = int(info[2].item()) if args.precision == "f64" and info[4].item() == 0.0 else 0
    if cg_iters > 0:
        # conjugate gradients: one product with the symmetric M per iteration
        # plus the start, 2 d^2 flops each, on the FP64 vector units
        solve_ms = stage_ms["solve"]
        sflops = 2.0 * d * d * (cg_iters + 1)
        sach = sflops / (solve_ms * 1e-3) / 1e12
        solve_roof = {"bound": "alu", "achieved": round(sach, 3), "peak": PEAKS_TFLOPS["f64"],
                      "unit": "TFLOP/s", "frac": round(sach / PEAKS_TFLOPS["f64"], 4),
                      "traffic": None,
                      "kernel": f"cg_kernel (persistent conjugate gradients, {cg_iters} "
                                "iterations, partials and shares polled between workgroups; "
                                "time of the solve stage)",
                      "algorithmic_flops": sflops, "kernel_ms": round(solve_ms, 4)}
    if solve_roof is not None and stage_ms["solve"] > gram_ms:
        roofline, other = solve_roof, gram_roof
    else:
        roofline, other = gram_roof, solve_roof

    extras = {}
    if not args.no_extras:
        _, info = run(7, check=True, info=True)
        G_s = run(7)
        torch.cuda.synchronize()
        # exact core update on the same factors
        G_e = tk.core_update_exact(X, F, lam, mask=mask)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            tk.core_update_exact(X, F, lam, mask=mask, check=False)
        e1.record()
        torch.cuda.synchronize()
        exact_ms = e0.elapsed_time(e1) / reps
        L_e = tk.loss(X, G_e, F, lam, mask=mask)
        L_s = tk.loss(X, G_s, F, lam, mask=mask)
        # one ALS iteration: N factor updates + core update
        def als_iter(core):
            Fi = list(F)
            Gi = G_e
            for n in range(len(Fi)):
                Fi[n] = tk.factor_update(X, Gi, Fi, n, lam, check=False, mask=mask)
            if core == "exact":
                return tk.core_update_exact(X, Fi, lam, check=False, mask=mask)
            return tk.core_update_sketched(X, Fi, lam, s, seed=cfg["seed"], counter=99,
                                           precision=args.precision, refine_max=args.refine_max,
                                           refine_tol=1e-13, check=False, mask=mask)
        als_ms = {}
        # with a mask every update (factors and core) fits the observed entries only
        for core in ("exact", "sketched"):
            als_iter(core)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(3):
                als_iter(core)
            e1.record()
            torch.cuda.synchronize()
            als_ms[core] = e0.elapsed_time(e1) / 3
        bound = None
        if mask is not None:
            # Cor. B.1: the count Alg. 1 would need for the masked design at
            # eps = delta = 0.1 (reported beside the configured s)
            ib, prod, beta_p, s_b = tk.masked_sample_bound(F, lam, 0.1, 0.1)
            bound = {"inv_beta_bound": ib, "beta_prime": beta_p, "samples_for_guarantee": s_b,
                     "samples_used": s}
        extras = {
            "masked_sample_bound": bound,
            "sketched_update_ms": round(ms, 4),
            "exact_update_ms": round(exact_ms, 4),
            "exact_over_sketched_speed": round(exact_ms / ms, 4),
            "als_iteration_ms": {k: round(v, 4) for k, v in als_ms.items()},
            "loss_after_exact_core": L_e[0],
            "loss_after_sketched_core": L_s[0],
            "loss_rel_gap": (L_s[0] - L_e[0]) / L_e[0],
            "rmse_exact": (L_e[1] / L_e[2]) ** 0.5,
            "rmse_sketched": (L_s[1] / L_s[2]) ** 0.5,
            "refine_steps": int(info[2].item()),
            "refine_rel_residual": float(info[3].item()),
            "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        }
        log(f"[bench] exact update {exact_ms:.3f} ms; ALS iteration {als_ms}; "
            f"loss exact {L_e[0]:.6e} sketched {L_s[0]:.6e}")

    cpu = None
    oracle_err = None
    if not args.no_cpu_baseline and not on_device:
        log(f"[bench] CPU oracle baseline on {args.cpu_samples} samples ...")
        cpu, g_ref = cpu_baseline(prob, [A.astype(np_dt) for A in F_host], lam, s,
                                  min(args.cpu_samples, s), cfg["seed"], prob.get("mask"))
        log(f"[bench] CPU oracle: {cpu['value']:.4g} updates/s on {cpu['cores']} threads")
        if g_ref is not None:
            # the GPU's counter-0 core against the oracle's solve of the same
            # samples (FP64): max |G - G_ref| / max |G_ref| and the 2-norm ratio
            a = G0.double().cpu().numpy().ravel()
            oracle_err = {
                "elementwise": float(np.max(np.abs(a - g_ref)) / np.max(np.abs(g_ref))),
                "norm": float(np.linalg.norm(a - g_ref) / np.linalg.norm(g_ref)),
                "what": "core of the counter-0 update vs the FP64 oracle's Cholesky solve of the "
                        "same sketched system (same seed and samples); the GPU core is returned "
                        f"in {cfg['dtype']}",
            }
            log(f"[bench] error vs FP64 oracle: element-wise {oracle_err['elementwise']:.3e}")

    out = {
        "metric": "sketched core updates/sec and ALS iteration time vs exact update at equal loss",
        "value": args.steps / wall,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload,
                   "gram_operands": args.precision, "gram_accumulate": "f32" if args.precision != "f64" else "f64",
                   "gram": "grouped by the last mode" if grouped else "per sample",
                   "solve": ("f64 Cholesky + f64 refinement" if args.precision != "f64" else
                             f"f64 conjugate gradients ({cg_iters} iterations)" if cg_iters else
                             "f64 Cholesky"),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_other_stage": other,
        "cpu_baseline": cpu,
        "oracle_rel_err": oracle_err,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def bench_protocol(args, tk, workloads, np, torch, dev):
    """The paper's ALS vs ALS-RS comparisons (Sec. 5), one JSON line per point.

    table1: the synthetic protocol (true core 8^3, U[0,1] core and factors,
    N(0,1) noise on 1 % of entries) at --dims (default 1024^3), fitted at ranks
    (2,2,2), (4,2,2), (4,4,2), (4,4,4) for 10 iterations from the same U[0,1)
    initial state; the sampled core uses s = 32 d and Alg. 1's count
    (eps = delta = 0.1).  movie: the (100, 1080, 1920, 3) stand-in, core
    (2, 4, 4, 2), 5 iterations.  Every step is timed with device events and the
    RMSE is taken after each iteration.
    """
    lam = 1e-3
    t_gen = time.perf_counter()
    if args.protocol == "table1":
        dims = tuple(int(v) for v in args.dims.split(",")) if args.dims else (1024, 1024, 1024)
        X = workloads.table1_problem_device(dims, 11, dev)["X"]
        rank_list = [(2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4)]
        iters, init_seed = 10, 1011
    else:
        dims = (100, 1080, 1920, 3)
        X = workloads.movie_problem_device(21, dev)
        rank_list = [(2, 4, 4, 2)]
        iters, init_seed = 5, 1021
    torch.cuda.synchronize()
    log(f"[bench] protocol {args.protocol}: X {dims} generated in {time.perf_counter() - t_gen:.1f} s")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    def run_als(ranks, core, s):
        G0, F0 = workloads.als_init(dims, ranks, init_seed, "f32")
        G = torch.from_numpy(np.ascontiguousarray(G0)).to(dev)
        F = [torch.from_numpy(np.ascontiguousarray(A)).to(dev) for A in F0]
        hist = []
        for it in range(iters):
            fms = []
            for n in range(len(F)):
                F[n], ms_f = timed(lambda: tk.factor_update(X, G, F, n, lam, check=False))
                fms.append(ms_f)
            if core == "exact":
                G, ms_c = timed(lambda: tk.core_update_exact(X, F, lam, check=False))
            else:
                G, ms_c = timed(lambda: tk.core_update_sketched(
                    X, F, lam, s, seed=7, counter=it, precision="bf16", refine_max=8,
                    refine_tol=1e-13, check=False))
            Lv, sq, cnt = tk.loss(X, G, F, lam)
            hist.append({"iter": it + 1, "factor_ms": [round(v, 4) for v in fms],
                         "core_ms": round(ms_c, 4), "rmse": (sq / cnt) ** 0.5, "loss": Lv})
        return hist

    for ranks in rank_list:
        d = int(np.prod(ranks))
        exact = run_als(ranks, "exact", None)
        for s_mode in ("32d", "theory"):
            s = 32 * d if s_mode == "32d" else tk.sample_count(d, 0.1, 0.1)
            sk = run_als(ranks, "sketched", s)

            def mean(h, key, skip=1):  # the first iteration includes warm-up
                vals = [r[key] for r in h[skip:]]
                return sum(vals) / len(vals)

            out = {
                "metric": "sketched core updates/sec and ALS iteration time vs exact update at "
                          "equal loss",
                "protocol": args.protocol,
                "dims": list(dims), "ranks": list(ranks), "lambda": lam, "samples": s,
                "samples_rule": "32 d" if s_mode == "32d" else "Alg. 1 count, eps = delta = 0.1",
                "iterations": iters,
                "mean_core_ms": {"exact": round(mean(exact, "core_ms"), 4),
                                 "sketched": round(mean(sk, "core_ms"), 4)},
                "mean_factor_ms": [round(sum(r["factor_ms"][n] for r in exact[1:]) /
                                         (iters - 1), 4) for n in range(len(dims))],
                "core_speedup": round(mean(exact, "core_ms") / mean(sk, "core_ms"), 3),
                "final_rmse": {"exact": exact[-1]["rmse"], "sketched": sk[-1]["rmse"]},
                "rmse_per_iteration": {"exact": [r["rmse"] for r in exact],
                                       "sketched": [r["rmse"] for r in sk]},
                "core_ms_per_iteration": {"exact": [r["core_ms"] for r in exact],
                                          "sketched": [r["core_ms"] for r in sk]},
                "data": "synthetic, generated on the device",
            }
            log(f"[bench] ranks {ranks} s {s}: core exact {out['mean_core_ms']['exact']:.3f} ms, "
                f"sketched {out['mean_core_ms']['sketched']:.3f} ms, rmse "
                f"{out['final_rmse']['exact']:.5f} / {out['final_rmse']['sketched']:.5f}")
            print(json.dumps(out), flush=True)


def bench_microbench(args, tk, workloads, np, torch, dev):
    """The sampling and gather steps (a2-a4) at sizes where their HBM rate means
    something: Alg. 1's count (s = 1687583) on the 1024^3 synthetic-protocol
    tensor fitted at rank 4^3 (whole sampled updates, stage events), and the
    sampler alone at s = 2^24 on the same tables.  Algorithmic bytes: the
    sampler writes s (4 N + 8) bytes (indices and weights; the CDF tables stay
    in LDS); the gather reads s (4 N + 8) bytes of samples plus one tensor
    element per sample and writes 16 s bytes."""
    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: 3 launches reading and writing {nbytes} bytes each")
    dims, ranks = (1024, 1024, 1024), (4, 4, 4)
    X = workloads.table1_problem_device(dims, 11, dev)["X"]
    _, F0 = workloads.als_init(dims, ranks, 1011, "f32")
    F = [torch.from_numpy(np.ascontiguousarray(A)).to(dev) for A in F0]
    lam, s = 1e-3, 1687583
    hip = HipEvents()
    nst = tk.tucker.L.NUM_STAGE_EVENTS
    for k in range(2):
        tk.core_update_sketched(X, F, lam, s, seed=11, counter=k, precision="bf16",
                                refine_max=8, refine_tol=1e-13, check=False)
    ev = [hip.create(nst) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        tk.core_update_sketched(X, F, lam, s, seed=11, counter=100 + k, precision="bf16",
                                refine_max=8, refine_tol=1e-13, check=False,
                                stage_events=ctypes.addressof(ev[k]))
    torch.cuda.synchronize()
    st = {"sample": 0.0, "gather": 0.0}
    for k in range(args.steps):
        st["sample"] += hip.elapsed_ms(ev[k][1], ev[k][2]) / args.steps
        st["gather"] += hip.elapsed_ms(ev[k][2], ev[k][3]) / args.steps
    for e in ev:
        hip.destroy(e)
    N = 3
    # the sampler alone at s = 2^24
    _, cdf = tk.leverage_scores(F)
    big = 1 << 24
    tk.sample(dims, cdf, big, seed=1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for k in range(reps):
        tk.sample(dims, cdf, big, seed=2, counter=k)
    e1.record()
    torch.cuda.synchronize()
    ms_big = e0.elapsed_time(e1) / reps
    out = {
        "microbench": "sampling and gather at Alg. 1's count (1024^3 synthetic protocol, rank 4^3)",
        "t1_samples": s,
        "t1_stage_ms": {k: round(v, 4) for k, v in st.items()},
        "t1_sample_write_GBps": round(s * (4 * N + 8) / (st["sample"] * 1e-3) / 1e9, 1),
        "sampler_2e24_ms": round(ms_big, 4),
        "sampler_2e24_write_GBps": round(big * (4 * N + 8) / (ms_big * 1e-3) / 1e9, 1),
        "sampler_2e24_frac_of_8TBps": round(big * (4 * N + 8) / (ms_big * 1e-3) / 8e12, 4),
    }
    print(json.dumps(out), flush=True)


def bench_batch(args, tk, workloads, np, torch, dev):
    """The 64-problem batch: tuner, graph capture, timed graph replays (BF16 or
    FP32 stream-K Gram; the default FP64 precision selects BF16 here)."""
    if args.precision == "f64":
        args.precision = "bf16"
    t_gen = time.perf_counter()
    probs = workloads.batch_problems(seed=4, count=64)
    lam = 1e-3
    Xs = [torch.from_numpy(p["X"]).to(dev) for p in probs]
    Fs = [[torch.from_numpy(np.ascontiguousarray(A.astype(np.float32))).to(dev)
           for A in p["factors_true"]] for p in probs]
    ss = [p["samples"] for p in probs]
    ds = [int(p["G_true"].size) for p in probs]
    torch.cuda.synchronize()
    log(f"[bench] batch of {len(probs)}: d in [{min(ds)}, {max(ds)}], sum s = {sum(ss)}, "
        f"generated in {time.perf_counter() - t_gen:.1f} s")
    best, times = tk.tune_batched(Xs, Fs, lam, ss, seeds=4, precision=args.precision)
    log(f"[bench] tuner: {best}; candidate Gram times (ms) {[round(t, 3) for t in times]}")
    upd = tk.BatchedSketchedUpdate(Xs, Fs, lam, ss, seeds=4, precision=args.precision,
                                   config=best, refine_max=args.refine_max)
    for _ in range(args.warmup):
        upd.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        upd.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = int(upd.status.abs().sum().item())
    info = upd.info.cpu().numpy()
    ms = wall * 1e3 / args.steps
    flops = float(sum(s * d * (d + 1) for s, d in zip(ss, ds)))
    gram_ms = min(times)
    achieved = flops / (gram_ms * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    log(f"[bench] {args.steps} graph replays: {ms:.3f} ms per batch; status words nonzero: {bad}; "
        f"max refinement residual {info[:, 3].max():.2e}")
    out = {
        "metric": "sketched core updates/sec and ALS iteration time vs exact update at equal loss",
        "value": len(probs) * args.steps / wall,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "name": "c4", "tuned": best,
                   "gram_operands": args.precision, "gram_accumulate": "f32",
                   "solve": "f64 Cholesky + f64 refinement", "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "batched stream-K Gram (one launch, tuner-timed)",
                     "algorithmic_flops": flops, "kernel_ms": round(gram_ms, 4)},
        "cpu_baseline": None,
        "status_nonzero": bad,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
