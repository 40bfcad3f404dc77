"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and assembles low-rank-plus-noise test
tensors; it contains none of the sampled core update's arithmetic (no leverage
scores, sampling, Gram or solve).  Everything is generated in float64 with
``numpy.random.default_rng(seed)`` and then cast, so the oracle and the GPU see
the same stored values.

Workloads (shapes follow the paper's experiments, Sec. 5, and the parity cases):

* ``c1``: 64^3 float64, core 4^3 ~ N(0,1), orthonormal Gaussian factors,
  noise N(0, 0.01^2); lambda 1e-3; 2048 samples; 5 ALS iterations.
* ``c2``: 512^3 float32, rank 16^3, Gaussian-then-QR factors, noise at 20 dB
  SNR; lambda 1e-2; 131072 samples.
* ``c3``: 128^4 float32, rank 8^4, 10 % of entries missing uniformly at random;
  lambda 1e-3; 65536 samples; BF16 Gram plus FP64 refinement.
* ``c4``: 64 order-3 float32 problems, sides U{32..384}, ranks U{4..24},
  Gaussian factors and core, 1 % relative noise; 16 * prod(ranks) samples each.
* ``c5``: 256^3 float32, rank 12^3; lambda 1e-2; 32768 samples; adjoint case.
* ``table1``: the synthetic protocol of Sec. 5 (true core 8^3, factor and core
  entries U[0,1], N(0,1) noise on 1 % of the entries), a stand-in for the
  paper's synthetic benchmark at any input shape.
* ``t1``: that protocol at the largest shape of the paper's synthetic table,
  1024^3 float32, fitted at rank 4^3 from the U[0,1] initial state of Alg. 2;
  lambda 1e-3; the Alg. 1 sample count for eps = delta = 0.1 at d = 64
  (1687583 samples).  Generated in mode-0 slabs with one child generator each.
* ``movie``: a stand-in for the paper's video tensor, (100, 1080, 1920, 3)
  float32 in [0, 1], low rank in time and colour and smooth in space, built on
  the device (``movie_problem_device``); fitted at core (2, 4, 4, 2).
* ``t1big``: the same protocol at 2560^3 float32 (67 GB), generated on the
  device by ``table1_problem_device`` (torch's seeded device generator, slab by
  slab); no oracle reads it.  It shows the sampled update's cost staying fixed
  while the exact update's pass over X grows with the tensor.
"""
import numpy as np

CONFIGS = {
    "c1": dict(dims=(64, 64, 64), ranks=(4, 4, 4), dtype="f64", lam=1e-3, samples=2048,
               seed=0, factor="qr", core="normal", noise=("sigma", 0.01), als_iters=5,
               gram="f64"),
    "c2": dict(dims=(512, 512, 512), ranks=(16, 16, 16), dtype="f32", lam=1e-2,
               samples=131072, seed=2, factor="qr", core="normal", noise=("snr_db", 20.0),
               gram="bf16"),
    "c3": dict(dims=(128, 128, 128, 128), ranks=(8, 8, 8, 8), dtype="f32", lam=1e-3,
               samples=65536, seed=3, factor="qr", core="normal", noise=("snr_db", 20.0),
               missing=0.1, gram="bf16"),
    "c5": dict(dims=(256, 256, 256), ranks=(12, 12, 12), dtype="f32", lam=1e-2,
               samples=32768, seed=5, factor="qr", core="normal", noise=("snr_db", 20.0),
               gram="f64"),
    "t1": dict(dims=(1024, 1024, 1024), ranks=(4, 4, 4), dtype="f32", lam=1e-3,
               samples=1687583, seed=11, protocol="table1", true_rank=(8, 8, 8), init_seed=1011,
               gram="bf16"),
    "t1big": dict(dims=(2560, 2560, 2560), ranks=(4, 4, 4), dtype="f32", lam=1e-3,
                  samples=1687583, seed=12, protocol="table1_device", true_rank=(8, 8, 8),
                  init_seed=1012, gram="bf16"),
}

NP_DTYPES = {"f64": np.float64, "f32": np.float32}


def _mode_mul(T, A, n):
    out = np.tensordot(A, T, axes=([1], [n]))
    return np.moveaxis(out, 0, n)


def _factor(rng, I, R, kind):
    if kind == "qr":
        Q, _ = np.linalg.qr(rng.standard_normal((I, R)))
        return Q
    if kind == "gaussian":
        return rng.standard_normal((I, R))
    if kind == "uniform":
        return rng.random((I, R))
    raise ValueError(kind)


def pack_mask(observed):
    """LSB-first uint32 words: bit j of word w is entry 32 w + j (1 = observed)."""
    flat = np.asarray(observed, dtype=bool).reshape(-1)
    pad = (-flat.size) % 32
    if pad:
        flat = np.concatenate([flat, np.zeros(pad, dtype=bool)])
    bits = flat.reshape(-1, 32).astype(np.uint64)
    words = (bits << np.arange(32, dtype=np.uint64)).sum(axis=1)
    return words.astype(np.uint32)


def tucker_tensor(dims, ranks, seed, dtype="f64", factor="qr", core="normal",
                  noise=("sigma", 0.01), missing=None):
    """Low-rank Tucker tensor plus noise; returns a dict of numpy arrays.

    Keys: X (dtype), G_true, factors_true (float64), mask (uint32 words or None).
    noise: ("sigma", s) adds N(0, s^2); ("snr_db", q) scales N(0,1) noise to
    RMS(Xhat) / 10^(q/20); ("rel", r) to r * RMS(Xhat); ("sparse", p, s) adds
    N(0, s^2) to a fraction p of the entries.
    """
    rng = np.random.default_rng(seed)
    A = [_factor(rng, I, R, factor) for I, R in zip(dims, ranks)]
    if core == "normal":
        G = rng.standard_normal(ranks)
    elif core == "uniform":
        G = rng.random(ranks)
    else:
        raise ValueError(core)
    X = G
    for n, An in enumerate(A):
        X = _mode_mul(X, An, n)
    kind = noise[0]
    if kind == "sigma":
        X = X + noise[1] * rng.standard_normal(X.shape)
    elif kind in ("snr_db", "rel"):
        rms = float(np.sqrt(np.mean(X * X)))
        scale = rms / 10.0 ** (noise[1] / 20.0) if kind == "snr_db" else rms * noise[1]
        X = X + scale * rng.standard_normal(X.shape)
    elif kind == "sparse":
        hit = rng.random(X.shape) < noise[1]
        X = X + hit * (noise[2] * rng.standard_normal(X.shape))
    elif kind != "none":
        raise ValueError(kind)
    mask = None
    if missing:
        mask = pack_mask(rng.random(X.shape) >= missing)
    return dict(X=np.ascontiguousarray(X.astype(NP_DTYPES[dtype])), G_true=G,
                factors_true=A, mask=mask)


def config_problem(name, **overrides):
    """The named workload (see module docstring) with optional overrides."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if cfg.get("protocol") == "table1_device":
        dev = overrides.get("device", "cuda")
        prob = table1_problem_device(cfg["dims"], cfg["seed"], dev, cfg["true_rank"])
        _, F0 = als_init(cfg["dims"], cfg["ranks"], cfg["init_seed"], "f64")
        prob["factors_fit"] = F0
        prob["cfg"] = cfg
        return prob
    if cfg.get("protocol") == "table1":
        prob = table1_problem(cfg["dims"], cfg["seed"], cfg["dtype"], cfg["true_rank"], slabs=True)
        _, F0 = als_init(cfg["dims"], cfg["ranks"], cfg["init_seed"], "f64")
        prob["factors_fit"] = F0
        prob["cfg"] = cfg
        return prob
    prob = tucker_tensor(cfg["dims"], cfg["ranks"], cfg["seed"], cfg["dtype"], cfg["factor"],
                         cfg["core"], cfg["noise"], cfg.get("missing"))
    prob["cfg"] = cfg
    return prob


def table1_problem(dims, seed, dtype="f32", true_rank=(8, 8, 8), slabs=False, slab_rows=32):
    """Sec. 5 synthetic protocol: U[0,1] core and factors, N(0,1) noise on 1 % of entries.

    With ``slabs`` the tensor is built ``slab_rows`` mode-0 rows at a time (same
    core and factors; the noise of slab b comes from default_rng([seed, 1, b])),
    so that a 1024^3 tensor needs no full-size float64 temporaries.
    """
    if not slabs:
        return tucker_tensor(dims, true_rank, seed, dtype, factor="uniform", core="uniform",
                             noise=("sparse", 0.01, 1.0))
    rng = np.random.default_rng(seed)
    A = [_factor(rng, I, R, "uniform") for I, R in zip(dims, true_rank)]
    G = rng.random(true_rank)
    # mode 0 applied last: W[j..., r0] = G x_1.. A(1..N-1) with the mode-0 index kept
    W = G
    for n in range(1, len(dims)):
        W = _mode_mul(W, A[n], n)
    W0 = W.reshape(true_rank[0], -1)
    X = np.empty(dims, dtype=NP_DTYPES[dtype])
    for b, i0 in enumerate(range(0, dims[0], slab_rows)):
        i1 = min(dims[0], i0 + slab_rows)
        child = np.random.default_rng([seed, 1, b])
        xs = (A[0][i0:i1] @ W0).reshape((i1 - i0,) + tuple(dims[1:]))
        hit = child.random(xs.shape) < 0.01
        xs[hit] += child.standard_normal(int(hit.sum()))
        X[i0:i1] = xs
    return dict(X=X, G_true=G, factors_true=A, mask=None)


def table1_problem_device(dims, seed, device, true_rank=(8, 8, 8), slab_rows=64):
    """Sec. 5 protocol built on a torch device in float32, for tensors too large
    for host memory: U[0,1] core and factors from default_rng(seed) (host, as
    in table1_problem), the low-rank part formed slab by slab on the device, and
    N(0,1) noise on 1 % of the entries from a torch generator seeded with seed.
    Returns X (device tensor), G_true and factors_true (numpy)."""
    import torch
    rng = np.random.default_rng(seed)
    A = [_factor(rng, I, R, "uniform") for I, R in zip(dims, true_rank)]
    G = rng.random(true_rank)
    W = G
    for n in range(1, len(dims)):
        W = _mode_mul(W, A[n], n)
    W0 = torch.from_numpy(np.ascontiguousarray(W.reshape(true_rank[0], -1))).to(device)
    A0 = torch.from_numpy(A[0]).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    X = torch.empty(dims, dtype=torch.float32, device=device)
    for i0 in range(0, dims[0], slab_rows):
        i1 = min(dims[0], i0 + slab_rows)
        xs = (A0[i0:i1] @ W0).reshape((i1 - i0,) + tuple(dims[1:]))
        hit = torch.rand(xs.shape, generator=gen, device=device, dtype=torch.float32) < 0.01
        noise = torch.randn(xs.shape, generator=gen, device=device, dtype=torch.float32)
        X[i0:i1] = (xs + hit * noise.double()).float()
        del xs, hit, noise
    return dict(X=X, G_true=G, factors_true=A, mask=None)


def movie_problem_device(seed, device, dims=(100, 1080, 1920, 3), components=6, sigma=0.02):
    """Stand-in for the paper's video tensor (Sec. 5: 100 frames of 1080 x 1920
    RGB; the dataset itself is not available): float32 in [0, 1], built on the
    device frame by frame as
      X[t, h, w, c] = clip(0.5 + sum_k a_k(t) s_k(h) r_k(w) q_k(c) + noise, 0, 1),
    with slowly varying temporal weights a_k(t), smooth low-frequency spatial
    profiles s_k, r_k (a separable picture per component), per-component colour
    vectors q_k, and N(0, sigma^2) pixel noise.  Low rank in time and colour,
    smooth in space; a (2, 4, 4, 2) Tucker model fits it only approximately.
    The parameters come from default_rng(seed), the noise from a torch
    generator seeded with seed.  Returns X (device tensor)."""
    import torch
    T, H, W, C = dims
    rng = np.random.default_rng(seed)
    tt, hh, ww = np.arange(T) / T, np.arange(H) / H, np.arange(W) / W
    a = np.stack([0.25 * np.sin(2 * np.pi * (rng.uniform(0.2, 1.5) * tt + rng.random()))
                  for _ in range(components)])                       # (K, T)
    sh = np.stack([np.cos(2 * np.pi * (rng.uniform(0.3, 2.5) * hh + rng.random()))
                   for _ in range(components)])                      # (K, H)
    sw = np.stack([np.cos(2 * np.pi * (rng.uniform(0.3, 2.5) * ww + rng.random()))
                   for _ in range(components)])                      # (K, W)
    q = rng.random((components, C))                                  # (K, C)
    dev_a = torch.from_numpy(a).to(device)
    S = torch.from_numpy(sh).to(device)
    R = torch.from_numpy(sw).to(device)
    Q = torch.from_numpy(q).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    X = torch.empty(dims, dtype=torch.float32, device=device)
    for t in range(T):
        # frame t: sum_k a_k(t) s_k(h) r_k(w) q_k(c), elementwise broadcasts only
        f = torch.full((H, W, C), 0.5, dtype=torch.float64, device=device)
        for k in range(components):
            f += dev_a[k, t] * (S[k][:, None, None] * R[k][None, :, None] * Q[k][None, None, :])
        f += sigma * torch.randn(f.shape, generator=gen, device=device, dtype=torch.float64)
        X[t] = f.clamp_(0.0, 1.0).float()
        del f
    return X


def als_init(dims, ranks, init_seed, dtype="f64"):
    """Random initial state of Alg. 2: core and factor entries i.i.d. U[0,1)."""
    rng = np.random.default_rng(init_seed)
    G = rng.random(ranks)
    A = [rng.random((I, R)) for I, R in zip(dims, ranks)]
    t = NP_DTYPES[dtype]
    return G.astype(t), [a.astype(t) for a in A]


def random_factors(dims, ranks, seed, kind="qr", dtype="f64"):
    """Factor matrices only (for sampler / leverage-score cases)."""
    rng = np.random.default_rng(seed)
    t = NP_DTYPES[dtype]
    return [_factor(rng, I, R, kind).astype(t) for I, R in zip(dims, ranks)]


def batch_problems(seed=4, count=64, side=(32, 384), rank=(4, 24), rel_noise=0.01,
                   dtype="f32", max_elems=None):
    """Uneven batch: order-3 tensors with sides U{side} and ranks U{rank} per mode.

    Gaussian factors and core, noise at ``rel_noise`` times RMS(Xhat).  Each
    problem gets 16 * prod(ranks) samples.  ``max_elems`` (optional) rejects
    and redraws tensors larger than that many entries, for small test batches.
    """
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        dims = tuple(int(v) for v in rng.integers(side[0], side[1] + 1, size=3))
        ranks = tuple(int(v) for v in rng.integers(rank[0], rank[1] + 1, size=3))
        sub_seed = int(rng.integers(0, 2 ** 31))
        if max_elems is not None and np.prod(dims) > max_elems:
            continue
        p = tucker_tensor(dims, ranks, sub_seed, dtype, factor="gaussian", core="normal",
                          noise=("rel", rel_noise))
        p["samples"] = 16 * int(np.prod(ranks))
        out.append(p)
    return out
