"""Philox4x64-10 counter-based generator, written from its published definition.

Test infrastructure only (see ``oracle/__init__.py``).

Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11) maps a 256-bit counter (four 64-bit words) and a 128-bit key
(two 64-bit words) to four 64-bit output words.  One round is

    (hi0, lo0) = M0 * c0        (full 128-bit product)
    (hi1, lo1) = M1 * c2
    c <- (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)

and the key is bumped by the Weyl constants (W0, W1) before every round but the
first.  Ten rounds.

The paper leaves the random source of its sampler unspecified (Alg. 1 draws
rows i.i.d.; Thm 4.2 draws each multi-index by one inverse-CDF search per
mode).  A counter-based generator lets any number of threads draw sample t
without a shared state, and lets this oracle reproduce every draw.

Two implementations live here: ``philox4x64_scalar`` on Python integers (the
definition, for tiny cases) and ``philox4x64`` vectorised over numpy uint64
arrays with the 128-bit products split into 32-bit limbs.
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10


def philox4x64_scalar(ctr, key):
    """Philox4x64-10 on Python ints: ctr is 4 words, key is 2 words."""
    c = [int(v) & MASK64 for v in ctr]
    k = [int(v) & MASK64 for v in key]
    for r in range(ROUNDS):
        if r > 0:
            k[0] = (k[0] + W0) & MASK64
            k[1] = (k[1] + W1) & MASK64
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit unsigned product of uint64 arrays: (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | ((mid & _M32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def mulhi64(a, b):
    """Upper 64 bits of the 128-bit product a*b (uint64 arrays)."""
    return mulhilo64(a, b)[0]


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10; every argument broadcasts as uint64."""
    with np.errstate(over="ignore"):
        c = [np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3)]
        c = list(np.broadcast_arrays(*c))
        k = [np.uint64(int(k0) & MASK64), np.uint64(int(k1) & MASK64)]
        m0, m1 = np.uint64(M0), np.uint64(M1)
        w0, w1 = np.uint64(W0), np.uint64(W1)
        for r in range(ROUNDS):
            if r > 0:
                k = [k[0] + w0, k[1] + w1]
            hi0, lo0 = mulhilo64(m0, c[0])
            hi1, lo1 = mulhilo64(m1, c[2])
            c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c
