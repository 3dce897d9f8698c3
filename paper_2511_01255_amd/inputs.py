"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks. This module holds none of the method's arithmetic: it only draws
boundaries, sign patterns and relaxation parameters, and packs +-1 patterns
into the library's bit layout.

Bit layout (population-major): bits[w, i] is a uint32 holding domains
32w .. 32w+31 of genome i; bit k is set exactly when d[i, 32w + k] = -1.
W = ceil(N / 32) rows, ld >= np columns with ld a multiple of 64. Padding
bits and padding columns are 0.

The paper's workloads (Sec. 5) are wavelength-specified lithium-niobate
crystals whose phase mismatch needs a dispersion model the paper does not
give; these generators stand in for them with the mismatch given directly.
"""
import math

import numpy as np

DK1 = 2.0 * math.pi / 19.5  # um^-1, second-harmonic step
DK2 = 2.0 * math.pi / 6.6   # um^-1, sum-frequency step


def words(n):
    return (n + 31) // 32


def ld_for(np_):
    return max(64, ((np_ + 63) // 64) * 64)


def uniform_boundaries(n, width=2.0, z0=0.0):
    """z[0..n] for n domains of one width (um)."""
    return z0 + width * np.arange(n + 1, dtype=np.float64)


def jittered_boundaries(n, width=2.0, jitter=0.25, seed=0, z0=0.0):
    """z[0..n] with widths uniform in width*(1 +- jitter)."""
    rng = np.random.default_rng(seed)
    w = width * (1.0 + rng.uniform(-jitter, jitter, size=n))
    return np.concatenate([[z0], z0 + np.cumsum(w)])


def random_signs(np_, n, seed=0):
    """iid +-1 with p = 1/2, shape (np_, n), int8."""
    rng = np.random.default_rng(seed)
    return np.where(rng.integers(0, 2, size=(np_, n), dtype=np.int8) == 1, -1, 1).astype(np.int8)


def periodic_signs(count, n, width=2.0, period=19.5, seed=0):
    """First-order periodic poling seeds with a random phase offset:
    d_n = +1 iff cos(2 pi (m_n - phi) / period) >= 0, m_n the domain centre,
    phi uniform on [0, period)."""
    rng = np.random.default_rng(seed)
    m = (np.arange(n, dtype=np.float64) + 0.5) * width
    out = np.empty((count, n), dtype=np.int8)
    for c in range(count):
        phi = rng.uniform(0.0, period)
        out[c] = np.where(np.cos(2.0 * math.pi * (m - phi) / period) >= 0.0, 1, -1)
    return out


def fitness_population(np_=4096, n=10000, width=2.0, n_periodic=32, seed=1):
    """The fitness-throughput population: np_ - n_periodic iid genomes
    followed by n_periodic periodic seeds."""
    a = random_signs(np_ - n_periodic, n, seed)
    b = periodic_signs(n_periodic, n, width, 19.5, seed + 1000)
    return np.concatenate([a, b], axis=0)


def pack_bits(d, ld=None):
    """(np, n) +-1 -> uint32 (W, ld) population-major bit words."""
    d = np.asarray(d)
    np_, n = d.shape
    W = words(n)
    ld = ld_for(np_) if ld is None else ld
    neg = np.zeros((np_, W * 32), dtype=np.uint8)
    neg[:, :n] = (d < 0)
    # bit k of word w <- domain 32 w + k
    b = neg.reshape(np_, W, 32).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    wordsv = (b * weights).sum(axis=2).astype(np.uint32)  # (np, W)
    out = np.zeros((W, ld), dtype=np.uint32)
    out[:, :np_] = wordsv.T
    return out


def unpack_bits(bits, np_, n):
    """uint32 (W, ld) -> (np_, n) int8 +-1."""
    bits = np.asarray(bits).view(np.uint32)
    W = bits.shape[0]
    cols = bits[:, :np_].T  # (np, W)
    k = np.arange(32, dtype=np.uint32)
    neg = ((cols[:, :, None] >> k) & 1).reshape(np_, W * 32)[:, :n]
    return np.where(neg == 1, -1, 1).astype(np.int8)


def batched_designs(n_inst=64, seed=1, n_lo=1000, n_hi=50000):
    """Uneven independent designs: N ~ U[n_lo, n_hi], width ~ U[1.5, 3.0] um,
    dk1 = 2 pi / U[18, 21] um^-1, dk2 = 2 pi / U[6.2, 7.0] um^-1.
    Returns a list of (z, dk1, dk2)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        n = int(rng.integers(n_lo, n_hi + 1))
        w = rng.uniform(1.5, 3.0)
        lam1 = rng.uniform(18.0, 21.0)
        lam2 = rng.uniform(6.2, 7.0)
        out.append((uniform_boundaries(n, w), 2.0 * math.pi / lam1, 2.0 * math.pi / lam2))
    return out


def relax_theta(B, n, seed=1):
    """theta ~ N(0, 1), float32, shape (B, n)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(B, n)).astype(np.float32)
