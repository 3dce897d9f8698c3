"""Worst-conditioned fitness inputs and the rare branches of the optimiser
steps, against the CPU oracle.

Periodic first-order poling seeds are the hardest genomes for the FP32
fitness: the prefix P grows linearly with N while the outer sum is not
phase-matched, so large terms cancel. Their |d_eff|^2 is large, so the
tolerance is checked as a plain relative error (no floor); iid genomes are
reported both ways and checked against max(f, 1e-2 median f).
"""
import math

import numpy as np
import pytest

from paper_2511_01255_amd import inputs

pytestmark = pytest.mark.gpu

DK1, DK2 = inputs.DK1, inputs.DK2
TOL = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_2511_01255_amd import qpm
    qpm.lib()
    return qpm


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(d, ld=None):
    return _dev(inputs.pack_bits(d, ld).view(np.int32))


@pytest.mark.parametrize("prec", [0, 1])
def test_fitness_periodic_seeds_n50000(q, orc, prec):
    # N = 5 x 10^4 domains x 2 um (the relaxation workload's length, the
    # largest instances of the batched workload): 32 periodic seeds with
    # random phase offsets and 96 iid genomes, every kernel
    n = 50000
    z = inputs.uniform_boundaries(n, 2.0)
    d = np.concatenate([inputs.periodic_signs(32, n, 2.0, 19.5, seed=11), inputs.random_signs(96, n, seed=12)])
    npop = d.shape[0]
    D = q.precompute_phases(z, DK1, DK2)
    _, fo = orc.Design(z, DK1, DK2).fitness(d)
    bits = _bits(d)
    kernels = [q.FIT_TABLE, q.FIT_SEGMENTED] + ([q.FIT_PER_GENOME] if prec == 1 else [])
    for kernel in kernels:
        f = q.eval_fitness(D, bits, npop, prec=prec, kernel=kernel).double().cpu().numpy()
        rel = np.abs(f - fo) / fo
        floored = np.abs(f - fo) / np.maximum(fo, 1e-2 * np.median(fo))
        print("prec %d kernel %d: periodic max rel %.3g; iid max rel %.3g (floored %.3g)"
              % (prec, kernel, rel[:32].max(), rel[32:].max(), floored[32:].max()))
        assert rel[:32].max() <= TOL[prec], (kernel, rel[:32].max())
        assert floored.max() <= TOL[prec], (kernel, floored.max())


def test_fitness_periodic_batched_design_range(q, orc):
    # designs drawn like the batched workload (uniform width in [1.5, 3] um,
    # dk1 = 2 pi / U[18, 21] um^-1, dk2 = 2 pi / U[6.2, 7] um^-1) at its
    # largest N, each with first-order periodic seeds of its own period:
    # the single-design FP32 kernels and the batched FP32 kernel
    rng = np.random.default_rng(21)
    specs, ds = [], []
    for k in range(4):
        n = int(rng.integers(40000, 50001))
        w = rng.uniform(1.5, 3.0)
        lam1, lam2 = rng.uniform(18.0, 21.0), rng.uniform(6.2, 7.0)
        z = inputs.uniform_boundaries(n, w)
        specs.append((z, 2 * math.pi / lam1, 2 * math.pi / lam2))
        ds.append(np.concatenate([inputs.periodic_signs(24, n, w, lam1, seed=30 + k),
                                  inputs.random_signs(40, n, seed=40 + k)]))
    npop = 64
    ld = inputs.ld_for(npop)
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    stacked = _dev(np.concatenate([inputs.pack_bits(d, ld) for d in ds], axis=0).view(np.int32))
    fb = q.batch_eval_fitness(B, stacked, npop, q.PREC_F32).double().cpu().numpy()
    worst = 0.0
    for k, (z, k1, k2) in enumerate(specs):
        _, fo = orc.Design(z, k1, k2).fitness(ds[k])
        D = q.precompute_phases(z, k1, k2)
        for name, f in (("table", q.eval_fitness(D, _bits(ds[k]), npop, prec=0, kernel=q.FIT_TABLE)),
                        ("segmented", q.eval_fitness(D, _bits(ds[k]), npop, prec=0, kernel=q.FIT_SEGMENTED)),
                        ("batched", fb[k])):
            f = np.asarray(f.double().cpu().numpy() if hasattr(f, "cpu") else f)
            rel = np.abs(f - fo) / fo
            floored = np.abs(f - fo) / np.maximum(fo, 1e-2 * np.median(fo))
            worst = max(worst, rel[:24].max())
            assert rel[:24].max() <= 1e-5, (k, name, rel[:24].max())
            assert floored.max() <= 1e-5, (k, name, floored.max())
    print("batched-range periodic seeds: max rel %.3g" % worst)


def _bitwise(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


@pytest.mark.parametrize("a", [0.0, 1.0])
@pytest.mark.parametrize("variant", [0, 1])
def test_gwo_zero_and_tiny_genes_bit_exact(q, orc, a, variant):
    # leaders and wolves holding 0.0, -0.0 and |x| < 2^-60 (subnormal results
    # included) mixed into the first wave of gene quads of half the wolves;
    # the weighted combination then leaves its short division form for the
    # full IEEE division, and a zero weight sum gives y = 0. The other waves
    # keep the short form. Candidates and bits must be the oracle's.
    import torch
    npop, D = 80, 1000
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, size=(npop, D)).astype(np.float32)
    specials = np.array([0.0, -0.0, 1e-20, -3e-25, 2.0 ** -70, -2.0 ** -61, 1e-38, 5e-42], dtype=np.float32)
    L = np.array([0, 1, 2], dtype=np.int32)
    # leaders: whole zero quads, tiny quads and mixed ones in genes 0..255
    for k in L:
        idx = rng.choice(256, size=96, replace=False)
        x[k, idx] = rng.choice(specials, size=96)
    x[L, 0:8] = 0.0          # every leader zero: s = 0 when the wolf is 0 too
    x[L[0], 8:12] = -0.0
    for i in range(3, npop, 2):
        idx = rng.choice(256, size=64, replace=False)
        x[i, idx] = rng.choice(specials, size=64)
        x[i, 0:4] = 0.0
    ldx = inputs.ld_for(D)
    xp = np.zeros((npop, ldx), dtype=np.float32)
    xp[:, :D] = x
    xd = _dev(xp)
    y, yb = q.gwo_step(xd, D, L, a, seed=7, generation=3, variant=variant)
    yo = orc.gwo_step(x, L, np.float32(a), seed=7, g=3, variant=variant)
    yg = y.cpu().numpy()[:, :D]
    assert np.array_equal(_bitwise(yg), _bitwise(yo))
    keep = np.setdiff1d(np.arange(npop), L)
    assert np.array_equal(inputs.unpack_bits(yb.cpu().numpy(), npop, D)[keep], orc.sign_map(yo)[keep])
    if a == 0.0 and variant == 0:
        # a = 0: Y_k = X_k, so where all three leaders are 0 the sum is 0
        assert np.all(_bitwise(yg[3:, 0:8]) == 0)
    nz = np.count_nonzero((np.abs(yo[keep, :256]) < 2.0 ** -60) & (yo[keep, :256] != 0))
    print("a %g variant %d: %d candidates below 2^-60 (nonzero), %d zero" %
          (a, variant, nz, np.count_nonzero(yo[keep, :256] == 0)))
