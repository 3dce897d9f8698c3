"""Whole generations in one workgroup (the population in LDS) against the
CPU oracle and against the multi-kernel path: the same trajectories bit for
bit (FP64 fitness within 1e-12 of the oracle, within 1e-13 between the two
paths, whose FP64 sums are associated differently)."""
import numpy as np
import pytest

from paper_2511_01255_amd import inputs

pytestmark = pytest.mark.gpu

DK1, DK2 = inputs.DK1, inputs.DK2


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_2511_01255_amd import qpm
    qpm.lib()
    return qpm


@pytest.mark.parametrize("case", [
    # (N, NP, G, algo, GWO variant, control, instance)
    (256, 32, 200, 0, 0, 0, 0),    # the plain configuration (tables in LDS)
    (256, 64, 40, 0, 0, 0, 1),     # tables read from global memory (LDS full)
    (257, 17, 30, 0, 1, 1, 2),     # ragged words and quads, mean variant, decaying F = a
    (33, 5, 50, 0, 0, 0, 0),       # one word and a bit
    (1, 4, 12, 0, 0, 0, 0),        # one domain: every genome ties
    (1000, 16, 25, 1, 0, 0, 3),    # DE alone
    (400, 40, 25, 2, 1, 1, 0),     # grey wolf alone
], ids=lambda c: "n%d_np%d_g%d_algo%d_v%d_c%d_i%d" % c)
def test_fused_run_equals_oracle_and_multikernel(q, orc, case):
    n, npop, G, algo, variant, control, inst = case
    z = inputs.jittered_boundaries(n, 2.0, 0.25, seed=n + 11)
    D = q.precompute_phases(z, DK1, DK2)
    xo, fo, _, par = orc.Design(z, DK1, DK2).run_algo(npop, G, 0.5, 0.9, 13, algo, inst=inst, variant=variant,
                                                      control=control)
    outs = []
    for fused in (1, -1):
        R = q.Run(D, npop, G, seed=13, inst=inst, prec=1, gwo_variant=variant, control=control, algo=algo,
                  fused=fused)
        R.advance(G // 3)
        R.advance(G - G // 3)
        x, f, L, g = R.read()
        _, _, st = R.best()
        outs.append((x.cpu().numpy(), f.cpu().numpy(), L, st.best_index))
        assert g == G
        R.destroy()
    for x, f, L, b in outs:
        assert np.array_equal(x, xo)
        assert np.max(np.abs(f - fo) / np.maximum(fo, 1e-300)) <= 1e-12
        assert b == int(np.argmax(fo))
    assert outs[0][2] == outs[1][2]  # the leaders reported
    assert np.max(np.abs(outs[0][1] - outs[1][1]) / np.maximum(outs[1][1], 1e-300)) <= 1e-13


def test_fused_alternates_with_multikernel_steps_and_polish(q, orc):
    # fused generations, then generations through the multi-kernel path
    # (timing mode launches step by step), a polish of the leaders, fused
    # again: the state moves between the paths intact, and the run without
    # the polish equals the oracle
    n, npop, G = 256, 32, 60
    z = inputs.uniform_boundaries(n, 2.0)
    D = q.precompute_phases(z, DK1, DK2)
    xo, fo, _ = orc.Design(z, DK1, DK2).hwsda_run(npop, G, 0.5, 0.9, 4)
    R = q.Run(D, npop, G, seed=4, prec=1, fused=1)
    R.advance(20)
    R.set_timing(True)
    R.advance(15)
    R.set_timing(False)
    R.advance(25)
    x, f, _, _ = R.read()
    assert np.array_equal(x.cpu().numpy(), xo)
    R.destroy()
    R = q.Run(D, npop, G, seed=4, prec=1, fused=1)
    R.advance(30)
    R.polish(5, 0.05)
    R.advance(30)
    x2, f2, _, _ = R.read()
    f2 = f2.cpu().numpy()
    # every stored fitness is the oracle's fitness of the stored genes
    _, fe = orc.Design(z, DK1, DK2).fitness(orc.sign_map(x2.cpu().numpy()))
    assert np.max(np.abs(f2 - fe) / fe) <= 1e-12
    R.destroy()


def test_fused_required_but_not_possible(q):
    D = q.precompute_phases(inputs.uniform_boundaries(256, 2.0), DK1, DK2)
    for kw in (dict(prec=1, control=2), dict(prec=1, gwo_variant=2), dict(prec=1, np_=65),
               dict(prec=1, fit_kernel=1), dict(prec=0, fit_kernel=1)):
        np_ = kw.pop("np_", 32)
        with pytest.raises(q.QpmError):
            q.Run(D, np_, 10, fused=1, **kw)
    with pytest.raises(q.QpmError):
        q.Run(D, 32, 10, prec=1, fused=2)


@pytest.mark.parametrize("case", [(256, 32, 40, 3), (257, 17, 30, 5), (600, 24, 12, 7)],
                         ids=lambda c: "n%d_np%d_g%d_s%d" % c)
def test_fused_fp32_run_lockstep(q, orc, case):
    # FP32 runs take the fused path too (the FP64 table walk, each fitness
    # rounded to binary32): every row of every generation against the
    # oracle's replay from the run's own state; a decision may go the other
    # way only on a near tie, and such adoptions must stay rare
    from test_gpu_parity import _lockstep_generation
    n, npop, G, seed = case
    F, CR = 0.5, 0.9
    z = inputs.uniform_boundaries(n, 2.0)
    D = q.precompute_phases(z, DK1, DK2)
    O = orc.Design(z, DK1, DK2)
    R = q.Run(D, npop, G, F=F, CR=CR, seed=seed, prec=0, fused=1)
    adoptions = sum(_lockstep_generation(orc, O, R, g, G, F, CR, seed) for g in range(G))
    print("fused FP32 lockstep: %d generations, %d adopted near-tie decisions" % (G, adoptions))
    assert adoptions <= max(2, G * (2 * npop - 3) // 1000), adoptions
    R.destroy()
