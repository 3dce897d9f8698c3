"""Batches of independent designs of uneven N and phase mismatch: the
batched tables, the batched fitness and the batched run against the CPU
oracle instance by instance."""
import math

import numpy as np
import pytest

from paper_2511_01255_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_01255_amd import qpm
    qpm.lib()
    return qpm


def _small_batch():
    rng = np.random.default_rng(4)
    specs = []
    for n in (1, 33, 1007, 300, 2049, 64):
        z = inputs.jittered_boundaries(n, rng.uniform(1.5, 3.0), 0.2, seed=n)
        specs.append((z, 2 * math.pi / rng.uniform(18, 21), 2 * math.pi / rng.uniform(6.2, 7.0)))
    return specs


def _stack_bits(ds, ld):
    return np.concatenate([inputs.pack_bits(d, ld) for d in ds], axis=0)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("shape", [(0, 0), (4, 1), (8, 3), (16, 40)])
def test_batch_fitness_matches_oracle(q, orc, prec, shape):
    import torch
    specs = _small_batch()
    npop = 70
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    ds = [inputs.random_signs(npop, len(s[0]) - 1, seed=k) for k, s in enumerate(specs)]
    ld = inputs.ld_for(npop)
    bits = torch.from_numpy(_stack_bits(ds, ld).view(np.int32)).cuda()
    f = q.batch_eval_fitness(B, bits, npop, prec, *shape).double().cpu().numpy()
    ns, Cs = B.info()
    for k, (z, k1, k2) in enumerate(specs):
        O = orc.Design(z, k1, k2)
        _, fo = O.fitness(ds[k])
        floor = 1e-2 * np.median(fo)
        err = np.max(np.abs(f[k] - fo) / np.maximum(fo, floor))
        assert err <= (1e-12 if prec == 1 else 1e-5), (k, err)
        assert ns[k] == len(z) - 1
        assert abs(Cs[k] - O.phases()[3]) <= 1e-12 * abs(O.phases()[3]) + 1e-300


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("groups", [1, 2, 4])
def test_batch_table_fitness_every_shape(q, orc, prec, groups):
    # the table kernel over uneven instances (N = 1 ... 2049), every words
    # per wave the LDS allows, ragged population
    import torch
    specs = _small_batch()
    npop = 197
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    ds = [inputs.random_signs(npop, len(s[0]) - 1, seed=10 + k) for k, s in enumerate(specs)]
    bits = torch.from_numpy(_stack_bits(ds, inputs.ld_for(npop)).view(np.int32)).cuda()
    refs = [orc.Design(z, k1, k2).fitness(ds[k])[1] for k, (z, k1, k2) in enumerate(specs)]
    for wpw in range(1, 6 if prec == 0 else 3):
        f = q.batch_eval_fitness_table(B, bits, npop, prec, groups, wpw).double().cpu().numpy()
        for k, fo in enumerate(refs):
            floor = 1e-2 * np.median(fo)
            err = np.max(np.abs(f[k] - fo) / np.maximum(fo, floor))
            assert err <= (1e-12 if prec == 1 else 1e-5), (wpw, k, err)


@pytest.mark.parametrize("trials", [1, 2])
def test_batch_run_fp64_equals_oracle_runs(q, orc, trials):
    # every instance follows the single-design run with instance number
    # inst0 + b: same trajectory as the oracle's run, bit for bit, with every
    # trial stored (1) or the accepted ones recomputed after selection (2)
    specs = _small_batch()[1:]  # N >= 33
    npop, G, inst0 = 24, 12, 5
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    R = q.BatchRun(B, npop, G, seed=3, inst=inst0, prec=q.PREC_F64, tune=0, trials=trials)
    R.advance(G)
    for b, (z, k1, k2) in enumerate(specs):
        x, f, L, _ = R.read(b)
        xo, fo, _ = orc.Design(z, k1, k2).hwsda_run(npop, G, 0.5, 0.9, 3, inst=inst0 + b)
        assert np.array_equal(x.cpu().numpy(), xo), b
        assert np.max(np.abs(f.cpu().numpy() - fo) / fo) <= 1e-12
    R.destroy()


def test_batch_run_rejects_unsupported_options(q):
    specs = _small_batch()[1:3]
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    with pytest.raises(q.QpmError):
        q.BatchRun(B, 16, 4, gwo_variant=2)


def test_batch_run_tuned_and_graph_agree(q):
    specs = _small_batch()
    npop, G = 40, 6
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    outs = []
    for tune, graph in ((1, 1), (0, 0)):
        R = q.BatchRun(B, npop, G, seed=7, prec=q.PREC_F64, tune=tune, use_graph=graph)
        R.advance(G)
        outs.append([R.read(b)[0].cpu().numpy() for b in range(B.n_inst)])
        R.destroy()
    # launch shapes only change the FP64 summation order of f (~1e-16), far
    # below any gap between distinct genomes: identical trajectories
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("graph,trials", [(1, 1), (0, 1), (1, 2)])
def test_batch_run_every_de_shape_same_trajectory(q, orc, graph, trials):
    # the DE launch shape (individuals per wave x passes) moves no gene: every
    # shape gives the oracle's FP64 trajectory; np = 37 leaves ragged groups
    # and N = 1007 / 2049 ragged gene chunks for every chunk width
    specs = _small_batch()[1:]
    npop, G, inst0 = 37, 5, 2
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    want = [orc.Design(z, k1, k2).hwsda_run(npop, G, 0.5, 0.9, 11, inst=inst0 + b)[0]
            for b, (z, k1, k2) in enumerate(specs)]
    R = q.BatchRun(B, npop, G, seed=11, inst=inst0, prec=q.PREC_F64, tune=0, use_graph=graph)
    with pytest.raises(q.QpmError):
        R.set_de_shape(3, 1)
    with pytest.raises(q.QpmError):
        R.set_de_shape(1, 8)
    R.destroy()
    for ipw in (1, 2, 4):
        for passes in (1, 2, 4):
            R = q.BatchRun(B, npop, G, seed=11, inst=inst0, prec=q.PREC_F64, tune=0, use_graph=graph,
                           trials=trials)
            R.set_de_shape(ipw, passes)
            R.advance(G)
            for b in range(len(specs)):
                assert np.array_equal(R.read(b)[0].cpu().numpy(), want[b]), (ipw, passes, b)
            R.destroy()


def test_batch_uneven_designs_full_recipe_fitness(q, orc):
    # 64 instances: N ~ U[1000, 50000], width U[1.5, 3] um, dk1 = 2pi/U[18,21],
    # dk2 = 2pi/U[6.2,7]; NP = 256. The initial population's fitness in every
    # instance against the oracle on sampled genomes.
    import torch
    specs = inputs.batched_designs(64, seed=1)
    npop = 256
    B = q.precompute_phases_batched([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    R = q.BatchRun(B, npop, 2, seed=0, prec=q.PREC_F32, tune=1)
    rng = np.random.default_rng(0)
    for b in rng.choice(64, size=6, replace=False):
        z, k1, k2 = specs[b]
        x, f, _, shape = R.read(int(b))
        pick = rng.choice(npop, size=8, replace=False)
        d = orc.sign_map(x.cpu().numpy()[pick])
        _, fo = orc.Design(z, k1, k2).fitness(d)
        floor = 1e-2 * np.median(fo)
        err = np.max(np.abs(f.cpu().numpy()[pick] - fo) / np.maximum(fo, floor))
        assert err <= 1e-5, (b, err)
        # the initial genes are the oracle's initial population of instance b
        xo = orc.init_pop(npop, len(z) - 1, seed=0, inst=int(b))
        assert np.array_equal(x.cpu().numpy()[pick], xo[pick])
    best0 = [float(R.read(b)[1].max()) for b in range(64)]
    R.advance(2)
    # after two generations: every stored fitness is the oracle's fitness of
    # the stored genes (sampled), and no instance's best decreased
    for b in range(64):
        assert float(R.read(b)[1].max()) >= best0[b]
    for b in rng.choice(64, size=6, replace=False):
        z, k1, k2 = specs[b]
        x, f, _, _ = R.read(int(b))
        pick = rng.choice(npop, size=8, replace=False)
        _, fo = orc.Design(z, k1, k2).fitness(orc.sign_map(x.cpu().numpy()[pick]))
        err = np.max(np.abs(f.cpu().numpy()[pick] - fo) / np.maximum(fo, 1e-2 * np.median(fo)))
        assert err <= 1e-5, (b, err)
    R.destroy()
