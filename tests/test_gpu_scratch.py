"""The evaluation entry points keep their device scratch with the design or
objective between calls (one buffer per stream, each use ordered after the
previous one by an event). These tests call them through the C ABI with
growing and shrinking populations, interleaved on several streams, and on
more streams than the handle keeps buffers for, and check every result
against the oracle (tolerance) and against a lone call (bit for bit: the
launch shape depends on the sizes only, so the arithmetic is the same)."""
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


def _bits(d):
    import torch
    return torch.from_numpy(inputs.pack_bits(d).view(np.int32)).cuda()


def _pops(n, sizes, seed):
    return [inputs.random_signs(m, n, seed=seed + k) for k, m in enumerate(sizes)]


@pytest.mark.parametrize("prec", [0, 1])
def test_fitness_scratch_grows_and_shrinks(q, orc, prec):
    n = 2500
    z = inputs.jittered_boundaries(n, 2.0, 0.3, seed=4)
    D = q.precompute_phases(z, DK1, DK2)
    O = orc.Design(z, DK1, DK2)
    tol = 1e-5 if prec == 0 else 1e-12
    # small, large (the buffer grows), small again (it is reused), large
    for d in _pops(n, [70, 1100, 5, 1100, 300], seed=10):
        f = q.eval_fitness(D, _bits(d), d.shape[0], prec).double().cpu().numpy()
        _, fo = O.fitness(d)
        assert np.max(np.abs(f - fo) / np.maximum(fo, 1e-2 * np.median(fo))) <= tol


@pytest.mark.parametrize("nstreams", [2, 6])
def test_fitness_interleaved_streams(q, nstreams):
    # 6 streams: four take the handle's buffers, two take the allocator
    import torch
    n = 3001
    D = q.precompute_phases(inputs.uniform_boundaries(n, 2.0), DK1, DK2)
    sizes = [64 * (k + 1) + 3 for k in range(nstreams)]
    pops = _pops(n, sizes, seed=20)
    bits = [_bits(d) for d in pops]
    ref = [q.eval_fitness(D, b, m, q.PREC_F32).clone() for b, m in zip(bits, sizes)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    outs = [[] for _ in range(nstreams)]
    for rep in range(8):
        for k, s in enumerate(streams):
            with torch.cuda.stream(s):
                o = torch.empty(sizes[k], dtype=torch.float32, device="cuda")
                q.eval_fitness(D, bits[k], sizes[k], q.PREC_F32, out=o)
                outs[k].append(o)
    torch.cuda.synchronize()
    for k in range(nstreams):
        for o in outs[k]:
            assert torch.equal(o, ref[k])


def test_objective_scratch_across_streams(q, orc):
    import torch
    n, K = 1537, 3
    z = inputs.jittered_boundaries(n, 2.0, 0.3, seed=7)
    dks = [(DK1, DK2), (0.31, 0.97), (0.335, 0.93)]
    O = q.Objective([q.precompute_phases(z, a, b) for a, b in dks[:K]], q.OBJ_THG, 0.6, 1.5)
    Oo = orc.Objective([orc.Design(z, a, b) for a, b in dks[:K]], q.OBJ_THG, 0.6, 1.5)
    pops = _pops(n, [40, 300, 7], seed=30)
    streams = [torch.cuda.Stream() for _ in pops]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    res = []
    for rep in range(3):
        for d, s in zip(pops, streams):
            with torch.cuda.stream(s):
                res.append((d, q.eval_objective(O, _bits(d), d.shape[0], 1)))
    torch.cuda.synchronize()
    for d, f in res:
        _, fo = Oo(d)
        assert np.max(np.abs(f.cpu().numpy() - fo)) <= 1e-12 * max(1.0, np.max(np.abs(fo)))


def test_relax_scratch_reused(q, orc):
    # forward then backward without saved edges (both use the scratch), at
    # two batch sizes, against the oracle's FP64 relaxation
    import torch
    n = 700
    z = inputs.uniform_boundaries(n, 2.0)
    D = q.precompute_phases(z, DK1, DK2)
    O = orc.Design(z, DK1, DK2)
    rng = np.random.default_rng(3)
    for B in (5, 70, 5):
        th = rng.standard_normal((B, n)).astype(np.float32)
        t = torch.from_numpy(th).cuda()
        f, S = q.relax_forward(D, t, prec=q.PREC_F64)
        g = q.relax_backward(D, t, S, torch.ones(B, dtype=torch.float32, device="cuda"), prec=q.PREC_F64)
        _, fo, go = O.relax(th.astype(np.float64))
        assert np.max(np.abs(f.double().cpu().numpy() - fo) / np.abs(fo)) <= 1e-6
        gn = g.double().cpu().numpy()
        assert np.max(np.abs(gn - go)) <= 1e-5 * np.max(np.abs(go))
