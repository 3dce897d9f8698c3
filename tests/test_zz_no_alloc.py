"""qpm_eval_fitness_noalloc (fixed device scratch, no allocation) against
qpm_eval_fitness through the C ABI: the same launch plan, so the same bits,
and both within the fitness tolerance of the oracle; two calls in a row,
the second on a smaller population, and the size limit."""
import ctypes as C

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


def _call_noalloc(q, D, bits, npop, prec, kernel, out):
    import torch
    st = q.lib().qpm_eval_fitness_noalloc(D.handle, prec, C.c_void_p(bits.data_ptr()), npop, bits.shape[1],
                                          C.c_void_p(out.data_ptr()), kernel,
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("prec,kernel", [(0, 0), (1, 0), (0, 1), (1, 1), (1, 2), (0, 3), (1, 3)])
def test_noalloc_equals_fitness_on_two_calls(q, orc, prec, kernel):
    import torch
    cases = [(3001, 300, 5), (1000, 70, 6)]  # the second call is smaller
    for n, npop, seed in cases:
        z = inputs.jittered_boundaries(n, 2.0, 0.2, seed=seed)
        d = inputs.fitness_population(npop, n, 2.0, n_periodic=npop // 5, seed=seed)
        D = q.precompute_phases(z, DK1, DK2)
        bits = torch.from_numpy(inputs.pack_bits(d).view(np.int32)).cuda()
        dt = torch.float64 if prec == 1 else torch.float32
        ref = q.eval_fitness(D, bits, npop, prec=prec, kernel=kernel)
        out = torch.full((npop,), -1.0, dtype=dt, device="cuda")
        assert _call_noalloc(q, D, bits, npop, prec, kernel, out) == 0, q.lib().qpm_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, npop)
        _, fo = orc.Design(z, DK1, DK2).fitness(d)
        f = out.double().cpu().numpy()
        err = np.abs(f - fo) / np.maximum(fo, 1e-2 * np.median(fo))
        assert err.max() <= TOL[prec], (n, npop, err.max())


def test_noalloc_rejects_a_population_beyond_its_scratch(q):
    import torch
    # 8192 genomes x 10^5 domains: about 40 MB of segment partials > 16 MiB
    n, npop = 100000, 8192
    D = q.precompute_phases(inputs.uniform_boundaries(n, 2.0), DK1, DK2)
    bits = torch.zeros((inputs.words(n), npop), dtype=torch.int32, device="cuda")
    out = torch.empty(npop, dtype=torch.float32, device="cuda")
    assert _call_noalloc(q, D, bits, npop, 0, 0, out) == -2
    assert b"16 MiB" in q.lib().qpm_last_error() or b"scratch" in q.lib().qpm_last_error()
