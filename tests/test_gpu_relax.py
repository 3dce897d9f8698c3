"""Parity of the relaxation d = tanh(theta) and its hand-written adjoint with
the CPU oracle: forward values, the analytic gradient, FP64 central finite
differences (h = 1e-6) on sampled coordinates, the torch autograd path, and
the +-1 corners."""
import numpy as np
import pytest

from paper_2511_01255_amd import inputs

pytestmark = pytest.mark.gpu

DK1, DK2 = inputs.DK1, inputs.DK2


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_01255_amd import qpm
    qpm.lib()
    return qpm


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# (B, N, widths): one ragged segment, ragged segments and rows, one domain,
# fewer domains than a sub-segment; rows of more than 256 segments (the
# combine's waves then take several rounds of 64 segments each: 5 rounds at
# N = 7 x 10^4, 19 at N = 3 x 10^5)
CASES = [(3, 120, "jitter"), (70, 5003, "uniform"), (1, 1, "uniform"), (65, 37, "jitter"),
         (3, 70000, "uniform"), (2, 300001, "jitter")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "B%d_n%d_%s" % c)
@pytest.mark.parametrize("prec", [1, 0])
def test_relax_forward_and_gradient_match_oracle(q, orc, case, prec):
    B, n, kind = case
    z = inputs.jittered_boundaries(n, 2.0, 0.3, seed=2) if kind == "jitter" else inputs.uniform_boundaries(n)
    theta = inputs.relax_theta(B, n, seed=n)
    D = q.precompute_phases(z, DK1, DK2)
    O = orc.Design(z, DK1, DK2)
    th = _t(theta)
    f, S_dev = q.relax_forward(D, th, prec)
    So, fo, go = O.relax(theta.astype(np.float64))
    f = f.double().cpu().numpy()
    S = S_dev.cpu().numpy()
    floor = 1e-2 * np.median(fo)
    # f is returned in float32; S (double) carries the FP64 accuracy
    assert np.max(np.abs(f - fo) / np.maximum(fo, floor)) <= (1e-6 if prec == 1 else 1e-5)
    Sc = S[:, 0] + 1j * S[:, 1]
    assert np.max(np.abs(Sc - So) / np.maximum(np.abs(So), np.sqrt(floor))) <= (1e-12 if prec == 1 else 1e-5)
    gf = np.random.default_rng(1).uniform(0.5, 1.5, B).astype(np.float32)
    g = q.relax_backward(D, th, S_dev, _t(gf), prec).cpu().numpy()
    want = go * gf[:, None].astype(np.float64)
    scale = np.maximum(np.max(np.abs(want), axis=1, keepdims=True), 1e-300)
    err = np.max(np.abs(g - want) / scale)
    # FP64: only the float32 output rounding; FP32: blocked FP32 scans
    assert err <= (1e-6 if prec == 1 else 1e-4), err


@pytest.mark.parametrize("prec", [1, 0])
def test_relax_gradient_vs_finite_differences_full_size(q, orc, prec):
    # N = 5 x 10^4 domains x 2 um, batch 256, theta ~ N(0, 1); central FP64
    # differences (h = 1e-6) of the oracle on 64 sampled coordinates
    B, n = 256, 50000
    z = inputs.uniform_boundaries(n, 2.0)
    theta = inputs.relax_theta(B, n, seed=5)
    D = q.precompute_phases(z, DK1, DK2)
    O = orc.Design(z, DK1, DK2)
    th = _t(theta)
    f, S = q.relax_forward(D, th, prec)
    g = q.relax_backward(D, th, S, _t(np.ones(B, np.float32)), prec).cpu().numpy()
    rng = np.random.default_rng(17)
    rows = rng.integers(0, B, 64)
    cols = rng.integers(0, n, 64)
    h = 1e-6
    fd = np.empty(64)
    for k, (b, c) in enumerate(zip(rows, cols)):
        tp = theta[b].astype(np.float64)
        tm = tp.copy()
        tp[c] += h
        tm[c] -= h
        _, fpm, _ = O.relax(np.stack([tp, tm]), grad=False)
        fd[k] = (fpm[0] - fpm[1]) / (2 * h)
    # normwise over the sampled rows' full gradients
    _, _, go = O.relax(theta[np.unique(rows)].astype(np.float64))
    scale = np.max(np.abs(go))
    got = g[rows, cols]
    assert np.max(np.abs(got - fd)) <= (1e-5 if prec == 1 else 1e-4) * scale, np.max(np.abs(got - fd)) / scale
    ref = {b: i for i, b in enumerate(np.unique(rows))}
    an = np.array([go[ref[b], c] for b, c in zip(rows, cols)])
    assert np.max(np.abs(got - an)) <= (1e-6 if prec == 1 else 1e-4) * scale
    fo = O.relax(theta[:8].astype(np.float64), grad=False)[1]
    assert np.max(np.abs(f[:8].double().cpu().numpy() - fo) / fo) <= (1e-6 if prec == 1 else 1e-5)


@pytest.mark.parametrize("prec", [1, 0])
def test_relax_saved_edges_equal_recomputed(q, prec):
    # the adjoint from the forward call's saved edges is bit-identical to
    # the adjoint that recomputes them (ragged B and N, unaligned ldt)
    for B, n, ldt in ((5, 4099, 4099), (67, 2048, 2052), (1, 3, 3), (2, 300001, 300003)):
        D = q.precompute_phases(inputs.jittered_boundaries(n, 2.0, 0.3, seed=n), DK1, DK2)
        th = _t(np.pad(inputs.relax_theta(B, n, seed=B), ((0, 0), (0, ldt - n))))
        f1, S1, E = q.relax_forward(D, th, prec, keep_edges=True)
        f2, S2 = q.relax_forward(D, th, prec)
        assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy()) and np.array_equal(S1.cpu().numpy(), S2.cpu().numpy())
        gf = _t(np.linspace(0.5, 1.5, B))
        g1 = q.relax_backward(D, th, S1, gf, prec, edges=E).cpu().numpy()
        g2 = q.relax_backward(D, th, S1, gf, prec).cpu().numpy()
        assert np.array_equal(g1, g2)
        assert not np.any(g1[:, n:])


def test_relax_autograd_function(q):
    import torch
    n, B = 777, 9
    D = q.precompute_phases(inputs.jittered_boundaries(n, 2.0, 0.2, seed=3), DK1, DK2)
    th = _t(inputs.relax_theta(B, n, seed=3)).requires_grad_(True)
    w = torch.linspace(0.5, 1.5, B, device="cuda")
    f = q.relax(th, D, q.PREC_F64)
    (f * w).sum().backward()
    _, S = q.relax_forward(D, th.detach(), q.PREC_F64)
    g = q.relax_backward(D, th.detach(), S, w, q.PREC_F64)
    assert torch.equal(th.grad, g)


def test_relax_corners_equal_pm1_fitness(q):
    n, B = 2049, 40
    z = inputs.uniform_boundaries(n, 2.0)
    d = inputs.random_signs(B, n, seed=8)
    D = q.precompute_phases(z, DK1, DK2)
    f, _ = q.relax_forward(D, _t(40.0 * d), q.PREC_F64)
    import torch
    bits = torch.from_numpy(inputs.pack_bits(d).view(np.int32)).cuda()
    fp = q.eval_fitness(D, bits, B, prec=q.PREC_F64).cpu().numpy()
    assert np.max(np.abs(f.double().cpu().numpy() - fp) / fp) <= 1e-6  # f is returned in float32


@pytest.mark.parametrize("prec", [1, 0])
def test_run_polish_of_leaders(q, prec):
    # polish never lowers a leader, touches nothing else, replaces a leader
    # only by genes whose exact +-1 fitness is higher, and is deterministic
    n, npop = 2000, 64
    D = q.precompute_phases(inputs.uniform_boundaries(n, 2.0), DK1, DK2)
    results = []
    for rep in range(2):
        R = q.Run(D, npop, 10, seed=2, prec=prec)
        R.advance(3)
        x0, f0, L, _ = R.read()
        acc = R.polish(20, 0.05)
        x1, f1, L1, _ = R.read()
        x0, f0, x1, f1 = (t.cpu().numpy() for t in (x0, f0, x1, f1))
        others = np.setdiff1d(np.arange(npop), L)
        assert np.array_equal(x1[others], x0[others]) and np.array_equal(f1[others], f0[others])
        changed = [k for k in L if not np.array_equal(x1[k], x0[k])]
        assert len(changed) == acc and 0 <= acc <= 3
        for k in L:
            assert f1[k] >= f0[k]
        for k in changed:
            assert f1[k] > f0[k] and np.all(np.abs(x1[k]) <= 1.0)
            import torch
            bits = torch.from_numpy(inputs.pack_bits(np.where(x1[k] < 0, -1, 1)[None].astype(np.int8))
                                    .view(np.int32)).cuda()
            fe = q.eval_fitness(D, bits, 1, prec=prec).double().cpu().numpy()[0]
            assert abs(fe - f1[k]) <= (1e-12 if prec == 1 else 1e-6) * fe
        R.advance(2)  # the run continues after a polish
        results.append((x1, f1, acc))
        R.destroy()
    assert np.array_equal(results[0][0], results[1][0]) and results[0][2] == results[1][2]


@pytest.mark.parametrize("prec", [1, 0])
def test_run_polish_then_continue_same_for_both_trial_storages(q, orc, prec):
    # a polish changes leader rows (and so the buffer flags the DE step
    # reads); the run that continues afterwards must take the same decisions
    # whether it stores every trial or only the accepted ones, and every
    # stored fitness must be the oracle's fitness of the stored genes
    n, npop = 1500, 96
    z = inputs.uniform_boundaries(n, 2.0)
    D = q.precompute_phases(z, DK1, DK2)
    out = []
    for trials in (q.TRIALS_STORE, q.TRIALS_ACCEPTED):
        R = q.Run(D, npop, 12, seed=5, prec=prec, trials=trials)
        R.advance(4)
        R.polish(20, 0.05)
        R.advance(5)
        x, f, L, _ = R.read()
        out.append((x.cpu().numpy(), f.double().cpu().numpy(), L))
        R.destroy()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]
    _, fo = orc.Design(z, DK1, DK2).fitness(orc.sign_map(out[0][0]))
    tol = 1e-12 if prec == 1 else 1e-5
    assert np.max(np.abs(out[0][1] - fo) / np.maximum(fo, 1e-2 * np.median(fo))) <= tol
