"""Pins of the oracle's two comparison optimisers (DE alone, paper Sec.
2.2.1; GWO alone, Sec. 2.2.2; compared with HWSDA in Tables 3-7) and of its
gradient polish (the relaxation used to refine +-1 designs; not in the
paper), against invariants of the stated rules and mathematical properties
of the ascent, not against the oracle itself."""
import numpy as np
import pytest

from paper_2511_01255_amd import inputs

DK1 = inputs.DK1
DK2 = inputs.DK2


def _design(orc, n):
    return orc.Design(inputs.uniform_boundaries(n), DK1, DK2)


# ---------------------------------------------------------------- DE alone

def test_de_alone_is_de_steps_with_greedy_selection(orc):
    # two generations of algo 1 equal the DE trials and the strict greedy
    # selection chained by hand, with no grey-wolf step in between
    n, np_, G = 40, 8, 2
    D = _design(orc, n)
    x1, f1, _, par = D.run_algo(np_, G, 0.5, 0.9, seed=3, algo=1)
    x = orc.init_pop(np_, n, seed=3)
    _, f = D.fitness(orc.sign_map(x))
    for g in range(G):
        u, _ = orc.de_step(x, 0.5, 0.9, seed=3, g=g)
        _, fu = D.fitness(orc.sign_map(u))
        acc = fu > f
        x[acc] = u[acc]
        f[acc] = fu[acc]
    assert np.array_equal(x, x1) and np.array_equal(f, f1)
    assert np.all(par[:, 0] == np.float32(0.5))


def test_de_alone_slots_never_get_worse(orc):
    # greedy one-to-one selection: every slot's fitness is monotone, so one
    # more generation of the same run can only raise each slot
    n, np_ = 48, 12
    D = _design(orc, n)
    _, f5, tr, _ = D.run_algo(np_, 5, 0.5, 0.9, seed=7, algo=1)
    _, f6, _, _ = D.run_algo(np_, 6, 0.5, 0.9, seed=7, algo=1)
    # the schedule's length changes nothing for DE with the fixed control
    assert np.all(f6 >= f5)
    assert np.all(np.diff(tr) >= 0)


def test_de_alone_ties_keep_the_target(orc):
    # one domain: every genome has the same f, so no trial is ever accepted
    D = orc.Design(np.array([0.0, 2.0]), DK1, DK2)
    x, f, _, _ = D.run_algo(6, 4, 0.5, 0.9, seed=4, algo=1)
    assert np.array_equal(x, orc.init_pop(6, 1, seed=4))


@pytest.mark.slow
def test_de_alone_reaches_bruteforce_optimum(orc):
    n = 10
    D = _design(orc, n)
    _, fb, _ = D.bruteforce()
    hits = 0
    for seed in range(6):
        _, f, _, _ = D.run_algo(32, 80, 0.5, 0.9, seed, algo=1)
        hits += abs(f.max() - fb) <= 1e-12 * fb
    assert hits >= 4


# ---------------------------------------------------------------- GWO alone

def test_gwo_alone_is_gwo_steps_without_selection(orc):
    # two generations of algo 2: leaders from the sorted fitness, every other
    # wolf takes its candidate whatever its fitness, leaders stay
    n, np_, G = 40, 8, 2
    D = _design(orc, n)
    x1, f1, _, _ = D.run_algo(np_, G, 0.5, 0.9, seed=5, algo=2)
    x = orc.init_pop(np_, n, seed=5)
    _, f = D.fitness(orc.sign_map(x))
    for g in range(G):
        L = orc.top3(f)
        y = orc.gwo_step(x, L, orc.a_schedule(g, G), seed=5, g=g)
        _, fy = D.fitness(orc.sign_map(y))
        keep = np.zeros(np_, dtype=bool)
        keep[L] = True
        x[~keep] = y[~keep]
        f[~keep] = fy[~keep]
    assert np.array_equal(x, x1) and np.array_equal(f, f1)


def test_gwo_alone_moves_without_selection_and_keeps_leaders(orc):
    # a wolf may get worse (no greedy selection), the leaders' rows do not
    # change, so the best never falls
    n, np_, G = 64, 16, 12
    D = _design(orc, n)
    worse = 0
    for seed in range(3):
        xs, fs = [], []
        for g in range(G + 1):
            if g == 0:
                x0 = orc.init_pop(np_, n, seed=seed)
                xs.append(x0)
                fs.append(D.fitness(orc.sign_map(x0))[1])
                continue
            # the run truncated after g generations of a G-generation schedule
            # is not what run_algo gives (a_g depends on G), so chain the steps
            L = orc.top3(fs[-1])
            y = orc.gwo_step(xs[-1], L, orc.a_schedule(g - 1, G), seed=seed, g=g - 1)
            _, fy = D.fitness(orc.sign_map(y))
            x = xs[-1].copy()
            f = fs[-1].copy()
            keep = np.zeros(np_, dtype=bool)
            keep[L] = True
            x[~keep] = y[~keep]
            f[~keep] = fy[~keep]
            assert np.array_equal(x[L], xs[-1][L])
            assert f.max() >= fs[-1].max()
            worse += int(np.sum(f[~keep] < fs[-1][~keep]))
            xs.append(x)
            fs.append(f)
        xr, fr, tr, _ = D.run_algo(np_, G, 0.5, 0.9, seed, algo=2)
        assert np.array_equal(xr, xs[-1]) and np.array_equal(fr, fs[-1])
        assert np.all(np.diff(tr) >= 0)
    # under greedy selection this count would be 0
    assert worse > 0


def test_algo_zero_is_hwsda(orc):
    n, np_, G = 40, 8, 3
    D = _design(orc, n)
    for control in (0, 1, 2):
        xa, fa, ta, pa = D.run_algo(np_, G, 0.5, 0.9, seed=2, algo=0, control=control)
        xh, fh, th, ph = D.hwsda_run(np_, G, 0.5, 0.9, seed=2, control=control)
        assert np.array_equal(xa, xh) and np.array_equal(fa, fh) and np.array_equal(pa, ph)


def test_algo_rejects_unknown(orc):
    D = _design(orc, 8)
    for algo in (-1, 3):
        with pytest.raises(ValueError):
            D.run_algo(8, 2, 0.5, 0.9, seed=0, algo=algo)


# ---------------------------------------------------------------- gradient polish

def _theta_rows(orc, n, rows, seed):
    # genes in [-1, 1) as a run holds them
    return orc.init_pop(rows, n, seed=seed)


def test_polish_without_steps_is_the_identity(orc):
    n = 200
    D = _design(orc, n)
    x = _theta_rows(orc, n, 3, seed=1)
    _, f0 = D.fitness(orc.sign_map(x))
    for steps, eta in ((0, 0.05), (5, 0.0)):
        th, f1, acc = D.polish(x, f0, steps, eta)
        assert np.array_equal(th, x.astype(np.float64))
        assert np.array_equal(f1, f0)
        assert not acc.any()  # strictly better is needed


def test_polish_step_length_is_eta(orc):
    # theta moves by eta in its largest coordinate, in no coordinate more
    n = 300
    D = _design(orc, n)
    x = _theta_rows(orc, n, 3, seed=2)
    _, f0 = D.fitness(orc.sign_map(x))
    for eta in (1e-3, 0.05, 0.7):
        th, _, _ = D.polish(x, f0, 1, eta)
        step = np.max(np.abs(th - x.astype(np.float64)), axis=1)
        assert np.allclose(step, eta, rtol=1e-12, atol=0)


def test_polish_is_first_order_ascent(orc):
    # for a small step the relaxed fitness rises by eta |g|_2^2 / |g|_inf
    # to first order: checks the direction, the sign and the normalisation
    n = 400
    D = _design(orc, n)
    x = _theta_rows(orc, n, 3, seed=3)
    _, f0 = D.fitness(orc.sign_map(x))
    x64 = x.astype(np.float64)
    _, fr0, g = D.relax(x64)
    eta = 1e-5
    th, _, _ = D.polish(x, f0, 1, eta)
    _, fr1, _ = D.relax(th)
    pred = eta * np.sum(g * g, axis=1) / np.max(np.abs(g), axis=1)
    assert np.all(fr1 > fr0)
    assert np.max(np.abs((fr1 - fr0) - pred) / pred) < 1e-3


def test_polish_small_steps_raise_the_relaxed_fitness(orc):
    n = 256
    D = _design(orc, n)
    x = _theta_rows(orc, n, 3, seed=4)
    _, f0 = D.fitness(orc.sign_map(x))
    prev = D.relax(x.astype(np.float64), grad=False)[1]
    for k in range(1, 6):
        th, _, _ = D.polish(x, f0, k, 2e-3)
        cur = D.relax(th, grad=False)[1]
        assert np.all(cur > prev)
        prev = cur


def test_polish_scores_the_signs_of_theta_and_accepts_strictly(orc):
    n = 320
    D = _design(orc, n)
    x = _theta_rows(orc, n, 3, seed=5)
    _, f0 = D.fitness(orc.sign_map(x))
    th, f1, acc = D.polish(x, f0, 20, 0.05)
    d = np.where(th < 0.0, -1, 1).astype(np.int8)
    _, fd = D.fitness(d)
    assert np.array_equal(f1, fd)
    assert np.array_equal(acc, f1 > f0)
    # the same rows with f0 equal to the polished value are not accepted,
    # one ulp below they are
    _, _, acc_eq = D.polish(x, f1, 20, 0.05)
    assert not acc_eq.any()
    _, _, acc_lo = D.polish(x, np.nextafter(f1, -np.inf), 20, 0.05)
    assert acc_lo.all()


def test_polish_saturated_rows_do_not_move(orc):
    # |theta| = 40: tanh is exactly +-1 in long double, so the gradient is
    # exactly zero and no step is taken
    n = 64
    D = _design(orc, n)
    s = orc.sign_map(_theta_rows(orc, n, 1, seed=6)).astype(np.float32)
    x = 40.0 * s
    _, f0 = D.fitness(s.astype(np.int8))
    th, f1, acc = D.polish(x, f0, 3, 0.05)
    assert np.array_equal(th, x.astype(np.float64))
    assert np.array_equal(f1, f0) and not acc.any()
