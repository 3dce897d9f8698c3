"""The C-ABI library loads, exports every entry point include/qpm.h declares,
and rejects invalid arguments on the host before touching a device (these
tests run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(qpm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2511_01255_amd import qpm
    return qpm.lib()


def test_header_declares_the_core_entry_points():
    names = _declared()
    for n in ["qpm_precompute_phases", "qpm_eval_fitness", "qpm_de_step", "qpm_gwo_step", "qpm_run"]:
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for n in _declared():
        assert hasattr(L, n), n


def test_hip_symbol_versions_are_in_the_loaded_runtime():
    # the library runs inside a process whose HIP runtime is the one torch
    # ships: every versioned HIP symbol it needs must exist in that runtime
    import shutil
    import subprocess

    import torch
    from paper_2511_01255_amd import qpm
    rt = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    if not (os.path.exists(rt) and shutil.which("nm") and shutil.which("objdump")):
        pytest.skip("no torch HIP runtime or binutils here")
    need = set(re.findall(r"@(hip_[0-9.]+)", subprocess.run(
        ["nm", "-D", "--undefined-only", qpm.LIB_PATH], capture_output=True, text=True, check=True).stdout))
    have = set(re.findall(r"\b(hip_[0-9.]+)\b", subprocess.run(
        ["objdump", "-T", rt], capture_output=True, text=True, check=True).stdout))
    assert need and need <= have, sorted(need - have)


def test_status_strings(L):
    for code in range(0, -6, -1):
        assert L.qpm_status_string(code)
    assert L.qpm_status_string(-99) == b"unknown status"


def _err(L):
    return L.qpm_last_error().decode()


def test_precompute_rejects_bad_boundaries(L):
    h = C.c_void_p()
    assert L.qpm_precompute_phases(None, 4, 0.1, 0.2, None, C.byref(h)) == -1
    z = np.array([0.0, 1.0, 1.0, 2.0])
    assert L.qpm_precompute_phases(z.ctypes.data, 3, 0.1, 0.2, None, C.byref(h)) == -1
    assert "strictly increasing" in _err(L)
    z = np.array([0.0, 1.0, np.nan])
    assert L.qpm_precompute_phases(z.ctypes.data, 2, 0.1, 0.2, None, C.byref(h)) == -1
    z = np.array([0.0, 1.0])
    assert L.qpm_precompute_phases(z.ctypes.data, 1, float("inf"), 0.2, None, C.byref(h)) == -1
    assert L.qpm_precompute_phases(z.ctypes.data, 0, 0.1, 0.2, None, C.byref(h)) == -1
    assert L.qpm_precompute_phases(z.ctypes.data, 1 << 28, 0.1, 0.2, None, C.byref(h)) == -2
    assert h.value is None  # nothing written on error


def test_fitness_rejects_bad_arguments(L):
    fake = C.c_void_p(0x10000)  # never dereferenced: validation fails first
    assert L.qpm_eval_fitness(None, 0, fake, 4, 64, fake, 0, None) == -1
    assert L.qpm_eval_fitness(fake, 7, fake, 4, 64, fake, 0, None) == -1
    assert "precision" in _err(L)
    assert L.qpm_eval_fitness(fake, 0, fake, 4, 64, fake, 2, None) == -1  # per-genome is FP64 only
    assert L.qpm_eval_fitness(fake, 1, fake, 0, 64, fake, 0, None) == -1
    assert L.qpm_eval_fitness(fake, 1, fake, 65, 64, fake, 0, None) == -1
    assert L.qpm_eval_fitness(fake, 1, fake, 10, 96, fake, 0, None) == -1
    assert "multiple of 64" in _err(L)
    assert L.qpm_eval_fitness(fake, 1, fake, 10, 64, fake, 9, None) == -1


def test_de_and_gwo_reject_bad_arguments(L):
    x = C.c_void_p(0x10000)
    u = C.c_void_p(0x20000000)
    b = C.c_void_p(0x30000000)

    def de(np_=8, D=10, ldx=12, F=0.5, CR=0.9, xx=x, uu=u, bb=b, ld=64):
        return L.qpm_de_step(xx, np_, D, ldx, C.c_float(F), C.c_float(CR), 0, 0, 0, uu, bb, ld, None)

    # every call below fails validation before any device work
    assert de(np_=3) == -1 and "np >= 4" in _err(L)
    assert de(F=2.5) == -1 and "F must be" in _err(L)
    assert de(CR=-0.1) == -1
    assert de(ldx=10) == -1 and "ldx" in _err(L)
    assert de(ld=32) == -1
    assert de(xx=C.c_void_p(0x10004)) == -1 and "aligned" in _err(L)
    assert de(uu=x) == -1 and "overlap" in _err(L)
    assert de(bb=None) == -1

    def de_shape(ipw, passes, np_=3):
        return L.qpm_de_step_shape(x, np_, 10, 12, C.c_float(0.5), C.c_float(0.9), 0, 0, 0, u, b, 64, ipw, passes,
                                   None)

    assert de_shape(3, 1) == -1 and "individuals_per_wave" in _err(L)
    assert de_shape(1, 3) == -1 and "passes" in _err(L)
    assert de_shape(2, 2) == -1 and "np >= 4" in _err(L)  # a valid shape goes on to the usual checks

    def gwo(np_=8, D=10, ldx=12, a=1.0, variant=0, leaders=(0, 1, 2)):
        lead = None if leaders is None else C.cast((C.c_int32 * 3)(*leaders), C.c_void_p)
        return L.qpm_gwo_step(x, np_, D, ldx, lead, C.c_float(a), 0, 0, 0, variant, u, b, 64, None)

    assert gwo(np_=3) == -1
    assert gwo(a=-1.0) == -1
    assert gwo(a=1e-35) == -1 and "2^-100" in _err(L)
    assert gwo(variant=2) == -1
    assert gwo(leaders=None) == -1
    # the leaders are host values, checked before any launch
    assert gwo(leaders=(0, 1, 8)) == -1 and "outside" in _err(L)
    assert gwo(leaders=(-1, 1, 2)) == -1 and "outside" in _err(L)
    assert gwo(leaders=(3, 1, 3)) == -1 and "distinct" in _err(L)


def test_run_rejects_bad_config(L):
    from paper_2511_01255_amd import qpm
    fake = C.c_void_p(0x10000)
    h = C.c_void_p()
    for kw in [dict(np_=3, generations=10), dict(np_=8, generations=0), dict(np_=8, generations=5, F=3.0),
               dict(np_=8, generations=5, CR=2.0), dict(np_=8, generations=5, prec=5),
               dict(np_=8, generations=5, gwo_variant=3)]:
        cfg = qpm._config(**kw)
        assert L.qpm_run_create(fake, C.byref(cfg), None, C.byref(h)) == -1
    assert h.value is None
    assert L.qpm_run_advance(None, 1) == -1


def test_run_rejects_unknown_control_and_trial_storage(L):
    from paper_2511_01255_amd import qpm
    fake = C.c_void_p(0x10000)
    h = C.c_void_p()
    for kw in [dict(control=3), dict(control=-1), dict(trials=3), dict(trials=-1)]:
        cfg = qpm._config(8, 5, **kw)
        assert L.qpm_run_create(fake, C.byref(cfg), None, C.byref(h)) == -1
        assert ("control" in _err(L)) or ("trial" in _err(L))
    # unknown optimiser; the accepted-only trial storage belongs to the hybrid
    for kw, word in [(dict(algo=3), "algorithm"), (dict(algo=-1), "algorithm"),
                     (dict(algo=1, trials=2), "accepted-only"), (dict(algo=2, trials=2), "accepted-only")]:
        cfg = qpm._config(8, 5, **kw)
        assert L.qpm_run_create(fake, C.byref(cfg), None, C.byref(h)) == -1
        assert word in _err(L)
    # batched runs apply the hybrid only: DE or GWO alone is not supported there
    for algo in (1, 2):
        cfg = qpm._config(8, 5, algo=algo)
        assert L.qpm_batch_run_create(fake, C.byref(cfg), 0, None, C.byref(h)) == -5
        assert "hybrid" in _err(L)
    # the adaptive control is not offered on a multi-wavelength objective
    cfg = qpm._config(8, 5, control=2)
    assert L.qpm_run_create_objective(fake, C.byref(cfg), None, C.byref(h)) == -1
    assert "adaptive" in _err(L)
    assert h.value is None


def test_discrete_gwo_and_objective_reject_bad_arguments(L):
    x = C.c_void_p(0x10000)
    y = C.c_void_p(0x20000)
    b = C.c_void_p(0x30000)
    lead = C.cast((C.c_int32 * 4)(0, 1, 2, 3), C.c_void_p)
    par = C.cast((C.c_float * 4)(0.5, 0.8, 0.1, 0.1), C.c_void_p)
    bad = C.cast((C.c_float * 4)(0.5, float("nan"), 0.1, 0.1), C.c_void_p)
    assert L.qpm_dgwo_step(x, 3, 10, 12, lead, par, 0, 0, 0, y, b, 64, None) == -1
    assert L.qpm_dgwo_step(x, 8, 10, 12, None, par, 0, 0, 0, y, b, 64, None) == -1
    assert L.qpm_dgwo_step(x, 8, 10, 12, lead, None, 0, 0, 0, y, b, 64, None) == -1
    assert L.qpm_dgwo_step(x, 8, 10, 12, lead, bad, 0, 0, 0, y, b, 64, None) == -1 and "finite" in _err(L)
    for bad_lead in ((0, 1, 2, 8), (0, 1, 2, 2)):
        bl = C.cast((C.c_int32 * 4)(*bad_lead), C.c_void_p)
        assert L.qpm_dgwo_step(x, 8, 10, 12, bl, par, 0, 0, 0, y, b, 64, None) == -1
        assert "outside" in _err(L) or "distinct" in _err(L)
    h = C.c_void_p()
    designs = (C.c_void_p * 9)(*([0x10000] * 9))
    assert L.qpm_objective_create(None, 1, 0, 1.0, 0.0, C.byref(h)) == -1
    assert L.qpm_objective_create(designs, 0, 0, 1.0, 0.0, C.byref(h)) == -1
    assert L.qpm_objective_create(designs, 9, 0, 1.0, 0.0, C.byref(h)) == -1 and "K must be" in _err(L)
    assert L.qpm_objective_create(designs, 2, 2, 1.0, 0.0, C.byref(h)) == -1 and "kind" in _err(L)
    assert L.qpm_objective_create(designs, 2, 1, float("inf"), 0.0, C.byref(h)) == -1
    assert h.value is None
    assert L.qpm_eval_objective(None, 0, b, 4, 64, y, None, 0, None) == -1
    assert L.qpm_objective_free(None) == 0


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
