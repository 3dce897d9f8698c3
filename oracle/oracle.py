"""ctypes wrappers over liboracle.so (test infrastructure only).

Every function here marshals numpy arrays into the plain-C oracle; no
arithmetic of the method lives in this file.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_P = C.c_void_p
_I64 = C.c_int64
_U64 = C.c_uint64
_U32 = C.c_uint32
_F = C.c_float
_D = C.c_double
_INT = C.c_int


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def lib():
    """Load liboracle.so, building it first only when it does not exist."""
    global _lib
    if _lib is None:
        path = os.environ.get("QPM_ORACLE_LIB")  # a planted-mistake copy in mutation tests
        if not path:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = C.CDLL(path)
        sig = {
            "orc_num_threads": (_INT, []),
            "orc_set_num_threads": (None, [_INT]),
            "orc_gl_rule": (None, [_INT, _P, _P]),
            "orc_G": (None, [_D, _D, _D, _P]),
            "orc_G_quad": (None, [_D, _D, _D, _P]),
            "orc_design_create": (_P, [_P, _I64, _D, _D]),
            "orc_design_free": (None, [_P]),
            "orc_design_n": (_I64, [_P]),
            "orc_design_phases": (None, [_P, _P, _P, _P, _P]),
            "orc_fitness": (None, [_P, _P, _I64, _P, _P]),
            "orc_fitness_pairs": (None, [_P, _P, _I64, _P, _P]),
            "orc_fitness_quad": (_INT, [_P, _I64, _D, _D, _P, _P]),
            "orc_bruteforce": (_INT, [_P, _P, _P, _P]),
            "orc_relax": (None, [_P, _P, _I64, _P, _P, _P]),
            "orc_philox": (None, [_P, _P, _P]),
            "orc_sign_map": (None, [_P, _I64, _P]),
            "orc_init_pop": (None, [_I64, _I64, _U64, _U32, _P]),
            "orc_de_step": (None, [_P, _I64, _I64, _F, _F, _U64, _U32, _U32, _P, _P]),
            "orc_gwo_step": (None, [_P, _I64, _I64, _P, _F, _U64, _U32, _U32, _INT, _P]),
            "orc_top3": (None, [_P, _I64, _P]),
            "orc_top4": (None, [_P, _I64, _P]),
            "orc_dgwo_params": (None, [_I64, _I64, _P]),
            "orc_dgwo_step": (None, [_P, _I64, _I64, _P, _P, _U64, _U32, _U32, _P]),
            "orc_a_schedule": (_F, [_I64, _I64]),
            "orc_hwsda_run": (_INT, [_P, _I64, _I64, _F, _F, _U64, _U32, _INT, _P, _P, _P]),
            "orc_hwsda_run_ctl": (_INT, [_P, _I64, _I64, _F, _F, _U64, _U32, _INT, _INT, _P, _P, _P, _P]),
            "orc_a_control": (_F, [_INT, _I64, _I64]),
            "orc_multi_objective": (_INT, [_P, _INT, _INT, _D, _D, _P, _I64, _P, _P]),
            "orc_hwsda_run_obj": (_INT, [_P, _INT, _INT, _D, _D, _I64, _I64, _F, _F, _U64, _U32, _INT, _INT, _P,
                                         _P, _P, _P]),
            "orc_adaptive_F": (_F, [_P, _I64, _I64, _I64]),
            "orc_run_algo": (_INT, [_P, _I64, _I64, _F, _F, _U64, _U32, _INT, _INT, _INT, _P, _P, _P, _P]),
            "orc_run_obj_algo": (_INT, [_P, _INT, _INT, _D, _D, _I64, _I64, _F, _F, _U64, _U32, _INT, _INT, _INT,
                                        _P, _P, _P, _P]),
            "orc_polish": (None, [_P, _P, _I64, _P, _INT, _D, _P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def gl_rule(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gl_rule(n, _ptr(x), _ptr(w))
    return x, w


def G(k1, k2, w, quad=False):
    out = np.zeros(2)
    (lib().orc_G_quad if quad else lib().orc_G)(k1, k2, w, _ptr(out))
    return complex(out[0], out[1])


class Design:
    """Boundaries z[0..N] (strictly increasing), dk1, dk2 -> oracle design."""

    def __init__(self, z, dk1, dk2):
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.n = len(self.z) - 1
        self.dk1 = float(dk1)
        self.dk2 = float(dk2)
        self._h = lib().orc_design_create(_ptr(self.z), self.n, self.dk1, self.dk2)
        if not self._h:
            raise ValueError("invalid design")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_design_free(h)
            self._h = None

    def phases(self):
        a = np.zeros(2 * self.n)
        b = np.zeros(2 * self.n)
        c = np.zeros(2 * self.n)
        Cc = np.zeros(2)
        lib().orc_design_phases(self._h, _ptr(a), _ptr(b), _ptr(c), _ptr(Cc))
        v = lambda t: t[0::2] + 1j * t[1::2]
        return v(a), v(b), v(c), complex(Cc[0], Cc[1])

    def fitness(self, d):
        """d: (np, n) of +-1 -> (S complex128 (np,), f float64 (np,))."""
        d = np.ascontiguousarray(d, dtype=np.int8).reshape(-1, self.n)
        npop = d.shape[0]
        S = np.zeros(2 * npop)
        f = np.zeros(npop)
        lib().orc_fitness(self._h, _ptr(d), npop, _ptr(S), _ptr(f))
        return S[0::2] + 1j * S[1::2], f

    def fitness_pairs(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, self.n)
        npop = d.shape[0]
        S = np.zeros(2 * npop)
        f = np.zeros(npop)
        lib().orc_fitness_pairs(self._h, _ptr(d), npop, _ptr(S), _ptr(f))
        return S[0::2] + 1j * S[1::2], f

    def bruteforce(self):
        d = np.zeros(self.n, dtype=np.int8)
        fb = np.zeros(1)
        fs = np.zeros(1)
        if lib().orc_bruteforce(self._h, _ptr(d), _ptr(fb), _ptr(fs)) != 0:
            raise ValueError("bruteforce needs 1 <= n <= 26")
        return d, float(fb[0]), float(fs[0])

    def relax(self, theta, grad=True):
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, self.n)
        B = theta.shape[0]
        S = np.zeros(2 * B)
        f = np.zeros(B)
        g = np.zeros((B, self.n)) if grad else None
        lib().orc_relax(self._h, _ptr(theta), B, _ptr(S), _ptr(f), _ptr(g))
        return S[0::2] + 1j * S[1::2], f, g

    def run_algo(self, np_, G, F, CR, seed, algo, inst=0, variant=0, control=0):
        """The loop with algo 0 (HWSDA), 1 (DE alone) or 2 (GWO alone) ->
        (x, f, best trace, (G, 2) float32 rows (F_g, a_g))."""
        x = np.zeros((np_, self.n), dtype=np.float32)
        f = np.zeros(np_)
        tr = np.zeros(G)
        par = np.zeros((G, 2), dtype=np.float32)
        rc = lib().orc_run_algo(self._h, np_, G, F, CR, seed, inst, variant, control, algo, _ptr(x), _ptr(f),
                                _ptr(tr), _ptr(par))
        if rc != 0:
            raise ValueError("invalid run arguments")
        return x, f, tr, par

    def polish(self, x, f0, steps=20, eta=0.05):
        """Gradient polish of gene rows x (rows, n) float32 whose exact
        fitness is f0 -> (theta (rows, n) float64, f1 (rows,), accept
        (rows,) bool)."""
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, self.n)
        rows = x.shape[0]
        f0 = np.ascontiguousarray(f0, dtype=np.float64).reshape(rows)
        th = np.zeros((rows, self.n))
        f1 = np.zeros(rows)
        acc = np.zeros(rows, dtype=np.int32)
        lib().orc_polish(self._h, _ptr(x), rows, _ptr(f0), int(steps), float(eta), _ptr(th), _ptr(f1), _ptr(acc))
        return th, f1, acc.astype(bool)

    def hwsda_run(self, np_, G, F, CR, seed, inst=0, variant=0, trace=True, control=None):
        """control None: the plain entry point (textbook parameters);
        0, 1, 2: the parameter control, returning also (G, 2) float32 rows
        (F_g, a_g)."""
        x = np.zeros((np_, self.n), dtype=np.float32)
        f = np.zeros(np_)
        tr = np.zeros(G) if trace else None
        if control is None:
            rc = lib().orc_hwsda_run(self._h, np_, G, F, CR, seed, inst, variant, _ptr(x), _ptr(f), _ptr(tr))
            if rc != 0:
                raise ValueError("invalid run arguments")
            return x, f, tr
        par = np.zeros((G, 2), dtype=np.float32)
        rc = lib().orc_hwsda_run_ctl(self._h, np_, G, F, CR, seed, inst, variant, control, _ptr(x), _ptr(f),
                                     _ptr(tr), _ptr(par))
        if rc != 0:
            raise ValueError("invalid run arguments")
        return x, f, tr, par


class Objective:
    """The multi-wavelength objective over K oracle designs that share
    their boundaries: kind 0 = SHG, 1 = THG (f = -h, maximised)."""

    def __init__(self, designs, kind, G0, beta):
        self.designs = list(designs)  # keeps the designs alive
        self.K = len(self.designs)
        self.n = self.designs[0].n
        self.kind, self.G0, self.beta = int(kind), float(G0), float(beta)
        self._arr = (C.c_void_p * self.K)(*[d._h for d in self.designs])

    def __call__(self, d):
        """d: (np, n) of +-1 -> (G (np, K), f (np,))."""
        d = np.ascontiguousarray(d, dtype=np.int8).reshape(-1, self.n)
        npop = d.shape[0]
        G = np.zeros((npop, self.K))
        f = np.zeros(npop)
        rc = lib().orc_multi_objective(self._arr, self.K, self.kind, self.G0, self.beta, _ptr(d), npop, _ptr(G),
                                       _ptr(f))
        if rc != 0:
            raise ValueError("designs differ in their boundaries, or bad arguments")
        return G, f

    def hwsda_run(self, np_, G, F, CR, seed, inst=0, variant=0, control=0, algo=0):
        x = np.zeros((np_, self.n), dtype=np.float32)
        f = np.zeros(np_)
        tr = np.zeros(G)
        par = np.zeros((G, 2), dtype=np.float32)
        rc = lib().orc_run_obj_algo(self._arr, self.K, self.kind, self.G0, self.beta, np_, G, F, CR, seed, inst,
                                    variant, control, algo, _ptr(x), _ptr(f), _ptr(tr), _ptr(par))
        if rc != 0:
            raise ValueError("invalid run arguments")
        return x, f, tr, par


def fitness_quad(z, dk1, dk2, d):
    z = np.ascontiguousarray(z, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.int8)
    S = np.zeros(2)
    if lib().orc_fitness_quad(_ptr(z), len(z) - 1, dk1, dk2, _ptr(d), _ptr(S)) != 0:
        raise ValueError("bad input")
    return complex(S[0], S[1])


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def sign_map(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    d = np.zeros(x.shape, dtype=np.int8)
    lib().orc_sign_map(_ptr(x), x.size, _ptr(d))
    return d


def init_pop(np_, D, seed, inst=0):
    x = np.zeros((np_, D), dtype=np.float32)
    lib().orc_init_pop(np_, D, seed, inst, _ptr(x))
    return x


def de_step(x, F, CR, seed, g, inst=0):
    x = np.ascontiguousarray(x, dtype=np.float32)
    np_, D = x.shape
    u = np.zeros_like(x)
    idx = np.zeros((np_, 4), dtype=np.int32)
    lib().orc_de_step(_ptr(x), np_, D, F, CR, seed, g, inst, _ptr(u), _ptr(idx))
    return u, idx


def gwo_step(x, leaders, a, seed, g, inst=0, variant=0):
    x = np.ascontiguousarray(x, dtype=np.float32)
    np_, D = x.shape
    L = np.ascontiguousarray(leaders, dtype=np.int32)
    y = np.zeros_like(x)
    lib().orc_gwo_step(_ptr(x), np_, D, _ptr(L), a, seed, g, inst, variant, _ptr(y))
    return y


def top4(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(4, dtype=np.int32)
    lib().orc_top4(_ptr(f), f.size, _ptr(out))
    return out


def dgwo_params(g, G):
    par = np.zeros(4, dtype=np.float32)
    lib().orc_dgwo_params(g, G, _ptr(par))
    return par


def dgwo_step(x, leaders4, par, seed, g, inst=0):
    x = np.ascontiguousarray(x, dtype=np.float32)
    np_, D = x.shape
    L = np.ascontiguousarray(leaders4, dtype=np.int32)
    pr = np.ascontiguousarray(par, dtype=np.float32)
    y = np.zeros_like(x)
    lib().orc_dgwo_step(_ptr(x), np_, D, _ptr(L), _ptr(pr), seed, g, inst, _ptr(y))
    return y


def top3(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(3, dtype=np.int32)
    lib().orc_top3(_ptr(f), len(f), _ptr(out))
    return out


def a_schedule(g, G):
    return lib().orc_a_schedule(g, G)


def a_control(control, g, G):
    return lib().orc_a_control(control, g, G)


def adaptive_F(f, g, G):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_adaptive_F(_ptr(f), f.size, g, G)
