"""Python binding of libqpm (include/qpm.h): the same entry points without the
`qpm_` prefix. Argument marshalling only -- every step runs in the HIP
library; there is no fallback path. Device buffers are torch CUDA tensors
(PyTorch provides device memory and streams), host buffers numpy arrays.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpm.so")

PREC_F32 = 0
PREC_F64 = 1
FIT_AUTO = 0
FIT_SEGMENTED = 1
FIT_PER_GENOME = 2
FIT_TABLE = 3
CONTROL_FIXED = 0     # F constant, a from 2 to 0
CONTROL_DECAY = 1     # F = a from 0.1 to 0.01
CONTROL_ADAPTIVE = 2  # adaptive F in [0.01, 0.1], a from 0.1 to 0.01
TRIALS_AUTO = 0      # accepted-only trial genes when the population exceeds 64 MB
TRIALS_STORE = 1     # every DE trial's genes written
TRIALS_ACCEPTED = 2  # bits only, accepted trials recomputed after selection
ALGO_HWSDA = 0  # the hybrid: DE + selection, leaders, GWO + selection
ALGO_DE = 1     # DE rand/1 alone
ALGO_GWO = 2    # the grey-wolf optimiser alone (omega wolves always move)
OBJ_SHG = 0  # multi-wavelength objective over |sum d a| / L
OBJ_THG = 1  # multi-wavelength objective over |d_eff| / L^2
# timing slots of one generation (QPM_K_*)
STEP_NAMES = ["de", "fitness_de", "finish_de", "gwo", "fitness_gwo", "finish_gwo"]

_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_U32 = C.c_uint32
_U64 = C.c_uint64
_F = C.c_float
_D = C.c_double


class QpmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("qpm error %d: %s" % (status, message))
        self.status = status


class RunConfig(C.Structure):
    _fields_ = [("np", _I64), ("generations", _I64), ("F", _F), ("CR", _F), ("seed", _U64),
                ("inst", _U32), ("prec", _I32), ("gwo_variant", _I32), ("use_graph", _I32),
                ("fit_kernel", _I32), ("tune", _I32), ("control", _I32), ("trials", _I32),
                ("algo", _I32), ("fused", _I32)]


class RunStats(C.Structure):
    _fields_ = [("best_fitness", _D), ("best_index", _I64), ("generations", _I64),
                ("fitness_evals", _I64), ("domain_evals", _D)]


_lib = None

_SIGS = {
    "qpm_status_string": (C.c_char_p, [_I32]),
    "qpm_last_error": (C.c_char_p, []),
    "qpm_precompute_phases": (_I32, [_P, _I64, _D, _D, _P, C.POINTER(_P)]),
    "qpm_design_free": (_I32, [_P]),
    "qpm_design_info": (_I32, [_P, _P, _P]),
    "qpm_design_read_phases": (_I32, [_P, _P, _P, _P]),
    "qpm_eval_fitness": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _P]),
    "qpm_eval_fitness_noalloc": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _P]),
    "qpm_eval_fitness_shape": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _I32, _P]),
    "qpm_eval_fitness_table_shape": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _I32, _P]),
    "qpm_init_population": (_I32, [_I64, _I64, _I64, _U64, _U32, _P, _P, _I64, _P]),
    "qpm_de_step": (_I32, [_P, _I64, _I64, _I64, _F, _F, _U64, _U32, _U32, _P, _P, _I64, _P]),
    "qpm_de_step_shape": (_I32, [_P, _I64, _I64, _I64, _F, _F, _U64, _U32, _U32, _P, _P, _I64, _I32, _I32, _P]),
    "qpm_gwo_step": (_I32, [_P, _I64, _I64, _I64, _P, _F, _U64, _U32, _U32, _I32, _P, _P, _I64, _P]),
    "qpm_dgwo_step": (_I32, [_P, _I64, _I64, _I64, _P, _P, _U64, _U32, _U32, _P, _P, _I64, _P]),
    "qpm_relax_forward": (_I32, [_P, _I32, _P, _I64, _I64, _P, _P, _P, _P]),
    "qpm_relax_edges_size": (_I32, [_P, _I32, _I64, _P]),
    "qpm_relax_backward": (_I32, [_P, _I32, _P, _I64, _I64, _P, _P, _P, _P, _I64, _P]),
    "qpm_run_create": (_I32, [_P, C.POINTER(RunConfig), _P, C.POINTER(_P)]),
    "qpm_run_advance": (_I32, [_P, _I64]),
    "qpm_run_read": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "qpm_run_best": (_I32, [_P, _P, _P, C.POINTER(RunStats)]),
    "qpm_run_params": (_I32, [_P, _I64, _P, _P]),
    "qpm_objective_create": (_I32, [_P, _I32, _I32, _D, _D, C.POINTER(_P)]),
    "qpm_objective_free": (_I32, [_P]),
    "qpm_eval_objective": (_I32, [_P, _I32, _P, _I64, _I64, _P, _P, _I64, _P]),
    "qpm_eval_objective_shape": (_I32, [_P, _I32, _P, _I64, _I64, _P, _P, _I64, _I32, _P]),
    "qpm_run_create_objective": (_I32, [_P, _P, _P, C.POINTER(_P)]),
    "qpm_run_destroy": (_I32, [_P]),
    "qpm_run_load": (_I32, [_P, _P, _I64]),
    "qpm_run_polish": (_I32, [_P, _I32, _F, _P]),
    "qpm_run_set_timing": (_I32, [_P, _I32]),
    "qpm_run_timing": (_I32, [_P, _P, _P, _I32]),
    "qpm_run": (_I32, [_P, C.POINTER(RunConfig), _P, _P, C.POINTER(RunStats), _P]),
    "qpm_precompute_phases_batched": (_I32, [_P, _P, _I32, _P, _P, _P, C.POINTER(_P)]),
    "qpm_batch_free": (_I32, [_P]),
    "qpm_batch_info": (_I32, [_P, _P, _P, _P]),
    "qpm_batch_eval_fitness": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _I32, _P]),
    "qpm_batch_eval_fitness_table": (_I32, [_P, _I32, _P, _I64, _I64, _P, _I32, _I32, _P]),
    "qpm_batch_run_create": (_I32, [_P, C.POINTER(RunConfig), _I32, _P, C.POINTER(_P)]),
    "qpm_batch_run_advance": (_I32, [_P, _I64]),
    "qpm_batch_run_set_timing": (_I32, [_P, _I32]),
    "qpm_batch_run_set_de_shape": (_I32, [_P, _I32, _I32]),
    "qpm_batch_run_timing": (_I32, [_P, _P, _P, _I32]),
    "qpm_batch_run_read": (_I32, [_P, _I32, _P, _I64, _P, _P, _P]),
    "qpm_batch_run_destroy": (_I32, [_P]),
}


def lib():
    """Load libqpm.so. Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqpm.so is not built (expected at %s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise QpmError(status, lib().qpm_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def words(n):
    return (n + 31) // 32


def ld_for(np_):
    return max(64, ((np_ + 63) // 64) * 64)


def ldx_for(D):
    return ((D + 63) // 64) * 64


class Design:
    """A design: device tables of the per-domain integrals."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    @property
    def handle(self):
        return self._h

    def info(self):
        n = C.c_int64()
        Cc = (C.c_double * 2)()
        _check(lib().qpm_design_info(self._h, C.byref(n), Cc))
        return int(n.value), complex(Cc[0], Cc[1])

    def read_phases(self):
        a = np.zeros(2 * self.n)
        b = np.zeros(2 * self.n)
        c = np.zeros(2 * self.n)
        _check(lib().qpm_design_read_phases(self._h, a.ctypes.data, b.ctypes.data, c.ctypes.data))
        v = lambda t: t[0::2] + 1j * t[1::2]
        return v(a), v(b), v(c)

    def free(self):
        if self._h is not None and _lib is not None:
            _lib.qpm_design_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def precompute_phases(z, dk1, dk2, stream=None):
    z = np.ascontiguousarray(z, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().qpm_precompute_phases(z.ctypes.data, len(z) - 1, float(dk1), float(dk2), _stream(stream),
                                       C.byref(h)))
    return Design(h, len(z) - 1)


def eval_fitness(design, bits, np_, prec=PREC_F32, kernel=FIT_AUTO, out=None, stream=None):
    """bits: int32 CUDA tensor (W, ld) -> fitness tensor (np_,) float32 / float64."""
    import torch
    if out is None:
        out = torch.empty(np_, dtype=torch.float64 if prec == PREC_F64 else torch.float32, device=bits.device)
    _check(lib().qpm_eval_fitness(design.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out), kernel,
                                  _stream(stream)))
    return out


class Objective:
    """The multi-wavelength objective over K designs that share their
    boundaries (kind OBJ_SHG or OBJ_THG); fitness = -h."""

    def __init__(self, designs, kind, G0=1.0, beta=0.0):
        self.designs = list(designs)  # the objective refers to their tables
        self.K = len(self.designs)
        self.n = self.designs[0].n
        self.kind = kind
        arr = (C.c_void_p * self.K)(*[d.handle for d in self.designs])
        h = C.c_void_p()
        _check(lib().qpm_objective_create(arr, self.K, kind, G0, beta, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.qpm_objective_free(self._h)
        self._h = None

    def __del__(self):
        self.free()


def eval_objective(obj, bits, np_, prec=PREC_F32, with_G=False, words_per_wave=None, stream=None):
    """bits: int32 CUDA tensor (W, ld) -> fitness (np_,) [, G (K, np_) float64]."""
    import torch
    f = torch.empty(np_, dtype=torch.float64 if prec == PREC_F64 else torch.float32, device=bits.device)
    G = torch.empty((obj.K, np_), dtype=torch.float64, device=bits.device) if with_G else None
    if words_per_wave is None:
        _check(lib().qpm_eval_objective(obj.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(f), _ptr(G), np_,
                                        _stream(stream)))
    else:
        _check(lib().qpm_eval_objective_shape(obj.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(f), _ptr(G),
                                              np_, words_per_wave, _stream(stream)))
    return (f, G) if with_G else f


def eval_fitness_noalloc(design, bits, np_, prec=PREC_F32, kernel=FIT_AUTO, out=None, stream=None):
    """eval_fitness through qpm_eval_fitness_noalloc (no device allocation in
    the library; out must be given by callers that cannot allocate)."""
    import torch
    if out is None:
        out = torch.empty(np_, dtype=torch.float64 if prec == PREC_F64 else torch.float32, device=bits.device)
    _check(lib().qpm_eval_fitness_noalloc(design.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out), kernel,
                                          _stream(stream)))
    return out


def eval_fitness_shape(design, bits, np_, prec, waves_per_group, words_per_wave, out=None, stream=None):
    """eval_fitness with an explicit segmented launch shape (tuning)."""
    import torch
    if out is None:
        out = torch.empty(np_, dtype=torch.float64 if prec == PREC_F64 else torch.float32, device=bits.device)
    _check(lib().qpm_eval_fitness_shape(design.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out),
                                        waves_per_group, words_per_wave, _stream(stream)))
    return out


def eval_fitness_table_shape(design, bits, np_, prec, groups_per_workgroup, words_per_wave, out=None, stream=None):
    """eval_fitness with the table kernel and an explicit launch shape."""
    import torch
    if out is None:
        out = torch.empty(np_, dtype=torch.float64 if prec == PREC_F64 else torch.float32, device=bits.device)
    _check(lib().qpm_eval_fitness_table_shape(design.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out),
                                              groups_per_workgroup, words_per_wave, _stream(stream)))
    return out


def init_population(np_, D, seed, inst=0, ldx=None, device="cuda", stream=None):
    import torch
    ldx = ldx_for(D) if ldx is None else ldx
    ld = ld_for(np_)
    x = torch.zeros((np_, ldx), dtype=torch.float32, device=device)
    bits = torch.zeros((words(D), ld), dtype=torch.int32, device=device)
    _check(lib().qpm_init_population(np_, D, ldx, seed, inst, _ptr(x), _ptr(bits), ld, _stream(stream)))
    return x, bits


def de_step(x, D, F, CR, seed, generation, inst=0, stream=None, shape=None):
    """x: float32 CUDA tensor (np, ldx) -> (u, u_bits). shape: optional
    (individuals_per_wave, passes) launch shape."""
    import torch
    np_, ldx = x.shape
    ld = ld_for(np_)
    u = torch.zeros_like(x)
    ub = torch.zeros((words(D), ld), dtype=torch.int32, device=x.device)
    if shape is None:
        _check(lib().qpm_de_step(_ptr(x), np_, D, ldx, F, CR, seed, generation, inst, _ptr(u), _ptr(ub), ld,
                                 _stream(stream)))
    else:
        _check(lib().qpm_de_step_shape(_ptr(x), np_, D, ldx, F, CR, seed, generation, inst, _ptr(u), _ptr(ub), ld,
                                       shape[0], shape[1], _stream(stream)))
    return u, ub


def _host_leaders(leaders, k):
    """Leader slots (a sequence, numpy array or tensor on any device) as a
    host int32 array of k entries."""
    if hasattr(leaders, "detach"):
        leaders = leaders.detach().cpu().numpy()
    L = np.ascontiguousarray(np.asarray(leaders).reshape(-1), dtype=np.int32)
    if L.size != k:
        raise ValueError("%d leader slots expected, got %d" % (k, L.size))
    return L


def gwo_step(x, D, leaders, a, seed, generation, inst=0, variant=0, stream=None):
    """x: float32 CUDA tensor (np, ldx); leaders: 3 slots (host values).
    Returns (y, y_bits); leader rows of y are a copy of x, their bit
    columns are left 0."""
    import torch
    np_, ldx = x.shape
    ld = ld_for(np_)
    y = x.clone()
    yb = torch.zeros((words(D), ld), dtype=torch.int32, device=x.device)
    L = _host_leaders(leaders, 3)
    _check(lib().qpm_gwo_step(_ptr(x), np_, D, ldx, L.ctypes.data, a, seed, generation, inst, variant, _ptr(y),
                              _ptr(yb), ld, _stream(stream)))
    return y, yb


def dgwo_step(x, D, leaders, params, seed, generation, inst=0, stream=None):
    """The discrete four-leader step. x: float32 CUDA tensor (np, ldx);
    leaders: 4 slots (host values); params: 4 floats (t, 1 - 2 eps, eps,
    lambda). Returns (y, y_bits) like gwo_step."""
    import torch
    np_, ldx = x.shape
    ld = ld_for(np_)
    y = x.clone()
    yb = torch.zeros((words(D), ld), dtype=torch.int32, device=x.device)
    par = np.ascontiguousarray(params, dtype=np.float32)
    L = _host_leaders(leaders, 4)
    _check(lib().qpm_dgwo_step(_ptr(x), np_, D, ldx, L.ctypes.data, par.ctypes.data, seed, generation, inst,
                               _ptr(y), _ptr(yb), ld, _stream(stream)))
    return y, yb


def relax_forward(design, theta, prec=PREC_F32, stream=None, keep_edges=False):
    """theta: float32 CUDA tensor (B, >= N) -> (f float32 (B,), S float64 (B, 2)),
    and with keep_edges the segment edges for relax_backward as a third value."""
    import torch
    B, ldt = theta.shape
    f = torch.empty(B, dtype=torch.float32, device=theta.device)
    S = torch.empty((B, 2), dtype=torch.float64, device=theta.device)
    E = None
    if keep_edges:
        n = C.c_int64()
        _check(lib().qpm_relax_edges_size(design.handle, prec, B, C.byref(n)))
        E = torch.empty(n.value, dtype=torch.float64, device=theta.device)
    _check(lib().qpm_relax_forward(design.handle, prec, _ptr(theta), B, ldt, _ptr(f), _ptr(S),
                                   _ptr(E) if E is not None else None, _stream(stream)))
    return (f, S, E) if keep_edges else (f, S)


def relax_backward(design, theta, S, grad_f, prec=PREC_F32, stream=None, edges=None):
    """-> grad_theta float32 (B, ldt) (entries past N are 0). edges: from
    relax_forward(..., keep_edges=True) on the same theta, or None."""
    import torch
    B, ldt = theta.shape
    g = torch.empty_like(theta) if ldt == design.n else torch.zeros_like(theta)
    gf = grad_f.to(torch.float32).contiguous()
    _check(lib().qpm_relax_backward(design.handle, prec, _ptr(theta), B, ldt, _ptr(S),
                                    _ptr(edges) if edges is not None else None, _ptr(gf), _ptr(g), ldt,
                                    _stream(stream)))
    return g


def _relax_function():
    import torch

    class QpmRelax(torch.autograd.Function):
        """f = |d_eff(tanh theta)|^2 per row, with the hand-written adjoint."""

        @staticmethod
        def forward(ctx, theta, design, prec=PREC_F32):
            theta = theta.contiguous()
            f, S, E = relax_forward(design, theta, prec, keep_edges=True)
            ctx.save_for_backward(theta, S, E)
            ctx.design = design
            ctx.prec = prec
            return f

        @staticmethod
        def backward(ctx, grad_f):
            theta, S, E = ctx.saved_tensors
            g = relax_backward(ctx.design, theta, S, grad_f, ctx.prec, edges=E)
            return g, None, None

    return QpmRelax


_QpmRelax = None


def relax(theta, design, prec=PREC_F32):
    """Differentiable f(theta) = |d_eff(tanh theta)|^2 (torch autograd)."""
    global _QpmRelax
    if _QpmRelax is None:
        _QpmRelax = _relax_function()
    return _QpmRelax.apply(theta, design, prec)


def _config(np_, generations, F=0.5, CR=0.9, seed=0, inst=0, prec=PREC_F32, gwo_variant=0, use_graph=1,
            fit_kernel=FIT_AUTO, tune=0, control=0, trials=0, algo=ALGO_HWSDA, fused=0):
    return RunConfig(np=np_, generations=generations, F=F, CR=CR, seed=seed, inst=inst, prec=prec,
                     gwo_variant=gwo_variant, use_graph=use_graph, fit_kernel=fit_kernel, tune=tune,
                     control=control, trials=trials, algo=algo, fused=fused)


class Run:
    """A whole optimisation on the device (run_create / advance / read / best).
    `design` is a Design (fitness |d_eff|^2) or an Objective (fitness -h)."""

    def __init__(self, design, np_, generations, F=0.5, CR=0.9, seed=0, inst=0, prec=PREC_F32, gwo_variant=0,
                 use_graph=1, fit_kernel=FIT_AUTO, tune=0, control=CONTROL_FIXED, trials=TRIALS_AUTO,
                 algo=ALGO_HWSDA, fused=0, stream=None):
        self.design = design
        self.cfg = _config(np_, generations, F, CR, seed, inst, prec, gwo_variant, use_graph, fit_kernel, tune,
                           control, trials, algo, fused)
        self.D = design.n
        h = C.c_void_p()
        create = lib().qpm_run_create_objective if isinstance(design, Objective) else lib().qpm_run_create
        _check(create(design.handle, C.byref(self.cfg), _stream(stream), C.byref(h)))
        self._h = h

    def advance(self, generations=1):
        _check(lib().qpm_run_advance(self._h, generations))

    def read(self, device="cuda"):
        import torch
        np_ = self.cfg.np
        x = torch.empty((np_, self.D), dtype=torch.float32, device=device)
        f = torch.empty(np_, dtype=torch.float64 if self.cfg.prec == PREC_F64 else torch.float32, device=device)
        L = (C.c_int32 * 3)()
        g = C.c_int64()
        _check(lib().qpm_run_read(self._h, _ptr(x), self.D, _ptr(f), L, C.byref(g)))
        return x, f, [L[0], L[1], L[2]], int(g.value)

    def best(self, device="cuda"):
        import torch
        bx = torch.empty(self.D, dtype=torch.float32, device=device)
        bb = torch.empty(words(self.D), dtype=torch.int32, device=device)
        st = RunStats()
        _check(lib().qpm_run_best(self._h, _ptr(bx), _ptr(bb), C.byref(st)))
        return bx, bb, st

    def load(self, x):
        """x: float32 CUDA tensor (np, >= D) -> becomes the population."""
        _check(lib().qpm_run_load(self._h, _ptr(x), x.shape[1]))

    def params(self, g):
        """(F_g, a_g) of generation g."""
        F = C.c_float()
        a = C.c_float()
        _check(lib().qpm_run_params(self._h, g, C.byref(F), C.byref(a)))
        return F.value, a.value

    def polish(self, steps=20, eta=0.05):
        """Gradient polish of the three leaders; returns how many improved."""
        acc = C.c_int32()
        _check(lib().qpm_run_polish(self._h, steps, eta, C.byref(acc)))
        return int(acc.value)

    def set_timing(self, enable=True):
        _check(lib().qpm_run_set_timing(self._h, 1 if enable else 0))

    def timing(self, reset=False):
        """-> ({step name: total ms}, timed generations)."""
        ms = (C.c_double * len(STEP_NAMES))()
        g = C.c_int64()
        _check(lib().qpm_run_timing(self._h, ms, C.byref(g), 1 if reset else 0))
        return dict(zip(STEP_NAMES, list(ms))), int(g.value)

    def destroy(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.qpm_run_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def run(design, np_, generations, F=0.5, CR=0.9, seed=0, inst=0, prec=PREC_F32, gwo_variant=0, use_graph=1,
        fit_kernel=FIT_AUTO, tune=0, control=CONTROL_FIXED, trials=TRIALS_AUTO, algo=ALGO_HWSDA, fused=0,
        stream=None, device="cuda"):
    """The one-shot run (qpm_run) -> (best genes (D,), best bits (W,), RunStats)."""
    import torch
    cfg = _config(np_, generations, F, CR, seed, inst, prec, gwo_variant, use_graph, fit_kernel, tune, control,
                  trials, algo, fused)
    bx = torch.empty(design.n, dtype=torch.float32, device=device)
    bb = torch.empty(words(design.n), dtype=torch.int32, device=device)
    st = RunStats()
    _check(lib().qpm_run(design.handle, C.byref(cfg), _ptr(bx), _ptr(bb), C.byref(st), _stream(stream)))
    return bx, bb, st


class Batch:
    """Many independent designs with concatenated device tables."""

    def __init__(self, handle, ns):
        self._h = handle
        self.ns = list(ns)
        self.n_inst = len(ns)
        self.words = [words(n) for n in ns]
        self.word_ofs = np.concatenate([[0], np.cumsum(self.words)]).astype(np.int64)

    @property
    def handle(self):
        return self._h

    def info(self):
        n = C.c_int32()
        ns = np.zeros(self.n_inst, dtype=np.int64)
        Cc = np.zeros(2 * self.n_inst)
        _check(lib().qpm_batch_info(self._h, C.byref(n), ns.ctypes.data, Cc.ctypes.data))
        return ns, Cc[0::2] + 1j * Cc[1::2]

    def free(self):
        if self._h is not None and _lib is not None:
            _lib.qpm_batch_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def precompute_phases_batched(zs, dk1s, dk2s, stream=None):
    """zs: list of boundary arrays (N_b + 1 each); dk1s, dk2s: per instance."""
    zs = [np.ascontiguousarray(z, dtype=np.float64) for z in zs]
    offsets = np.concatenate([[0], np.cumsum([len(z) for z in zs])]).astype(np.int64)
    zc = np.ascontiguousarray(np.concatenate(zs))
    d1 = np.ascontiguousarray(dk1s, dtype=np.float64)
    d2 = np.ascontiguousarray(dk2s, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().qpm_precompute_phases_batched(zc.ctypes.data, offsets.ctypes.data, len(zs), d1.ctypes.data,
                                               d2.ctypes.data, _stream(stream), C.byref(h)))
    return Batch(h, [len(z) - 1 for z in zs])


def batch_eval_fitness(batch, bits, np_, prec=PREC_F32, waves_per_group=0, words_per_wave=0, out=None,
                       stream=None):
    """bits: int32 CUDA tensor (sum W_b, ld) -> fitness (n_inst, np_)."""
    import torch
    if out is None:
        out = torch.empty((batch.n_inst, np_), dtype=torch.float64 if prec == PREC_F64 else torch.float32,
                          device=bits.device)
    _check(lib().qpm_batch_eval_fitness(batch.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out),
                                        waves_per_group, words_per_wave, _stream(stream)))
    return out


def batch_eval_fitness_table(batch, bits, np_, prec, groups_per_workgroup, words_per_wave, out=None, stream=None):
    """batch_eval_fitness with the table kernel and an explicit shape."""
    import torch
    if out is None:
        out = torch.empty((batch.n_inst, np_), dtype=torch.float64 if prec == PREC_F64 else torch.float32,
                          device=bits.device)
    _check(lib().qpm_batch_eval_fitness_table(batch.handle, prec, _ptr(bits), np_, bits.shape[1], _ptr(out),
                                              groups_per_workgroup, words_per_wave, _stream(stream)))
    return out


class BatchRun:
    """One HWSDA run per instance of a Batch, advanced together."""

    def __init__(self, batch, np_, generations, F=0.5, CR=0.9, seed=0, inst=0, prec=PREC_F32, gwo_variant=0,
                 use_graph=1, tune=1, trials=TRIALS_AUTO, stream=None):
        self.batch = batch
        self.cfg = _config(np_, generations, F, CR, seed, inst, prec, gwo_variant, use_graph, FIT_AUTO,
                           trials=trials)
        h = C.c_void_p()
        _check(lib().qpm_batch_run_create(batch.handle, C.byref(self.cfg), 1 if tune else 0, _stream(stream),
                                          C.byref(h)))
        self._h = h

    def advance(self, generations=1):
        _check(lib().qpm_batch_run_advance(self._h, generations))

    def read(self, inst, device="cuda"):
        import torch
        n = self.batch.ns[inst]
        np_ = self.cfg.np
        x = torch.empty((np_, n), dtype=torch.float32, device=device)
        f = torch.empty(np_, dtype=torch.float64 if self.cfg.prec == PREC_F64 else torch.float32, device=device)
        L = (C.c_int32 * 3)()
        shape = (C.c_int32 * 2)()
        _check(lib().qpm_batch_run_read(self._h, inst, _ptr(x), n, _ptr(f), L, shape))
        return x, f, [L[0], L[1], L[2]], (shape[0], shape[1])

    def set_timing(self, enable=True):
        _check(lib().qpm_batch_run_set_timing(self._h, 1 if enable else 0))

    def set_de_shape(self, individuals_per_wave, passes):
        _check(lib().qpm_batch_run_set_de_shape(self._h, individuals_per_wave, passes))

    def timing(self, reset=False):
        ms = (C.c_double * len(STEP_NAMES))()
        g = C.c_int64()
        _check(lib().qpm_batch_run_timing(self._h, ms, C.byref(g), 1 if reset else 0))
        return dict(zip(STEP_NAMES, list(ms))), int(g.value)

    def destroy(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.qpm_batch_run_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
