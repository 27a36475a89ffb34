"""Python binding of the MI355X implicit M1 radiation step (libm1.so, C ABI in include/m1.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libm1.so.  PyTorch provides device memory and the stream.  If the library has
not been built this module raises on import -- there is no CPU fallback.

Low level: ``m1_setup``, ``m1_linearize``, ``m1_apply_operator``,
``m1_precondition``, ``m1_residual``, ``m1_implicit_step``, ``m1_explicit_step``,
``m1_semi_implicit_step``, ``m1_velocity_sources``, ``m1_time_steps_noalloc``, ``m1_destroy``,
``m1_last_error``, ``m1_profile_enable``, ``m1_profile_query`` mirror the C
functions one to one (pointers are passed as Python ints / ctypes structs).
High level: :class:`Solver` builds the structs from a problem description.
"""
from __future__ import annotations

import ctypes
import os

# torch is imported first so that libm1.so binds to the HIP runtime torch has
# loaded: device pointers and streams from torch are only valid in that runtime.
import torch as _torch_module  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libm1.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_13926_amd.build` "
                      "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------
# enums and structs (must match include/m1.h)
# ---------------------------------------------------------------------------
M1_OK, M1_NOT_CONVERGED, M1_NOT_ADMISSIBLE = 0, 1, 2
M1_ERR_INVALID_ARG, M1_ERR_OUT_OF_MEMORY, M1_ERR_HIP, M1_ERR_NONFINITE, M1_ERR_STATE = -1, -2, -3, -4, -5
SOURCE = {"none": 0, "absorption": 1, "coupled_t": 2}
FLUX_SOURCE = {"wb": 0, "centered": 1}
CLOSURE = {"m1": 0, "p1": 1}
LINEARIZATION = {"newton": 0, "picard": 1}
BC = {"periodic": 0, "outflow": 1, "dirichlet": 2, "reflect": 3}
PRECISION = {"fp64": 0, "mixed": 1}
PC = {"bj": 0, "none": 1, "learned": 2, "mg": 3}


class M1Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("newton_flags", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double), ("c", ctypes.c_double), ("a_r", ctypes.c_double),
        ("source", ctypes.c_int32), ("flux_source", ctypes.c_int32), ("closure", ctypes.c_int32),
        ("ap_correction", ctypes.c_int32), ("lambda_floor", ctypes.c_double), ("bc", ctypes.c_int32 * 6),
        ("linearization", ctypes.c_int32), ("precision", ctypes.c_int32), ("pc", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("newton_max", ctypes.c_int32),
        ("fixed_iters", ctypes.c_int32), ("basis_fp32", ctypes.c_int32), ("rtol", ctypes.c_double),
        ("newton_rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("ptc_psi0", ctypes.c_double),
        ("ptc_rtol", ctypes.c_double), ("positivity_clip", ctypes.c_double), ("newton_forcing", ctypes.c_double),
        ("nn_weights_path", ctypes.c_char_p),
        ("mg_omega", ctypes.c_double), ("mg_nu1", ctypes.c_int32), ("mg_nu2", ctypes.c_int32),
        ("mg_nmin", ctypes.c_int32), ("wb_boundary", ctypes.c_int32), ("mg_nu1_coarse", ctypes.c_int32),
        ("mg_nu2_coarse", ctypes.c_int32),
    ]


class M1State(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("F", ctypes.c_void_p * 3), ("T", ctypes.c_void_p)]


class M1Fields(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_void_p), ("rho_cv", ctypes.c_void_p),
                ("bc_ghost", ctypes.c_void_p * 6), ("bc_mask", ctypes.c_void_p * 6)]


class M1Stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("krylov_iters", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("fell_back", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("nonlinear_residual", ctypes.c_double),
                ("cells_f_gt_1", ctypes.c_int64), ("cells_e_nonpos", ctypes.c_int64), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_sig = {
    "m1_config_size": (ctypes.c_size_t, []),
    "m1_stats_size": (ctypes.c_size_t, []),
    "m1_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "m1_setup": (ctypes.c_int32, [_P(M1Config), _P(M1Fields), _P(M1State), _P(M1State), ctypes.c_double, _vp,
                                  _P(_vp)]),
    "m1_linearize": (ctypes.c_int32, [_vp, _P(M1State), _P(M1State), ctypes.c_double]),
    "m1_apply_operator": (ctypes.c_int32, [_vp, _vp, _vp]),
    "m1_precondition": (ctypes.c_int32, [_vp, _vp, _vp]),
    "m1_residual": (ctypes.c_int32, [_vp, _vp]),
    "m1_implicit_step": (ctypes.c_int32, [_vp, _P(M1State), ctypes.c_double, _P(M1Stats)]),
    "m1_explicit_step": (ctypes.c_int32, [_vp, _P(M1State), ctypes.c_double, ctypes.c_int32, _P(M1Stats)]),
    "m1_semi_implicit_step": (ctypes.c_int32, [_vp, _P(M1State), ctypes.c_double, ctypes.c_int32, _P(M1Stats)]),
    "m1_velocity_sources": (ctypes.c_int32, [_vp, _P(M1State), _vp, _vp, _vp, ctypes.c_double, _P(M1Stats)]),
    "m1_time_steps_noalloc": (ctypes.c_int32, [_P(M1Config), _P(M1Fields), _P(M1State), ctypes.c_double,
                                               ctypes.c_int32, ctypes.c_int32, _vp, _P(M1Stats)]),
    "m1_destroy": (None, [_vp]),
    "m1_last_error": (ctypes.c_char_p, [_vp]),
    "m1_profile_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "m1_profile_query": (ctypes.c_int32, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_double),
                                          _P(ctypes.c_double)]),
    "m1_profile_issued": (ctypes.c_int32, [_vp, ctypes.c_int32, _P(ctypes.c_int64)]),
    "m1_kernel_class_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "m1_kernel_class_count": (ctypes.c_int32, []),
    "m1_set_network": (ctypes.c_int32, [_vp, _vp]),
    "m1_nn_features": (ctypes.c_int32, [_vp, _vp, _vp]),
    "m1_nn_target": (ctypes.c_int32, [_vp, _vp, _vp, _vp]),
    "m1_solve_linear": (ctypes.c_int32, [_vp, _vp, _vp, _P(M1Stats)]),
    "m1nn_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_int32),
                                     ctypes.c_int32, ctypes.c_int32, _vp, _P(_vp)]),
    "m1nn_param_count": (ctypes.c_int64, [_vp]),
    "m1nn_set_params": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64]),
    "m1nn_get_params": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64]),
    "m1nn_init_params": (ctypes.c_int32, [_vp, ctypes.c_uint64, ctypes.c_float]),
    "m1nn_get_grads": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64]),
    "m1nn_forward": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp]),
    "m1nn_backward": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double)]),
    "m1nn_adam_step": (ctypes.c_int32, [_vp, ctypes.c_float]),
    "m1nn_train_step": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                         _P(ctypes.c_double)]),
    "m1nn_save": (ctypes.c_int32, [_vp, ctypes.c_char_p]),
    "m1nn_load": (ctypes.c_int32, [_vp, ctypes.c_char_p]),
    "m1nn_destroy": (None, [_vp]),
    "m1nn_last_error": (ctypes.c_char_p, [_vp]),
}
EXPORTED = tuple(_sig)
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

if _lib.m1_config_size() != ctypes.sizeof(M1Config) or _lib.m1_stats_size() != ctypes.sizeof(M1Stats):
    raise ImportError("libm1.so ABI mismatch with the Python structs")

# thin one-to-one wrappers ---------------------------------------------------
m1_setup = _lib.m1_setup
m1_linearize = _lib.m1_linearize
m1_apply_operator = _lib.m1_apply_operator
m1_precondition = _lib.m1_precondition
m1_residual = _lib.m1_residual
m1_implicit_step = _lib.m1_implicit_step
m1_explicit_step = _lib.m1_explicit_step
m1_semi_implicit_step = _lib.m1_semi_implicit_step
m1_velocity_sources = _lib.m1_velocity_sources
m1_time_steps_noalloc = _lib.m1_time_steps_noalloc
m1_destroy = _lib.m1_destroy
m1_last_error = _lib.m1_last_error
m1_profile_enable = _lib.m1_profile_enable
m1_profile_query = _lib.m1_profile_query
m1_profile_issued = _lib.m1_profile_issued
m1_kernel_class_name = _lib.m1_kernel_class_name
m1_kernel_class_count = _lib.m1_kernel_class_count
m1_status_string = _lib.m1_status_string
m1_set_network = _lib.m1_set_network
m1_nn_features = _lib.m1_nn_features
m1_nn_target = _lib.m1_nn_target
m1_solve_linear = _lib.m1_solve_linear
m1nn_create = _lib.m1nn_create
m1nn_param_count = _lib.m1nn_param_count
m1nn_set_params = _lib.m1nn_set_params
m1nn_get_params = _lib.m1nn_get_params
m1nn_init_params = _lib.m1nn_init_params
m1nn_get_grads = _lib.m1nn_get_grads
m1nn_forward = _lib.m1nn_forward
m1nn_backward = _lib.m1nn_backward
m1nn_adam_step = _lib.m1nn_adam_step
m1nn_train_step = _lib.m1nn_train_step
m1nn_save = _lib.m1nn_save
m1nn_load = _lib.m1nn_load
m1nn_destroy = _lib.m1nn_destroy
m1nn_last_error = _lib.m1nn_last_error


class M1Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.m1_status_string(status).decode()}: {msg}")
        self.status = status


def kernel_classes():
    return [_lib.m1_kernel_class_name(k).decode() for k in range(_lib.m1_kernel_class_count())]


# ---------------------------------------------------------------------------
# high-level wrapper
# ---------------------------------------------------------------------------
def make_config(p, *, precision="fp64", pc="bj", restart=30, max_iters=20000, newton_max=20, fixed_iters=0,
                rtol=1e-10, newton_rtol=None, inner_rtol=1e-6, basis_fp32=False, line_search=False,
                ptc_psi0=0.0, ptc_rtol=0.0, positivity_clip=0.0, newton_forcing=0.0, mg_omega=0.7, mg_nu1=1,
                mg_nu2=1, mg_nmin=0, mg_nu1_coarse=-1, mg_nu2_coarse=-1, commit_nonadmissible=False):
    """m1_config from a problem description (the dict layout of ``workloads``)."""
    cfg = M1Config()
    cfg.ndim = p["ndim"]
    cfg.newton_flags = (1 if line_search else 0) | (2 if commit_nonadmissible else 0)
    for d in range(3):
        cfg.n[d] = p["n"][d] if d < p["ndim"] else 1
    cfg.dx, cfg.c, cfg.a_r = p["dx"], p["c"], p["a_r"]
    cfg.source = SOURCE[p["source"]]
    cfg.flux_source = FLUX_SOURCE[p["flux_source"]]
    cfg.closure = CLOSURE[p.get("closure", "m1")]
    cfg.ap_correction = 1 if p["ap"] else 0
    cfg.lambda_floor = p["lambda_floor"]
    for f in range(6):
        cfg.bc[f] = BC[p["bc"][f]] if f < 2 * p["ndim"] else 0
    cfg.linearization = LINEARIZATION[p.get("linearization", "newton")]
    cfg.precision = PRECISION[precision]
    cfg.pc = PC[pc]
    cfg.restart, cfg.max_iters, cfg.newton_max, cfg.fixed_iters = restart, max_iters, newton_max, fixed_iters
    cfg.basis_fp32 = 1 if basis_fp32 else 0
    cfg.rtol = rtol
    cfg.newton_rtol = rtol if newton_rtol is None else newton_rtol
    cfg.inner_rtol = inner_rtol
    cfg.ptc_psi0, cfg.ptc_rtol, cfg.positivity_clip = ptc_psi0, ptc_rtol, positivity_clip
    cfg.newton_forcing = newton_forcing
    cfg.nn_weights_path = None
    cfg.mg_omega, cfg.mg_nu1, cfg.mg_nu2, cfg.mg_nmin = mg_omega, mg_nu1, mg_nu2, mg_nmin
    cfg.wb_boundary = 1 if p.get("wb_boundary", False) else 0
    cfg.mg_nu1_coarse, cfg.mg_nu2_coarse = mg_nu1_coarse, mg_nu2_coarse
    return cfg


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the M1 library runs on a GPU; none is visible")
    return torch


def state_struct(U, ndim, coupled):
    """m1_state pointing into a component-major (n_u, *grid) float64 CUDA tensor."""
    s = M1State()
    s.E = U[0].data_ptr()
    for d in range(3):
        s.F[d] = U[1 + d].data_ptr() if d < ndim else None
    s.T = U[1 + ndim].data_ptr() if coupled else None
    return s


class Solver:
    """Owns an m1_ctx and the device copies of a problem's fields.

    ``p``: problem dict (``workloads``); keyword options go to :func:`make_config`.
    ``U_lin``/``U_n``: optional (n_u, *grid) arrays to linearise at immediately.
    """

    def __init__(self, p, *, U_lin=None, U_n=None, dt=None, device="cuda", **opts):
        torch = _torch()
        self.torch = torch
        self.p = p
        self.ndim = p["ndim"]
        self.coupled = p["source"] == "coupled_t"
        self.nu = 1 + self.ndim + (1 if self.coupled else 0)
        self.shape = tuple(reversed(p["n"]))
        self.N = 1
        for v in p["n"]:
            self.N *= int(v)
        self.device = torch.device(device)
        self.cfg = make_config(p, **opts)
        dev = lambda a: torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
        self._keep = []
        self.fields = M1Fields()
        sig = dev(p["sigma"])
        self._keep.append(sig)
        self.fields.sigma = sig.data_ptr()
        if self.coupled:
            rc = dev(p["rho_cv"])
            self._keep.append(rc)
            self.fields.rho_cv = rc.data_ptr()
        for f in range(6):
            if f < 2 * self.ndim and p["bc"][f] == "dirichlet":
                g = dev(p["ghost"][f])
                self._keep.append(g)
                self.fields.bc_ghost[f] = g.data_ptr()
                if f in p.get("ghost_mask", {}):
                    m = dev(p["ghost_mask"][f])
                    self._keep.append(m)
                    self.fields.bc_mask[f] = m.data_ptr()
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        sl = sn = None
        if U_lin is not None:
            self._Ul = self.to_device(U_lin)
            self._Un = self.to_device(U_n)
            sl = ctypes.byref(state_struct(self._Ul, self.ndim, self.coupled))
            sn = ctypes.byref(state_struct(self._Un, self.ndim, self.coupled))
        st = _lib.m1_setup(ctypes.byref(self.cfg), ctypes.byref(self.fields), sl, sn,
                           float(dt if dt is not None else p["dt"]), ctypes.c_void_p(self.stream.cuda_stream),
                           ctypes.byref(ctx))
        if st != M1_OK:
            raise M1Error(st, _lib.m1_last_error(None).decode())
        self.ctx = ctx

    # -- helpers ------------------------------------------------------------
    def to_device(self, U):
        t = self.torch.as_tensor(U, dtype=self.torch.float64).to(self.device)
        return t.reshape((self.nu,) + self.shape).contiguous()

    def _check(self, st):
        if st not in (M1_OK,):
            raise M1Error(st, _lib.m1_last_error(self.ctx).decode())

    def vector(self):
        return self.torch.zeros((self.nu,) + self.shape, dtype=self.torch.float64, device=self.device)

    # -- one-to-one calls -------------------------------------------------------
    def linearize(self, U_lin, U_n, dt=None):
        self._Ul = self.to_device(U_lin)
        self._Un = self.to_device(U_n)
        self._check(_lib.m1_linearize(self.ctx, ctypes.byref(state_struct(self._Ul, self.ndim, self.coupled)),
                                      ctypes.byref(state_struct(self._Un, self.ndim, self.coupled)),
                                      float(dt if dt is not None else self.p["dt"])))

    def apply_operator(self, x):
        x = self.to_device(x)
        y = self.vector()
        self._check(_lib.m1_apply_operator(self.ctx, x.data_ptr(), y.data_ptr()))
        return y

    def precondition(self, r):
        r = self.to_device(r)
        z = self.vector()
        self._check(_lib.m1_precondition(self.ctx, r.data_ptr(), z.data_ptr()))
        return z

    def residual(self):
        R = self.vector()
        self._check(_lib.m1_residual(self.ctx, R.data_ptr()))
        return R

    def implicit_step(self, U, dt=None, *, raise_on_fail=True):
        """Advance the device tensor U (n_u, *grid) in place; returns (status, stats dict)."""
        stats = M1Stats()
        st = _lib.m1_implicit_step(self.ctx, ctypes.byref(state_struct(U, self.ndim, self.coupled)),
                                   float(dt if dt is not None else self.p["dt"]), ctypes.byref(stats))
        if raise_on_fail and st not in (M1_OK,):
            raise M1Error(st, _lib.m1_last_error(self.ctx).decode())
        return st, stats.as_dict()

    def _time_step(self, fn, U, dt, nsteps, raise_on_fail):
        stats = M1Stats()
        st = fn(self.ctx, ctypes.byref(state_struct(U, self.ndim, self.coupled)),
                float(dt if dt is not None else self.p["dt"]), int(nsteps), ctypes.byref(stats))
        if raise_on_fail and st != M1_OK:
            raise M1Error(st, _lib.m1_last_error(self.ctx).decode())
        return st, stats.as_dict()

    def explicit_step(self, U, dt=None, nsteps=1, *, raise_on_fail=True):
        """nsteps forward-Euler steps of the device tensor U in place; returns (status, stats dict)."""
        return self._time_step(_lib.m1_explicit_step, U, dt, nsteps, raise_on_fail)

    def semi_implicit_step(self, U, dt=None, nsteps=1, *, raise_on_fail=True):
        """nsteps semi-implicit steps (sources implicit, fluxes explicit) of U in place (centred flux source)."""
        return self._time_step(_lib.m1_semi_implicit_step, U, dt, nsteps, raise_on_fail)

    def velocity_sources(self, U, u, dt=None, *, raise_on_fail=True):
        """Add the velocity-dependent sources to U in place; u: device tensor (ndim, *grid)."""
        u = self.torch.as_tensor(u, dtype=self.torch.float64).to(self.device)
        u = u.reshape((self.ndim,) + self.shape).contiguous()
        ptr = [u[m].data_ptr() for m in range(self.ndim)] + [None] * (3 - self.ndim)
        stats = M1Stats()
        st = _lib.m1_velocity_sources(self.ctx, ctypes.byref(state_struct(U, self.ndim, self.coupled)), ptr[0],
                                      ptr[1], ptr[2], float(dt if dt is not None else self.p["dt"]),
                                      ctypes.byref(stats))
        if raise_on_fail and st != M1_OK:
            raise M1Error(st, _lib.m1_last_error(self.ctx).decode())
        return st, stats.as_dict()

    def set_network(self, net):
        self._net = net
        self._check(_lib.m1_set_network(self.ctx, net.handle if net is not None else None))

    def nn_features(self, r):
        r = self.to_device(r)
        f = self.torch.zeros(self.shape + (9,), dtype=self.torch.float32, device=self.device)
        self._check(_lib.m1_nn_features(self.ctx, r.data_ptr(), f.data_ptr()))
        return f

    def nn_target(self, r, e):
        r = self.to_device(r)
        e = self.to_device(e)
        t = self.torch.zeros(self.shape + (3,), dtype=self.torch.float32, device=self.device)
        self._check(_lib.m1_nn_target(self.ctx, r.data_ptr(), e.data_ptr(), t.data_ptr()))
        return t

    def solve_linear(self, b, *, raise_on_fail=True):
        b = self.to_device(b)
        x = self.vector()
        stats = M1Stats()
        st = _lib.m1_solve_linear(self.ctx, b.data_ptr(), x.data_ptr(), ctypes.byref(stats))
        if raise_on_fail and st != M1_OK:
            raise M1Error(st, _lib.m1_last_error(self.ctx).decode())
        return x, st, stats.as_dict()

    def profile_enable(self, on=True):
        self._check(_lib.m1_profile_enable(self.ctx, 1 if on else 0))

    def profile(self):
        out = {}
        for k, name in enumerate(kernel_classes()):
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            nbytes = ctypes.c_double()
            self._check(_lib.m1_profile_query(self.ctx, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nbytes)))
            if n.value:
                issued = ctypes.c_int64()
                self._check(_lib.m1_profile_issued(self.ctx, k, ctypes.byref(issued)))
                out[name] = {"launches": n.value, "ms": ms.value, "bytes": nbytes.value, "issued": issued.value}
        return out

    def close(self):
        if getattr(self, "ctx", None):
            _lib.m1_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned preconditioner's network (m1nn handle) with torch-tensor I/O."""

    def __init__(self, cin=9, cout=3, channels=(32, 48, 64, 64), Hmax=512, Wmax=512, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.cin, self.cout, self.channels = cin, cout, tuple(channels)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        ch = (ctypes.c_int32 * len(channels))(*channels)
        h = ctypes.c_void_p()
        st = _lib.m1nn_create(cin, cout, len(channels), ch, Hmax, Wmax, ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(h))
        if st != M1_OK:
            raise M1Error(st, "m1nn_create failed")
        self.handle = h

    def _check(self, st):
        if st != M1_OK:
            raise M1Error(st, _lib.m1nn_last_error(self.handle).decode())

    @property
    def param_count(self):
        return int(_lib.m1nn_param_count(self.handle))

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(_lib.m1nn_set_params(self.handle, a.ctypes.data, a.size))

    def init_params(self, seed=0, head_scale=0.1):
        """He-normal initial weights drawn by the library (m1nn_init_params)."""
        self._check(_lib.m1nn_init_params(self.handle, int(seed), float(head_scale)))

    def get_params(self):
        import numpy as np
        a = np.zeros(self.param_count, dtype=np.float32)
        self._check(_lib.m1nn_get_params(self.handle, a.ctypes.data, a.size))
        return a

    def get_grads(self):
        import numpy as np
        a = np.zeros(self.param_count, dtype=np.float32)
        self._check(_lib.m1nn_get_grads(self.handle, a.ctypes.data, a.size))
        return a

    def _t(self, a, C):
        t = self.torch.as_tensor(a, dtype=self.torch.float32).to(self.device).contiguous()
        assert t.dim() == 3 and t.shape[2] == C
        return t

    def forward(self, x):
        x = self._t(x, self.cin)
        H, W = x.shape[0], x.shape[1]
        y = self.torch.zeros((H, W, self.cout), dtype=self.torch.float32, device=self.device)
        self._check(_lib.m1nn_forward(self.handle, x.data_ptr(), H, W, y.data_ptr()))
        return y

    def backward(self, x, target):
        x = self._t(x, self.cin)
        t = self._t(target, self.cout)
        loss = ctypes.c_double()
        self._check(_lib.m1nn_backward(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], x.shape[1],
                                       ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr):
        self._check(_lib.m1nn_adam_step(self.handle, float(lr)))

    def train_step(self, x, target, lr):
        x = self._t(x, self.cin)
        t = self._t(target, self.cout)
        loss = ctypes.c_double()
        self._check(_lib.m1nn_train_step(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], x.shape[1],
                                         float(lr), ctypes.byref(loss)))
        return loss.value

    def save(self, path):
        self._check(_lib.m1nn_save(self.handle, str(path).encode()))

    def load(self, path):
        self._check(_lib.m1nn_load(self.handle, str(path).encode()))

    def close(self):
        if getattr(self, "handle", None):
            _lib.m1nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
