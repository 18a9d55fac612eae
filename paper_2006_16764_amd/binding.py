"""Thin ctypes binding of libpfjfnk (argument marshalling only).

Every function of include/pfjfnk.h is exposed under the same name.  Device
arrays are passed as torch CUDA tensors (float64, contiguous); the stream is
torch's current stream unless given.  All arithmetic happens in the library's
HIP kernels; this module never computes on the data.  Loading fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PF_LIB", os.path.join(_PKG, "libpfjfnk.so"))

PF_OK = 0
PF_ERR_INVALID_ARG = -1
PF_ERR_HIP = -2
PF_ERR_NONFINITE = -3
PF_ERR_NOT_CONVERGED = -4
PF_ERR_LINEAR = -5
PF_ERR_LINESEARCH = -6
PF_ERR_OOM = -7
PF_JV_FD = 0
PF_JV_ANALYTIC = 1
PF_PC_NONE = 0
PF_PC_JACOBI = 1
PF_PC_GMG = 2
PF_FP64 = 0
PF_FP32 = 1
PF_MAX_LOG = 64

ERROR_NAMES = {
    PF_ERR_INVALID_ARG: "PF_ERR_INVALID_ARG", PF_ERR_HIP: "PF_ERR_HIP",
    PF_ERR_NONFINITE: "PF_ERR_NONFINITE", PF_ERR_NOT_CONVERGED: "PF_ERR_NOT_CONVERGED",
    PF_ERR_LINEAR: "PF_ERR_LINEAR", PF_ERR_LINESEARCH: "PF_ERR_LINESEARCH", PF_ERR_OOM: "PF_ERR_OOM",
}


class pf_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("half_width", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("eps4", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("D", ctypes.c_double), ("delta2", ctypes.c_double), ("theta", ctypes.c_double),
                ("order", ctypes.c_int)]


class pf_alloy_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("l_T", ctypes.c_double), ("x_iso", ctypes.c_double),
                ("v_pull", ctypes.c_double)]


class pf_freegrowth_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("Gamma", ctypes.c_double), ("W", ctypes.c_double),
                ("alpha", ctypes.c_double), ("Lcp", ctypes.c_double), ("Tm", ctypes.c_double)]


class pf_solver_opts(ctypes.Structure):
    _fields_ = [("tau_r", ctypes.c_double), ("tau_a", ctypes.c_double),
                ("max_newton", ctypes.c_int), ("max_backtracks", ctypes.c_int),
                ("gmres_m", ctypes.c_int), ("gmres_maxit", ctypes.c_int),
                ("eta0", ctypes.c_double), ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double),
                ("gamma", ctypes.c_double), ("omega", ctypes.c_double),
                ("jv_mode", ctypes.c_int), ("pc", ctypes.c_int), ("pc_precision", ctypes.c_int)]


class pf_solver_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_its", ctypes.c_int),
                ("gmres_its_total", ctypes.c_int), ("backtracks", ctypes.c_int),
                ("f0", ctypes.c_double), ("f_final", ctypes.c_double),
                ("gmres_its", ctypes.c_int * PF_MAX_LOG), ("fnorm", ctypes.c_double * (PF_MAX_LOG + 1)),
                ("t_total_ms", ctypes.c_double)]

    def as_dict(self):
        k = min(self.newton_its, PF_MAX_LOG)
        return dict(status=self.status, newton_its=self.newton_its,
                    gmres_its_total=self.gmres_its_total, backtracks=self.backtracks,
                    f0=self.f0, f_final=self.f_final, gmres_its=list(self.gmres_its[:max(k, 1)]),
                    fnorm=list(self.fnorm[:k + 1]), t_total_ms=self.t_total_ms)


_VP = ctypes.c_void_p
_SIGS = {
    "pf_default_opts": (None, [ctypes.POINTER(pf_solver_opts)]),
    "pf_create": (ctypes.c_int, [ctypes.POINTER(pf_params), ctypes.c_int, ctypes.POINTER(_VP)]),
    "pf_destroy": (ctypes.c_int, [_VP]),
    "pf_set_params": (ctypes.c_int, [_VP, ctypes.POINTER(pf_params)]),
    "pf_num_nodes": (ctypes.c_longlong, [_VP]),
    "pf_residual": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pf_residual_noalloc": (ctypes.c_int, [ctypes.POINTER(pf_params), _VP, _VP, _VP, _VP]),
    "pf_theta_explicit": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "pf_jvp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP]),
    "pf_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pf_precond_setup": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.c_int, _VP]),
    "pf_precond_apply": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "pf_linear_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(pf_solver_opts), ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_newton_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(pf_solver_opts),
                                      ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_newton_step_theta": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(pf_solver_opts),
                                            ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_evolve": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.POINTER(pf_solver_opts),
                                 ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_adjoint_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(pf_solver_opts),
                                       ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_adjoint_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(pf_solver_opts),
                                        ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_misfit": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pf_dot": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "pf_set_alloy": (ctypes.c_int, [_VP, ctypes.POINTER(pf_alloy_params)]),
    "pf_alloy_residual": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    "pf_alloy_explicit": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP]),
    "pf_alloy_jvp": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, ctypes.c_int, _VP,
                                    _VP]),
    "pf_alloy_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, _VP, ctypes.POINTER(pf_solver_opts),
                                     ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_alloy_evolve": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(pf_solver_opts), ctypes.POINTER(pf_solver_stats),
                                       _VP]),
    "pf_set_freegrowth": (ctypes.c_int, [_VP, ctypes.POINTER(pf_freegrowth_params)]),
    "pf_fg_residual": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pf_fg_explicit": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "pf_fg_jvp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP]),
    "pf_fg_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(pf_solver_opts),
                                  ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_fg_evolve": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.POINTER(pf_solver_opts),
                                    ctypes.POINTER(pf_solver_stats), _VP]),
    "pf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libpfjfnk.so and declare every function's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2006_16764_amd.build`"
                           " (there is no fallback path)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PFError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, fn: str):
    if code != PF_OK:
        raise PFError(code, fn, load().pf_last_error().decode())


def _ptr(t: Optional[torch.Tensor], n: int = 0):
    """Device address of t (None passes through).  The library takes plain
    pointers, so the sizes it will touch are checked here: t must hold at least
    n float64 entries."""
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"tensor of {t.numel()} entries where {n} are needed")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_opts(**kw) -> pf_solver_opts:
    o = pf_solver_opts()
    load().pf_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def make_params(dim, n, half_width, dt, eps4, lam, D, delta2=1e-8, theta=1.0, order=1) -> pf_params:
    p = pf_params()
    p.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    hw = list(half_width) + [1.0] * (3 - len(half_width))
    for k in range(3):
        p.n[k] = int(nn[k])
        p.half_width[k] = float(hw[k])
    p.dt, p.eps4, p.lambda_, p.D, p.delta2, p.theta = dt, eps4, lam, D, delta2, theta
    p.order = order
    return p


class Problem:
    """Owns a pf_problem handle; methods mirror the C ABI one to one."""

    def __init__(self, params: pf_params, gmres_m_max: int = 30):
        lib = load()
        self.params = params
        h = ctypes.c_void_p()
        _check(lib.pf_create(ctypes.byref(params), gmres_m_max, ctypes.byref(h)), "pf_create")
        self.h = h
        self.n_nodes = int(lib.pf_num_nodes(h))
        self.n_dof = 2 * self.n_nodes

    def close(self) -> int:
        """pf_destroy; returns its code (the message stays in last_destroy_error)."""
        rc = PF_OK
        if getattr(self, "h", None):
            rc = load().pf_destroy(self.h)
            self.h = None
            self.last_destroy_error = load().pf_last_error().decode() if rc != PF_OK else ""
        return rc

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _v(self, t, n=None):
        """_ptr of a vector argument: 2 * n_nodes entries unless n says otherwise."""
        return _ptr(t, self.n_dof if n is None else n)

    def new_vector(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.n_dof, dtype=torch.float64, device=device)

    def set_params(self, params: pf_params):
        _check(load().pf_set_params(self.h, ctypes.byref(params)), "pf_set_params")
        self.params = params

    def pf_residual(self, U, Uprev, F, rhs=None, stream=None):
        _check(load().pf_residual(self.h, self._v(U), self._v(Uprev), self._v(rhs), self._v(F),
                                  _stream(stream)), "pf_residual")
        return F

    def pf_theta_explicit(self, Uprev, Uprev2, E, stream=None):
        _check(load().pf_theta_explicit(self.h, self._v(Uprev), self._v(Uprev2), self._v(E), _stream(stream)),
               "pf_theta_explicit")
        return E

    def pf_jvp(self, U, Uprev, v, Jv, mode=PF_JV_ANALYTIC, F0=None, stream=None):
        _check(load().pf_jvp(self.h, self._v(U), self._v(Uprev), self._v(v), self._v(F0), mode, self._v(Jv),
                             _stream(stream)), "pf_jvp")
        return Jv

    def pf_vjp(self, U, Uprev, w, gU=None, gUprev=None, gparams=None, stream=None):
        _check(load().pf_vjp(self.h, self._v(U), self._v(Uprev), self._v(w), self._v(gU), self._v(gUprev),
                             self._v(gparams, 2), _stream(stream)), "pf_vjp")

    def pf_precond_setup(self, U, kind=PF_PC_GMG, precision=PF_FP64, stream=None):
        _check(load().pf_precond_setup(self.h, self._v(U), kind, precision, _stream(stream)),
               "pf_precond_setup")

    def pf_precond_apply(self, r, z, stream=None):
        _check(load().pf_precond_apply(self.h, self._v(r), self._v(z), _stream(stream)), "pf_precond_apply")
        return z

    def pf_linear_solve(self, U, Uprev, b, x, transpose=0, rtol=1e-10, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_linear_solve(self.h, self._v(U), self._v(Uprev), self._v(b), self._v(x),
                                      transpose, rtol, ctypes.byref(o), ctypes.byref(st),
                                      _stream(stream)), "pf_linear_solve")
        return st.as_dict()

    def pf_newton_step(self, Uprev, U, opts=None, stream=None, check=True):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        rc = load().pf_newton_step(self.h, self._v(Uprev), self._v(U), ctypes.byref(o), ctypes.byref(st),
                                   _stream(stream))
        if check:
            _check(rc, "pf_newton_step")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def pf_newton_step_theta(self, Uprev2, Uprev, U, opts=None, stream=None, check=True):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        rc = load().pf_newton_step_theta(self.h, self._v(Uprev2), self._v(Uprev), self._v(U), ctypes.byref(o),
                                         ctypes.byref(st), _stream(stream))
        if check:
            _check(rc, "pf_newton_step_theta")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def pf_evolve(self, states, steps, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_evolve(self.h, self._v(states, (steps + 1) * self.n_dof), steps,
                                ctypes.byref(o), ctypes.byref(st), _stream(stream)), "pf_evolve")
        return st.as_dict()

    def pf_adjoint_step(self, U, Uprev, mu, lam, mu_prev, gparams, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_adjoint_step(self.h, self._v(U), self._v(Uprev), self._v(mu), self._v(lam),
                                      self._v(mu_prev), self._v(gparams, 2), ctypes.byref(o),
                                      ctypes.byref(st), _stream(stream)), "pf_adjoint_step")
        return st.as_dict()

    def pf_adjoint_solve(self, U, Uprev, rhs, lam, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_adjoint_solve(self.h, self._v(U), self._v(Uprev), self._v(rhs), self._v(lam),
                                       ctypes.byref(o), ctypes.byref(st), _stream(stream)),
               "pf_adjoint_solve")
        return st.as_dict()

    def pf_set_alloy(self, alloy: pf_alloy_params):
        _check(load().pf_set_alloy(self.h, ctypes.byref(alloy)), "pf_set_alloy")
        self.alloy = alloy

    def pf_alloy_residual(self, U, Uprev, Uprev2, t, F, stream=None):
        _check(load().pf_alloy_residual(self.h, self._v(U), self._v(Uprev), self._v(Uprev2), float(t),
                                        self._v(F), _stream(stream)), "pf_alloy_residual")
        return F

    def pf_alloy_explicit(self, Uprev, t_prev, E, stream=None):
        _check(load().pf_alloy_explicit(self.h, self._v(Uprev), float(t_prev), self._v(E), _stream(stream)),
               "pf_alloy_explicit")
        return E

    def pf_alloy_jvp(self, U, Uprev, Uprev2, t, v, Jv, mode=PF_JV_ANALYTIC, F0=None, stream=None):
        _check(load().pf_alloy_jvp(self.h, self._v(U), self._v(Uprev), self._v(Uprev2), float(t), self._v(v),
                                   self._v(F0), mode, self._v(Jv), _stream(stream)), "pf_alloy_jvp")
        return Jv

    def pf_alloy_step(self, Uprev2, Uprev, t_prev, U, opts=None, stream=None, check=True):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        rc = load().pf_alloy_step(self.h, self._v(Uprev2), self._v(Uprev), float(t_prev), self._v(U),
                                  ctypes.byref(o), ctypes.byref(st), _stream(stream))
        if check:
            _check(rc, "pf_alloy_step")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def pf_alloy_evolve(self, states, steps, t0=0.0, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_alloy_evolve(self.h, self._v(states, (steps + 1) * self.n_dof), steps,
                                      float(t0), ctypes.byref(o), ctypes.byref(st), _stream(stream)),
               "pf_alloy_evolve")
        return st.as_dict()

    def pf_set_freegrowth(self, fgp: pf_freegrowth_params):
        _check(load().pf_set_freegrowth(self.h, ctypes.byref(fgp)), "pf_set_freegrowth")
        self.fg = fgp

    def pf_fg_residual(self, U, Uprev, Uprev2, F, stream=None):
        _check(load().pf_fg_residual(self.h, self._v(U), self._v(Uprev), self._v(Uprev2), self._v(F),
                                     _stream(stream)), "pf_fg_residual")
        return F

    def pf_fg_explicit(self, Uprev, E, stream=None):
        _check(load().pf_fg_explicit(self.h, self._v(Uprev), self._v(E), _stream(stream)), "pf_fg_explicit")
        return E

    def pf_fg_jvp(self, U, Uprev, Uprev2, v, Jv, mode=PF_JV_ANALYTIC, F0=None, stream=None):
        _check(load().pf_fg_jvp(self.h, self._v(U), self._v(Uprev), self._v(Uprev2), self._v(v),
                                self._v(F0), mode, self._v(Jv), _stream(stream)), "pf_fg_jvp")
        return Jv

    def pf_fg_step(self, Uprev2, Uprev, U, opts=None, stream=None, check=True):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        rc = load().pf_fg_step(self.h, self._v(Uprev2), self._v(Uprev), self._v(U), ctypes.byref(o),
                               ctypes.byref(st), _stream(stream))
        if check:
            _check(rc, "pf_fg_step")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def pf_fg_evolve(self, states, steps, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        st = pf_solver_stats()
        _check(load().pf_fg_evolve(self.h, self._v(states, (steps + 1) * self.n_dof), steps,
                                   ctypes.byref(o), ctypes.byref(st), _stream(stream)), "pf_fg_evolve")
        return st.as_dict()

    def pf_misfit(self, U, phi_target, L_dev, dLdU=None, stream=None):
        _check(load().pf_misfit(self.h, self._v(U), self._v(phi_target, self.n_nodes),
                                self._v(L_dev, 1), self._v(dLdU), _stream(stream)), "pf_misfit")

    def pf_dot(self, x, y, out_dev, stream=None):
        _check(load().pf_dot(self.h, self._v(x), self._v(y), self._v(out_dev, 1), _stream(stream)), "pf_dot")


def pf_residual_noalloc(params: pf_params, U, Uprev, F, stream=None):
    """F = F(U; Uprev) with no handle and no device allocation (the library's
    fixed scratch array); same arguments as Problem.pf_residual plus params."""
    n = 1
    for k in range(params.dim):
        n *= params.n[k] + 1
    _check(load().pf_residual_noalloc(ctypes.byref(params), _ptr(U, 2 * n), _ptr(Uprev, 2 * n),
                                      _ptr(F, 2 * n), _stream(stream)), "pf_residual_noalloc")
    return F


def problem_for(w, gmres_m_max: int = 30, eps4=None, lam=None, theta=1.0) -> Problem:
    """Problem for an inputs.Workload (same mesh/parameter recipe)."""
    p = make_params(w.dim, [w.n] * w.dim, [w.half_width] * w.dim, w.dt,
                    w.eps4 if eps4 is None else eps4, w.lam if lam is None else lam, w.D, w.delta2,
                    theta)
    return Problem(p, gmres_m_max)


def alloy_problem_for(w, gmres_m_max: int = 30, dt=None) -> Problem:
    """Problem in the alloy model for an inputs.AlloyWorkload."""
    D, l_T, v_pull = w.scales()
    p = make_params(w.dim, list(w.n), list(w.half_width), w.dt if dt is None else dt, w.eps4, w.lam, D,
                    w.delta2, w.theta)
    pb = Problem(p, gmres_m_max)
    a = pf_alloy_params()
    a.k, a.l_T, a.x_iso, a.v_pull = w.k, l_T, w.x_iso, v_pull
    pb.pf_set_alloy(a)
    return pb


def freegrowth_problem_for(w, gmres_m_max: int = 30, dt=None) -> Problem:
    """Problem in the free-growth model for an inputs.FreeGrowthWorkload."""
    p = make_params(w.dim, list(w.n), list(w.half_width), w.dt if dt is None else dt, w.eps4, 0.0, 1.0,
                    w.delta2, w.theta, w.order)
    pb = Problem(p, gmres_m_max)
    f = pf_freegrowth_params()
    f.beta, f.Gamma, f.W, f.alpha, f.Lcp, f.Tm = w.beta, w.Gamma, w.W, w.alpha, w.Lcp, w.Tm
    pb.pf_set_freegrowth(f)
    return pb
