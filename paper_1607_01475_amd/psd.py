"""Thin Python binding of the gfx950 PSD solver library (``libpsd.so``).

Argument marshalling only: every step of the solver runs in the HIP
kernels behind the C ABI declared in ``include/psd.h``.  PyTorch provides
device memory (tensors) and the stream.  Loading fails loudly when the
library has not been built; there is no CPU fallback.

Arrays are float64 CUDA tensors of shape (n, n) or (n, n, n), C-contiguous,
x fastest (the last tensor axis is x).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence, Union

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsd.so")

PSD_OK = 0
PSD_NOT_CONVERGED = 1
PSD_ERR_ARG = -1
PSD_ERR_RANGE = -2
PSD_ERR_HIP = -3
PSD_ERR_NONFINITE = -4
PSD_ERR_NOT_DESCENT = -5
PSD_ERR_MEAN = -6
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_RANGE", -3: "ERR_HIP",
                -4: "ERR_NONFINITE", -5: "ERR_NOT_DESCENT", -6: "ERR_MEAN"}

PSD_FP64 = 0
PSD_MIXED = 1

PASS_NAMES = ["rows_r2c", "cols_fwd", "cols_fused", "cols_inv", "rows_c2r", "ls", "ls_fin",
              "res", "res_fin"]


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("L", ctypes.c_double),
                ("order", ctypes.c_int), ("p", ctypes.c_double), ("s", ctypes.c_double),
                ("eps", ctypes.c_double), ("lam", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("graph_chunk", ctypes.c_int),
                ("history", ctypes.c_int), ("profile", ctypes.c_int),
                ("autotune", ctypes.c_int), ("metric", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("inner_iters", ctypes.c_int)]


PSD_METRIC_CONSTANT = 0
PSD_METRIC_VARIABLE = 1


class _StepStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("psd_iters", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("res_inf", ctypes.c_double), ("status", ctypes.c_int)]


PSD_SCHEME_THINFILM = 0
PSD_SCHEME_SPFC = 1
SCHEMES = {"thinfilm": PSD_SCHEME_THINFILM, "spfc": PSD_SCHEME_SPFC}


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("res_inf", ctypes.c_double),
                ("res_l2", ctypes.c_double), ("energy", ctypes.c_double),
                ("status", ctypes.c_int), ("ls_truncated", ctypes.c_int)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_lib = None

SIGNATURES = {
    "psd_check_problem": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_char_p, ctypes.c_int]),
    "psd_create": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(_Options),
                                  _vp, ctypes.POINTER(_vp)]),
    "psd_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_Stats)]),
    "psd_solve_noalloc": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), _vp,
                                         _vp, _vp, _vp, _vp, ctypes.POINTER(_Stats)]),
    "psd_residual": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _dp]),
    "psd_residual_mixed": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _dp]),
    "psd_energy": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _dp]),
    "psd_grad": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "psd_adjoint": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                   _dp, _dp, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]),
    "psd_timestep": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_StepStats),
                                    ctypes.POINTER(ctypes.c_int)]),
    "psd_adjoint6": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]),
    "psd_history": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "psd_pass_times": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int)]),
    "psd_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "psd_destroy": (ctypes.c_int, [_vp]),
    "psd_last_error": (ctypes.c_char_p, [_vp]),
}


def load_library(path: str = LIB_PATH):
    """Load libpsd.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"PSD HIP library not built: {path} is missing "
                               "(run __graft_entry__.build() or paper_1607_01475_amd/build.py)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class PSDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


@dataclasses.dataclass
class Problem:
    """Problem statement (order 4: Sec. 5.3; order 6: Sec. 5.4)."""
    dim: int
    n: int
    L: float
    order: int = 4
    p: float = 4.0
    s: float = 0.01
    eps: float = 0.1
    lam: float = 0.0

    def c(self) -> _Problem:
        return _Problem(self.dim, self.n, float(self.L), self.order, float(self.p), float(self.s),
                        float(self.eps), float(self.lam))

    @property
    def shape(self):
        return (self.n,) * self.dim


def check_problem(prob: Problem):
    """Host-side validation (no GPU): returns (status, message)."""
    buf = ctypes.create_string_buffer(128)
    st = load_library().psd_check_problem(ctypes.byref(prob.c()), buf, 128)
    return st, buf.value.decode()


@dataclasses.dataclass
class Stats:
    iters: int
    res_inf: float
    res_l2: float
    energy: float
    status: int
    ls_truncated: int = 0


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts: Sequence[Optional[torch.Tensor]]):
    arr = (_vp * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else _ptr(t).value
    return arr


class Solver:
    """A handle over one or more instances (same dim, order and p)."""

    def __init__(self, problems: Union[Problem, List[Problem]], tol: float = 1e-10,
                 max_iter: int = 500, precision: str = "fp64", graph_chunk: int = 0,
                 history: bool = False, profile: bool = False, autotune: bool = False,
                 stream: Optional[torch.cuda.Stream] = None, metric: str = "constant",
                 inner_rtol: float = 0.0, inner_iters: int = 20):
        self._lib = load_library()
        self.problems = [problems] if isinstance(problems, Problem) else list(problems)
        self.batch = len(self.problems)
        arr = (_Problem * self.batch)(*[p.c() for p in self.problems])
        prec = {"fp64": PSD_FP64, "mixed": PSD_MIXED}[precision]
        met = {"constant": PSD_METRIC_CONSTANT, "variable": PSD_METRIC_VARIABLE}[metric]
        self.opt = _Options(float(tol), int(max_iter), prec, int(graph_chunk), 1 if history else 0,
                            1 if profile else 0, 1 if autotune else 0, met, float(inner_rtol),
                            int(inner_iters))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        st = self._lib.psd_create(arr, self.batch, ctypes.byref(self.opt),
                                  _vp(self.stream.cuda_stream), ctypes.byref(h))
        if st != PSD_OK:
            raise PSDError(st, self._lib.psd_last_error(None).decode())
        self._h = h

    def _check(self, st: int, allow=(PSD_OK,)):
        if st not in allow:
            raise PSDError(st, self._lib.psd_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._lib.psd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def solve(self, f: Sequence[torch.Tensor], u: Sequence[torch.Tensor],
              g: Optional[Sequence[torch.Tensor]] = None,
              w: Optional[Sequence[torch.Tensor]] = None, raise_on_error: bool = True):
        """Solve in place: u[b] holds u0 on entry and the final iterate on exit."""
        B = self.batch
        stats = (_Stats * B)()
        st = self._lib.psd_solve(self._h, _ptr_array(f), _ptr_array(g) if g is not None else None,
                                 _ptr_array(u), _ptr_array(w) if w is not None else None, stats)
        if raise_on_error:
            self._check(st, allow=(PSD_OK, PSD_NOT_CONVERGED))
        return [Stats(s.iters, s.res_inf, s.res_l2, s.energy, s.status, s.ls_truncated) for s in stats]

    def timestep(self, u: Sequence[torch.Tensor], nsteps: int, scheme: str = "thinfilm",
                 gamma1: float = 0.0, w: Optional[Sequence[torch.Tensor]] = None,
                 per_step: bool = False, raise_on_error: bool = True):
        """Convex-splitting time stepping (psd_timestep): u[b] holds u^0 on
        entry and u^nsteps on exit.  Returns per-instance dicts (steps,
        psd_iters, max_iters, res_inf, status) and, with per_step, the
        (nsteps, batch) array of PSD iteration counts."""
        import numpy as np
        B = self.batch
        stats = (_StepStats * B)()
        its = (ctypes.c_int * max(1, nsteps * B))() if per_step else None
        st = self._lib.psd_timestep(self._h, SCHEMES[scheme], float(gamma1), _ptr_array(u),
                                    _ptr_array(w) if w is not None else None, int(nsteps), stats, its)
        if raise_on_error:
            self._check(st, allow=(PSD_OK, PSD_NOT_CONVERGED))
        out = [dict(steps=x.steps, psd_iters=x.psd_iters, max_iters=x.max_iters, res_inf=x.res_inf,
                    status=x.status) for x in stats]
        if per_step:
            return out, np.array(its[: nsteps * B], dtype=np.int64).reshape(nsteps, B)
        return out

    def residual(self, inst: int, f, u, g=None, r=None):
        rinf = ctypes.c_double()
        self._check(self._lib.psd_residual(self._h, inst, _ptr(f), _ptr(g), _ptr(u), _ptr(r),
                                           ctypes.byref(rinf)))
        return rinf.value

    def residual_mixed(self, inst: int, f, g, u, w, r1=None, r2=None):
        rinf = ctypes.c_double()
        self._check(self._lib.psd_residual_mixed(self._h, inst, _ptr(f), _ptr(g), _ptr(u), _ptr(w),
                                                 _ptr(r1), _ptr(r2), ctypes.byref(rinf)))
        return rinf.value

    def energy(self, inst: int, f, u, g=None) -> float:
        E = ctypes.c_double()
        self._check(self._lib.psd_energy(self._h, inst, _ptr(f), _ptr(g), _ptr(u), ctypes.byref(E)))
        return E.value

    def grad(self, inst: int, f, u, g=None, out=None):
        if out is None:
            out = torch.empty_like(u)
        self._check(self._lib.psd_grad(self._h, inst, _ptr(f), _ptr(g), _ptr(u), _ptr(out)))
        return out

    def history(self, inst: int = 0):
        cap = self.opt.max_iter
        buf = (ctypes.c_double * (4 * max(cap, 1)))()
        cnt = ctypes.c_int()
        self._check(self._lib.psd_history(self._h, inst, buf, cap, ctypes.byref(cnt)))
        import numpy as np
        return np.array(buf[: 4 * cnt.value]).reshape(cnt.value, 4)

    def tuning(self):
        """(z-chunk residual, z-chunk line search, XCD order residual, XCD order line search,
        3D line-search tile width, row-transform layout)."""
        out = (ctypes.c_int * 6)()
        self._check(self._lib.psd_tuning(self._h, out))
        return tuple(out)

    def pass_times(self):
        """{pass name: (total ms, launches)} of the last solve (profile=True)."""
        ms = (ctypes.c_double * len(PASS_NAMES))()
        cnt = (ctypes.c_int * len(PASS_NAMES))()
        self._check(self._lib.psd_pass_times(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(PASS_NAMES)}

    def adjoint(self, u_star: Sequence[torch.Tensor], dJdu: Sequence[torch.Tensor],
                rtol: float = 1e-12, max_iter: int = 1000):
        B = self.batch
        dJdf = [torch.empty_like(t) for t in u_star]
        ds = (ctypes.c_double * B)()
        de = (ctypes.c_double * B)()
        it = (ctypes.c_int * B)()
        self._check(self._lib.psd_adjoint(self._h, _ptr_array(u_star), _ptr_array(dJdu),
                                          _ptr_array(dJdf), ds, de, float(rtol), int(max_iter), it))
        return dJdf, list(ds), list(de), list(it)


def solve_noalloc(problem: Problem, f: torch.Tensor, u: torch.Tensor, g: Optional[torch.Tensor] = None,
                  w: Optional[torch.Tensor] = None, tol: float = 1e-10, max_iter: int = 500,
                  precision: str = "fp64", history: bool = False,
                  stream: Optional[torch.cuda.Stream] = None) -> Stats:
    """One solve through psd_solve_noalloc (no device allocation: workspace in
    the library's static scratch array).  u holds u0 on entry and the final
    iterate on exit."""
    lib = load_library()
    prec = {"fp64": PSD_FP64, "mixed": PSD_MIXED}[precision]
    opt = _Options(float(tol), int(max_iter), prec, 0, 1 if history else 0, 0, 0, PSD_METRIC_CONSTANT, 0.0, 1)
    st = _Stats()
    strm = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.psd_solve_noalloc(ctypes.byref(problem.c()), ctypes.byref(opt), _vp(strm.cuda_stream),
                               _ptr(f), _ptr(g), _ptr(u), _ptr(w), ctypes.byref(st))
    if rc not in (PSD_OK, PSD_NOT_CONVERGED):
        raise PSDError(rc, lib.psd_last_error(None).decode())
    return Stats(st.iters, st.res_inf, st.res_l2, st.energy, st.status, st.ls_truncated)


def _adjoint6(self, u_star: Sequence[torch.Tensor], dJdu: Sequence[torch.Tensor],
              rtol: float = 1e-12, max_iter: int = 2000):
    """Adjoint of the converged sixth-order solves (psd_adjoint6): returns
    (dJdf, dJdg, dJds, dJdeps, dJdlam, cg_iters)."""
    B = self.batch
    dJdf = [torch.empty_like(t) for t in u_star]
    dJdg = [torch.empty_like(t) for t in u_star]
    ds, de, dl = (ctypes.c_double * B)(), (ctypes.c_double * B)(), (ctypes.c_double * B)()
    it = (ctypes.c_int * B)()
    self._check(self._lib.psd_adjoint6(self._h, _ptr_array(u_star), _ptr_array(dJdu), _ptr_array(dJdf),
                                       _ptr_array(dJdg), ds, de, dl, float(rtol), int(max_iter), it))
    return dJdf, dJdg, list(ds), list(de), list(dl), list(it)


Solver.adjoint6 = _adjoint6


class PSDSolveFn(torch.autograd.Function):
    """u* = PSD solve of N_h[u] = f (order 4) with an implicit adjoint.

    forward(f, s, eps, solver): f has shape (B, n, ..) for a solver of batch B
    (or (n, ..) when B = 1); s and eps are 0-d tensors that must equal the
    solver's problem values (they are inputs so that autograd can return
    their gradients).  backward solves H lam = dJ/du by the library's
    preconditioned conjugate gradients (psd_adjoint): dJ/df = lam,
    dJ/ds = -lam.dN/ds, dJ/deps = -lam.dN/deps; no solver trajectory is kept.
    """

    @staticmethod
    def forward(ctx, f, s, eps, solver, adj_rtol=1e-12, adj_max_iter=500):
        for P in solver.problems:
            if abs(P.s - float(s)) > 1e-15 * abs(P.s) or abs(P.eps - float(eps)) > 1e-15 * abs(P.eps):
                raise ValueError("s and eps must match the solver's problems")
        batched = f.dim() == solver.problems[0].dim + 1
        fs = list(f.detach().contiguous()) if batched else [f.detach().contiguous()]
        us = [torch.zeros_like(x) for x in fs]
        stats = solver.solve(fs, us)
        for st in stats:
            if st.status != PSD_OK:
                raise PSDError(st.status, "forward solve did not converge")
        u = torch.stack(us) if batched else us[0]
        ctx.solver, ctx.batched = solver, batched
        ctx.adj_rtol, ctx.adj_max_iter = adj_rtol, adj_max_iter
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        us = list(u) if ctx.batched else [u]
        gs = list(grad_u.contiguous()) if ctx.batched else [grad_u.contiguous()]
        gs = [g.contiguous() for g in gs]
        dJdf, ds, de, _ = ctx.solver.adjoint(us, gs, rtol=ctx.adj_rtol, max_iter=ctx.adj_max_iter)
        gf = torch.stack(dJdf) if ctx.batched else dJdf[0]
        dev = grad_u.device
        return (gf, torch.tensor(sum(ds), dtype=torch.float64, device=dev),
                torch.tensor(sum(de), dtype=torch.float64, device=dev), None, None, None)


def solve_differentiable(f, s, eps, solver, adj_rtol=1e-12, adj_max_iter=500):
    """Functional form of PSDSolveFn.apply."""
    return PSDSolveFn.apply(f, s, eps, solver, adj_rtol, adj_max_iter)
