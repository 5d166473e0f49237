"""Python access to the plain FP64 CPU oracle (``psd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product package never
imports this module.  Arrays are numpy float64, C-contiguous, x fastest
(numpy shape (n, n) or (n, n, n) with the last axis = x).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Prob(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("L", ctypes.c_double),
                ("order", ctypes.c_int), ("p", ctypes.c_double), ("s", ctypes.c_double),
                ("eps", ctypes.c_double), ("lam", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Prob)
        sig = {
            "orc_vgrad": (None, [P, _dp, _dp]),
            "orc_vgrad_axis": (None, [P, ctypes.c_int, _dp, _dp]),
            "orc_vdiv_axis": (None, [P, ctypes.c_int, _dp, _dp]),
            "orc_vdiv": (None, [P, _dp, _dp]),
            "orc_lap": (None, [P, _dp, _dp]),
            "orc_plap": (None, [P, _dp, _dp]),
            "orc_plap_lin": (None, [P, _dp, _dp, _dp]),
            "orc_dft1": (None, [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int]),
            "orc_fft1": (None, [ctypes.c_int, _dp, _dp, ctypes.c_int]),
            "orc_fftn": (None, [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int]),
            "orc_symbol_neglap": (None, [P, _dp]),
            "orc_symbol_precond": (None, [P, _dp]),
            "orc_precond": (None, [P, _dp, _dp]),
            "orc_T": (None, [P, _dp, _dp]),
            "orc_ip": (ctypes.c_double, [P, _dp, _dp]),
            "orc_maxabs": (ctypes.c_double, [P, _dp]),
            "orc_N4": (None, [P, _dp, _dp]),
            "orc_energy4": (ctypes.c_double, [P, _dp, _dp]),
            "orc_residual4": (None, [P, _dp, _dp, _dp]),
            "orc_residual6": (None, [P, _dp, _dp, _dp, _dp]),
            "orc_energy6": (ctypes.c_double, [P, _dp, _dp, _dp]),
            "orc_w_from_u": (None, [P, _dp, _dp, _dp, _dp]),
            "orc_mixed_residuals": (None, [P, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_ls_coeffs4": (None, [P, _dp, _dp, _dp, _dp]),
            "orc_q_eval": (None, [P, _dp, _dp, _dp, _dp, ctypes.c_double, _dp, _dp]),
            "orc_root_cubic": (ctypes.c_double, [_dp, ctypes.POINTER(ctypes.c_int)]),
            "orc_solve": (ctypes.c_int, [P, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                         _dp, _dp]),
            "orc_hessvec": (None, [P, _dp, _dp, _dp]),
            "orc_dN_dparams": (None, [P, _dp, _dp, _dp]),
            "orc_adjoint": (ctypes.c_int, [P, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp,
                                           _dp]),
            "orc_cholesky_solve": (ctypes.c_int, [ctypes.c_int, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Problem statement (Sec. 1 and Sec. 5): dim, n, L, order, p, s, eps, lam."""

    def __init__(self, dim: int, n: int, L: float, order: int = 4, p: float = 4.0,
                 s: float = 0.01, eps: float = 0.1, lam: float = 0.0):
        self.dim, self.n, self.L, self.order = dim, n, L, order
        self.p, self.s, self.eps, self.lam = p, s, eps, lam
        self._c = Prob(dim, n, L, order, p, s, eps, lam)

    @property
    def shape(self) -> Tuple[int, ...]:
        return (self.n,) * self.dim

    @property
    def h(self) -> float:
        return self.L / self.n

    @property
    def hd(self) -> float:
        return self.h ** self.dim

    def replace(self, **kw) -> "Problem":
        d = dict(dim=self.dim, n=self.n, L=self.L, order=self.order, p=self.p, s=self.s,
                 eps=self.eps, lam=self.lam)
        d.update(kw)
        return Problem(**d)

    # -- operators ---------------------------------------------------------
    def _unary(self, name, v):
        v = _arr(v)
        out = np.empty_like(v)
        getattr(_load(), name)(ctypes.byref(self._c), _ptr(v), _ptr(out))
        return out

    def lap(self, v):
        return self._unary("orc_lap", v)

    def plap(self, v):
        return self._unary("orc_plap", v)

    def N4(self, u):
        return self._unary("orc_N4", u)

    def precond(self, r):
        return self._unary("orc_precond", r)

    def T(self, z):
        return self._unary("orc_T", z)

    def vgrad(self, v):
        v = _arr(v)
        out = np.empty((self.dim,) + v.shape)
        _load().orc_vgrad(ctypes.byref(self._c), _ptr(v), _ptr(out))
        return out

    def vgrad_axis(self, axis: int, v):
        v = _arr(v)
        out = np.empty_like(v)
        _load().orc_vgrad_axis(ctypes.byref(self._c), axis, _ptr(v), _ptr(out))
        return out

    def vdiv_axis(self, axis: int, v):
        v = _arr(v)
        out = np.empty_like(v)
        _load().orc_vdiv_axis(ctypes.byref(self._c), axis, _ptr(v), _ptr(out))
        return out

    def vdiv(self, F):
        F = _arr(F)
        out = np.empty(F.shape[1:])
        _load().orc_vdiv(ctypes.byref(self._c), _ptr(F), _ptr(out))
        return out

    def plap_lin(self, u, xi):
        u, xi = _arr(u), _arr(xi)
        out = np.empty_like(u)
        _load().orc_plap_lin(ctypes.byref(self._c), _ptr(u), _ptr(xi), _ptr(out))
        return out

    def symbol_neglap(self):
        out = np.empty(self.shape)
        _load().orc_symbol_neglap(ctypes.byref(self._c), _ptr(out))
        return out

    def symbol_precond(self):
        out = np.empty(self.shape)
        _load().orc_symbol_precond(ctypes.byref(self._c), _ptr(out))
        return out

    def ip(self, a, b) -> float:
        return _load().orc_ip(ctypes.byref(self._c), _ptr(_arr(a)), _ptr(_arr(b)))

    def residual(self, f, u, g=None):
        f, u = _arr(f), _arr(u)
        out = np.empty_like(u)
        if self.order == 4:
            _load().orc_residual4(ctypes.byref(self._c), _ptr(f), _ptr(u), _ptr(out))
        else:
            _load().orc_residual6(ctypes.byref(self._c), _ptr(f), _ptr(_arr(g)), _ptr(u),
                                  _ptr(out))
        return out

    def energy(self, f, u, g=None) -> float:
        f, u = _arr(f), _arr(u)
        if self.order == 4:
            return _load().orc_energy4(ctypes.byref(self._c), _ptr(f), _ptr(u))
        return _load().orc_energy6(ctypes.byref(self._c), _ptr(f), _ptr(_arr(g)), _ptr(u))

    def w_from_u(self, f, g, u):
        out = np.empty_like(_arr(u))
        _load().orc_w_from_u(ctypes.byref(self._c), _ptr(_arr(f)), _ptr(_arr(g)),
                             _ptr(_arr(u)), _ptr(out))
        return out

    def mixed_residuals(self, f, g, u, w):
        r1 = np.empty_like(_arr(u))
        r2 = np.empty_like(r1)
        _load().orc_mixed_residuals(ctypes.byref(self._c), _ptr(_arr(f)), _ptr(_arr(g)),
                                    _ptr(_arr(u)), _ptr(_arr(w)), _ptr(r1), _ptr(r2))
        return r1, r2

    def ls_coeffs4(self, u, d, r):
        c = np.empty(4)
        _load().orc_ls_coeffs4(ctypes.byref(self._c), _ptr(_arr(u)), _ptr(_arr(d)),
                               _ptr(_arr(r)), _ptr(c))
        return c

    def q_eval(self, f, u, d, alpha, g=None):
        q = ctypes.c_double()
        dq = ctypes.c_double()
        _load().orc_q_eval(ctypes.byref(self._c), _ptr(_arr(f)),
                           _ptr(_arr(g)) if g is not None else None, _ptr(_arr(u)),
                           _ptr(_arr(d)), float(alpha), ctypes.byref(q), ctypes.byref(dq))
        return q.value, dq.value

    def solve(self, f, u0=None, g=None, tol: float = 1e-10, max_iter: int = 500,
              history: bool = False):
        """Run the PSD loop.  Returns dict(u, w, iters, res_inf, res_l2, energy, hist)."""
        f = _arr(f)
        if u0 is None:
            u = np.zeros_like(f)
            if self.order == 6:
                u += float(np.mean(g))
        else:
            u = _arr(u0).copy()
        w = np.empty_like(f) if self.order == 6 else None
        hist = np.zeros((max_iter, 4)) if history else None
        stats = np.zeros(3)
        k = _load().orc_solve(ctypes.byref(self._c), _ptr(f),
                              _ptr(_arr(g)) if g is not None else None, _ptr(u), _ptr(w),
                              float(tol), int(max_iter), _ptr(hist), _ptr(stats))
        if k < 0:
            raise RuntimeError(f"oracle solve failed with status {k}")
        return dict(u=u, w=w, iters=k, res_inf=stats[0], res_l2=stats[1], energy=stats[2],
                    hist=hist[:k] if history else None)

    def hessvec(self, u, xi):
        out = np.empty_like(_arr(u))
        _load().orc_hessvec(ctypes.byref(self._c), _ptr(_arr(u)), _ptr(_arr(xi)), _ptr(out))
        return out

    def dN_dparams(self, u):
        ds = np.empty_like(_arr(u))
        de = np.empty_like(ds)
        _load().orc_dN_dparams(ctypes.byref(self._c), _ptr(_arr(u)), _ptr(ds), _ptr(de))
        return ds, de

    def adjoint(self, u, gu, rtol: float = 1e-13, max_iter: int = 1000):
        lam = np.empty_like(_arr(u))
        js = ctypes.c_double()
        je = ctypes.c_double()
        it = _load().orc_adjoint(ctypes.byref(self._c), _ptr(_arr(u)), _ptr(_arr(gu)),
                                 float(rtol), int(max_iter), _ptr(lam), ctypes.byref(js),
                                 ctypes.byref(je))
        if it < 0:
            raise RuntimeError("oracle adjoint failed")
        return dict(dJdf=lam, dJds=js.value, dJdeps=je.value, iters=it)


def root_cubic(c) -> Tuple[float, int]:
    c = _arr(c)
    ev = ctypes.c_int()
    x = _load().orc_root_cubic(_ptr(c), ctypes.byref(ev))
    return x, ev.value


def dft1(x: np.ndarray, sign: int = -1) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    n = len(x)
    xr, xi = _arr(x.real), _arr(x.imag)
    yr, yi = np.empty(n), np.empty(n)
    _load().orc_dft1(n, _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi), sign)
    return yr + 1j * yi


def fft1(x: np.ndarray, sign: int = -1) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    xr, xi = _arr(x.real).copy(), _arr(x.imag).copy()
    _load().orc_fft1(len(x), _ptr(xr), _ptr(xi), sign)
    return xr + 1j * xi


def fftn(x: np.ndarray, sign: int = -1, naive: bool = False) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    dim = x.ndim
    n = x.shape[0]
    assert all(s == n for s in x.shape)
    xr, xi = _arr(x.real).copy(), _arr(x.imag).copy()
    _load().orc_fftn(dim, n, _ptr(xr), _ptr(xi), sign, 1 if naive else 0)
    return xr + 1j * xi


def cholesky_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    A = _arr(A).copy()
    x = _arr(b).copy()
    st = _load().orc_cholesky_solve(len(x), _ptr(A), _ptr(x))
    if st != 0:
        raise RuntimeError("matrix not SPD")
    return x


# ---------------------------------------------------------------------------
# Convex-splitting time stepping (Sec. 6.1 thin film, Sec. 6.2 SPFC): each
# step is one PSD solve, warm-started from the previous time level.
# ---------------------------------------------------------------------------
def skew_lap(P: "Problem", v) -> np.ndarray:
    """Delta_h^v v = d.(D v): the vertex gradient of Sec. 5.1 followed by the
    vertex-to-centre divergence (the 'skew' Laplacian of the thin-film
    scheme)."""
    return P.vdiv(P.vgrad(v))


def thinfilm_steps(P: "Problem", u0, nsteps: int, tol: float = 1e-10, max_iter: int = 500):
    """Thin-film convex-splitting scheme (Sec. 6.1): N_h[u^{n+1}] = u^n - s Delta_h^v u^n
    with N_h of the fourth-order problem (time step s, exponent p, eps), PSD
    started from u^n.  Returns (u^N, list of PSD iteration counts per step)."""
    assert P.order == 4
    u = _arr(u0).copy()
    iters = []
    for _ in range(nsteps):
        f = u - P.s * skew_lap(P, u)
        out = P.solve(f, u0=u, tol=tol, max_iter=max_iter)
        u = out["u"]
        iters.append(out["iters"])
    return u, iters


def spfc_steps(P: "Problem", u0, gamma1: float, nsteps: int, tol: float = 1e-10,
               max_iter: int = 500):
    """Square phase field crystal scheme (Sec. 6.2): the sixth-order mixed
    system with lambda = gamma0, g = u^n and f = -s gamma1 Delta_h u^n (time
    step s), PSD started from u^n.  The factor s on the explicit term is the
    one that makes the step consistent with the H^-1 gradient flow of the SPFC
    energy (the scheme is printed without it).  Returns (u^N, w^N, iteration
    counts)."""
    assert P.order == 6
    u = _arr(u0).copy()
    iters = []
    w = None
    for _ in range(nsteps):
        g = u.copy()
        f = -P.s * gamma1 * P.lap(u)
        out = P.solve(f, u0=u, g=g, tol=tol, max_iter=max_iter)
        u, w = out["u"], out["w"]
        iters.append(out["iters"])
    return u, w, iters


def interp_coarse_to_fine(uc: np.ndarray) -> np.ndarray:
    """Bilinear (2D) / trilinear (3D) interpolation from a periodic
    cell-centred grid to the grid of half the spacing: fine cell 2i lies a
    quarter of a coarse cell below coarse centre i, fine cell 2i+1 a quarter
    above, so per axis the weights are 3/4 on the nearer and 1/4 on the
    farther coarse centre."""
    out = np.asarray(uc, dtype=np.float64)
    for ax in range(out.ndim):
        lo = np.roll(out, 1, axis=ax)    # coarse centre i-1
        hi = np.roll(out, -1, axis=ax)   # coarse centre i+1
        even = 0.75 * out + 0.25 * lo
        odd = 0.75 * out + 0.25 * hi
        shape = list(out.shape)
        shape[ax] *= 2
        res = np.empty(shape)
        idx = [slice(None)] * out.ndim
        idx[ax] = slice(0, None, 2)
        res[tuple(idx)] = even
        idx[ax] = slice(1, None, 2)
        res[tuple(idx)] = odd
        out = res
    return out


# ---------------------------------------------------------------------------
# Variable-metric search direction (Remark in Sec. 3): L_k[nu] = nu - s div_h(
# |grad_h u^k|^{p-2} grad_h nu) + s eps^2 Delta_h^2 nu, the p-Laplacian's
# coefficient frozen at the current iterate.  L_k is not diagonal in Fourier
# space; d^k = L_k^{-1} r^k is computed by conjugate gradients preconditioned
# with the constant-coefficient operator L_h (FFT, Sec. 5.3).
# ---------------------------------------------------------------------------
def apply_Lk(P: "Problem", u, nu) -> np.ndarray:
    """L_k[nu] with the frozen coefficient R = |grad_h u|^{p-2} at the vertices."""
    G = P.vgrad(u)
    R = (G * G).sum(axis=0) ** ((P.p - 2.0) / 2.0) if P.p != 2.0 else np.ones(G.shape[1:])
    Gn = P.vgrad(nu)
    return nu - P.s * P.vdiv(R[None] * Gn) + P.s * P.eps ** 2 * P.lap(P.lap(nu))


def pcg_Lk(P: "Problem", u, r, rtol: float = 0.0, iters: int = 20):
    """Preconditioned conjugate gradients for L_k d = r from d = 0 (textbook form,
    preconditioner L_h^{-1}): stops after `iters` iterations, or earlier when
    ||res||_2 <= rtol ||r||_2 (rtol > 0).  Returns (d, iterations)."""
    d = np.zeros_like(r)
    res = r.copy()
    z = P.precond(res)
    pdir = z.copy()
    rz = P.ip(res, z)
    r0 = np.sqrt(P.ip(r, r))
    k = 0
    while k < iters:
        Ap = apply_Lk(P, u, pdir)
        a = rz / P.ip(pdir, Ap)
        d = d + a * pdir
        res = res - a * Ap
        k += 1
        if rtol > 0 and np.sqrt(P.ip(res, res)) <= rtol * r0:
            break
        z = P.precond(res)
        rz_new = P.ip(res, z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return d, k


def _root(qfun, c0: float, c1: float) -> float:
    """Root of the increasing q (Sec. 6.1) by the rule of the oracle's C solve:
    x = -c0/c1, double until q > 0, then Newton with bisection when a step
    leaves the bracket; stop at |q| <= 1e-16 (|c0| + c1 x) or |dx| <= 1e-15 x."""
    lo, hi, x = 0.0, np.inf, -c0 / c1
    for _ in range(200):
        q, dq = qfun(x)
        if q > 0:
            hi = x
            break
        if q == 0:
            return x
        lo, x = x, 2 * x
    for _ in range(100):
        if abs(q) <= 1e-16 * (abs(c0) + c1 * x):
            break
        xn = x - q / dq
        if not (lo < xn < hi):
            xn = 0.5 * (lo + hi)
        if abs(xn - x) <= 1e-15 * x:
            return xn
        x = xn
        q, dq = qfun(x)
        if q > 0:
            hi = x
        elif q < 0:
            lo = x
        else:
            break
    return x


def solve_variable_metric(P: "Problem", f, u0=None, tol: float = 1e-10, max_iter: int = 200,
                          inner_rtol: float = 0.0, inner_iters: int = 20):
    """PSD with the variable metric L_k (order 4): d = L_k^{-1} r by PCG (fixed
    count when inner_rtol = 0), the exact line search of Sec. 6.1, u += alpha d.
    Returns dict(u, iters, res_inf, alphas, inner, res0, res_hist) with res_hist
    the max-norm residual after each update and res0 the initial one."""
    assert P.order == 4
    f = _arr(f)
    u = np.zeros_like(f) if u0 is None else _arr(u0).copy()
    r = P.residual(f, u)
    res0 = float(np.abs(r).max())
    alphas, inner, res_hist = [], [], []
    k = 0
    while np.abs(r).max() > tol and k < max_iter:
        d, m = pcg_Lk(P, u, r, inner_rtol, inner_iters)
        c0 = -P.ip(r, d) / P.hd
        if P.p == 4.0:
            c = P.ls_coeffs4(u, d, r)
            alpha, _ = root_cubic(c)
        else:
            _, dq0 = P.q_eval(f, u, d, 0.0)
            alpha = _root(lambda x: P.q_eval(f, u, d, x), c0, dq0)
        u = u + alpha * d
        r = P.residual(f, u)
        k += 1
        alphas.append(alpha)
        inner.append(m)
        res_hist.append(float(np.abs(r).max()))
    return dict(u=u, iters=k, res_inf=float(np.abs(r).max()), alphas=np.array(alphas), inner=inner,
                res0=res0, res_hist=np.array(res_hist))


# ---------------------------------------------------------------------------
# Adjoint of the converged sixth-order solve (Sec. 4 and 5.4).  With
# u = mean(g) + nu (nu mean-zero) the solution satisfies
#   F(nu) = P0[s lam u - s div_h(|grad_h u|^{p-2} grad_h u) + s eps^2 Delta_h^2 u
#           + T_h(nu - g) - f] = 0,
# whose Jacobian H (the Hessian of E_h on mean-zero functions) is symmetric
# positive definite.  For a loss J(u) with plain partials G = dJ/du:
#   Lam = H^{-1} P0 G,  dJ/df = Lam,  dJ/dg = sum(G)/N + T_h Lam,
#   dJ/ds = -Lam.(lam u - div_h(...) + eps^2 Delta_h^2 u),
#   dJ/deps = -Lam.(2 s eps Delta_h^2 u),  dJ/dlam = -s Lam.u.
# ---------------------------------------------------------------------------
def hessvec6(P: "Problem", u, xi) -> np.ndarray:
    """H xi = P0[s lam xi - s (linearised p-Laplacian at u) xi + s eps^2 Delta_h^2 xi + T_h xi]."""
    xi = _arr(xi) - float(np.mean(xi))
    out = (P.s * P.lam * xi - P.s * P.plap_lin(u, xi) + P.s * P.eps ** 2 * P.lap(P.lap(xi)) + P.T(xi))
    return out - float(np.mean(out))


def _precond6(P: "Problem", r) -> np.ndarray:
    """z = L_h^{-1} r for the sixth-order preconditioner of Sec. 5.4, symbol
    s lam + s kappa + s eps^2 kappa^2 + 1/kappa (kappa the symbol of -Delta_h),
    zero mode set to 0 (numpy FFT)."""
    kap = P.symbol_neglap()
    sig = np.full_like(kap, np.inf)
    nz = kap > 0
    sig[nz] = P.s * P.lam + P.s * kap[nz] + P.s * P.eps ** 2 * kap[nz] ** 2 + 1.0 / kap[nz]
    return np.fft.ifftn(np.fft.fftn(r) / sig).real


def adjoint6(P: "Problem", u, G, rtol: float = 1e-13, max_iter: int = 2000):
    """Adjoint of the converged sixth-order solve (see above): preconditioned
    conjugate gradients for H Lam = P0 G.  Returns dict(dJdf, dJdg, dJds,
    dJdeps, dJdlam, iters)."""
    assert P.order == 6
    u, G = _arr(u), _arr(G)
    b = G - float(np.mean(G))
    lam_ = np.zeros_like(b)
    r = b.copy()
    z = _precond6(P, r)
    p = z.copy()
    rz = float((r * z).sum())
    nb = float(np.sqrt((b * b).sum()))
    k = 0
    while k < max_iter and np.sqrt((r * r).sum()) > rtol * nb:
        Hp = hessvec6(P, u, p)
        a = rz / float((p * Hp).sum())
        lam_ += a * p
        r -= a * Hp
        z = _precond6(P, r)
        rz_new = float((r * z).sum())
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
    d2 = P.lap(P.lap(u))
    dNds = P.lam * u - P.plap(u) + P.eps ** 2 * d2
    return dict(dJdf=lam_, dJdg=float(G.sum()) / G.size + P.T(lam_),
                dJds=-float((lam_ * dNds).sum()), dJdeps=-float((lam_ * 2 * P.s * P.eps * d2).sum()),
                dJdlam=-P.s * float((lam_ * u).sum()), iters=k)
