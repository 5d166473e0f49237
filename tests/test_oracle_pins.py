"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here is CPU-only.  The oracle is checked against facts that do not
come from the oracle itself: the expanded stencils printed in Sec. 5.1, the
Fourier symbols of the appendix, closed forms, summation by parts, the
variational identities of Sec. 5.3, brute-force DFTs and library routines.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Problem
import psd_inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def cell_coords(P):
    x = (np.arange(P.n) + 0.5) * P.h
    return np.meshgrid(*([x] * P.dim), indexing="ij")[::-1]  # x varies along last axis


# --------------------------------------------------------------------------
# Fourier transforms (appendix: discrete Fourier expansion, Parseval)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", list(range(1, 17)) + [18, 24, 27, 30])
def test_fft1_matches_bruteforce_and_numpy(n):
    x = rand(n, n) + 1j * rand(n, 100 + n)
    y = oracle.fft1(x, -1)
    yb = oracle.dft1(x, -1)
    yn = np.fft.fft(x)
    scale = max(1.0, np.abs(yn).max())
    assert np.abs(y - yb).max() <= 1e-14 * scale * max(1, math.log2(max(n, 2)))
    assert np.abs(y - yn).max() <= 1e-14 * scale * max(1, math.log2(max(n, 2)))
    xi = oracle.fft1(y, +1) / n
    assert np.abs(xi - x).max() <= 1e-14 * max(1.0, np.abs(x).max()) * max(1, n // 4)


@pytest.mark.parametrize("dim,n", [(2, 6), (2, 8), (2, 12), (3, 4), (3, 6)])
def test_fftn_matches_bruteforce_and_parseval(dim, n):
    x = rand((n,) * dim, 7) + 1j * rand((n,) * dim, 8)
    y = oracle.fftn(x, -1)
    yb = oracle.fftn(x, -1, naive=True)
    assert np.abs(y - yb).max() <= 1e-13
    assert np.abs(y - np.fft.fftn(x)).max() <= 1e-13
    # Parseval: sum |x|^2 = (1/N) sum |X|^2
    N = n ** dim
    assert abs((np.abs(x) ** 2).sum() - (np.abs(y) ** 2).sum() / N) <= 1e-12 * (np.abs(x) ** 2).sum()


# --------------------------------------------------------------------------
# stencils printed in Sec. 5.1
# --------------------------------------------------------------------------

def apply_weights(v, spec, h):
    out = np.zeros_like(v)
    for di, dj, w in spec["weights"]:
        out += w * np.roll(np.roll(v, -di, axis=1), -dj, axis=0)
    return out / h ** spec["power"]


def test_operators_match_printed_stencils_2d():
    gold = json.load(open(os.path.join(GOLD, "stencils_sec5_1.json")))
    P = Problem(2, 12, 3.0, p=2.0)
    v = rand(P.shape, 1)
    tol = 1e-12 * np.abs(v).max() / P.h ** 2
    assert np.abs(P.vgrad_axis(0, v) - apply_weights(v, gold["frakD_x"], P.h)).max() < tol
    assert np.abs(P.vgrad_axis(1, v) - apply_weights(v, gold["frakD_y"], P.h)).max() < tol
    assert np.abs(P.vdiv_axis(0, v) - apply_weights(v, gold["frakd_x"], P.h)).max() < tol
    assert np.abs(P.vdiv_axis(1, v) - apply_weights(v, gold["frakd_y"], P.h)).max() < tol
    assert np.abs(P.lap(v) - apply_weights(v, gold["Delta_h"], P.h)).max() < tol
    # p = 2: the p-Laplacian is the skew Laplacian (Sec. 5.1)
    assert np.abs(P.plap(v) - apply_weights(v, gold["skew_Delta_h"], P.h)).max() < tol


# --------------------------------------------------------------------------
# eigenfunctions and symbols (appendix)
# --------------------------------------------------------------------------

def kappa_closed(P, k):
    return sum(4.0 / P.h ** 2 * math.sin(math.pi * ka / P.n) ** 2 for ka in k)


def kappa_v_closed(P, k):
    th = [2 * math.pi * ka / P.n for ka in k]
    tot = 0.0
    for a in range(P.dim):
        term = 4.0 / P.h ** 2 * math.sin(th[a] / 2) ** 2
        for b in range(P.dim):
            if b != a:
                term *= math.cos(th[b] / 2) ** 2
        tot += term
    return tot


@pytest.mark.parametrize("dim,n,k", [(2, 16, (1, 0)), (2, 16, (3, 5)), (2, 12, (6, 6)),
                                     (2, 10, (2, 7)), (3, 8, (1, 2, 3)), (3, 6, (3, 1, 0))])
def test_eigenfunctions(dim, n, k):
    P = Problem(dim, n, 2.5, p=2.0)
    X = cell_coords(P)
    phase = 0.3
    e = np.cos(sum(2 * math.pi * ka * Xa / P.L for ka, Xa in zip(k, X)) + phase)
    # Delta_h e_k = -kappa e_k
    assert np.abs(P.lap(e) + kappa_closed(P, k) * e).max() < 1e-11 / P.h ** 2
    # frak-d . frak-D e_k = -kappa_v e_k (p = 2 p-Laplacian)
    assert np.abs(P.plap(e) + kappa_v_closed(P, k) * e).max() < 1e-11 / P.h ** 2
    # the oracle's symbols (taken from impulse responses) agree with the closed form
    kap = P.symbol_neglap()
    idx = tuple(k[::-1])
    assert abs(kap[idx] - kappa_closed(P, k)) < 1e-10 / P.h ** 2
    sig = P.symbol_precond()
    kc = kappa_closed(P, k)
    assert abs(sig[idx] - (1 + P.s * kc + P.s * P.eps ** 2 * kc ** 2)) < 1e-10 * (1 + kc) ** 2


def test_difference_symbol_bounds():
    # (2/pi)|nu_l| <= |w_l| <= |nu_l| for |l| <= K, m = 2K+1 (appendix)
    for K in (3, 10, 50):
        m = 2 * K + 1
        L = 3.2
        h = L / m
        for l in range(-K, K + 1):
            w = 2 * abs(math.sin(l * math.pi * h / L)) / h
            nu = 2 * abs(l) * math.pi / L
            assert 2 / math.pi * nu - 1e-12 <= w <= nu + 1e-12


# --------------------------------------------------------------------------
# summation by parts and the variational identities (Sec. 5.1, 5.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n", [(2, 10), (2, 7), (3, 6)])
def test_summation_by_parts(dim, n):
    P = Problem(dim, n, 1.7)
    nu = rand(P.shape, 11)
    for a in range(dim):
        phi = rand(P.shape, 20 + a)  # vertex function
        lhs = P.hd * (P.vgrad_axis(a, nu) * phi).sum()   # <frak-D_a nu, phi>
        rhs = -P.ip(nu, P.vdiv_axis(a, phi))             # -(nu, frak-d_a phi)_2
        assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)
    # Delta_h symmetric, negative semidefinite
    a, b = rand(P.shape, 1), rand(P.shape, 2)
    assert abs(P.ip(P.lap(a), b) - P.ip(a, P.lap(b))) < 1e-10 * abs(P.ip(P.lap(a), b))
    assert P.ip(P.lap(a), a) <= 0


def test_energy_closed_form_one_mode():
    # u = cos(theta i + phi) along x only; f = 0.
    # sum_V |G|^4 = n^{d-1} (2 sin(theta/2)/h)^4 * 3n/8, sum (Delta_h u)^2 = kappa^2 n^d/2
    for dim, n, k in [(2, 16, 3), (3, 8, 1)]:
        P = Problem(dim, n, 2.0, p=4.0, s=0.3, eps=0.2)
        X = cell_coords(P)
        th = 2 * math.pi * k / n
        u = np.cos(2 * math.pi * k * X[0] / P.L + 0.4)
        G4 = n ** (dim - 1) * (2 * math.sin(th / 2) / P.h) ** 4 * 3 * n / 8
        kap = 4 / P.h ** 2 * math.sin(th / 2) ** 2
        E = P.hd * (0.5 * n ** dim / 2 + P.s / 4 * G4 + 0.5 * P.s * P.eps ** 2 * kap ** 2 * n ** dim / 2)
        assert abs(P.energy(np.zeros_like(u), u) - E) < 1e-12 * E


def test_energy6_closed_form_one_mode():
    # Sixth-order discrete energy (Sec. 5.4) at nu = u - gbar on x-only data:
    #   u = gbar + A cos(th i + phi), g = gbar + B cos(th i + psi),
    #   f = fbar + F cos(th i + om).
    # z = nu - g + gbar is one mode of squared amplitude C^2 = A^2 + B^2 - 2AB cos(phi - psi),
    # and T_h z = z / kappa, so
    #   E/h^d = n^d C^2/(4 kappa) + lam s/2 n^d (A^2/2 + gbar^2) - n^d A F cos(phi - om)/2
    #           + s/4 n^(d-1) (2A sin(th/2)/h)^4 3n/8 + s eps^2/2 kappa^2 n^d A^2/2.
    # Every term is non-zero, the gbar^2 term included, and f's mean drops out.
    A, B, F, gbar, fbar = 0.7, 0.4, 0.9, 0.35, -0.6
    phi, psi, om = 0.4, 1.3, -0.8
    for dim, n, k in [(2, 16, 3), (3, 8, 1)]:
        P = Problem(dim, n, 2.0, order=6, p=4.0, s=0.3, eps=0.2, lam=0.7)
        i = np.arange(n, dtype=np.float64)
        th = 2 * math.pi * k / n
        row = lambda amp, ph, c: np.broadcast_to(c + amp * np.cos(th * i + ph), P.shape).copy()
        u, g, f = row(A, phi, gbar), row(B, psi, gbar), row(F, om, fbar)
        kap = 4 / P.h ** 2 * math.sin(th / 2) ** 2
        C2 = A * A + B * B - 2 * A * B * math.cos(phi - psi)
        Nd = n ** dim
        G4 = n ** (dim - 1) * (2 * A * math.sin(th / 2) / P.h) ** 4 * 3 * n / 8
        E = P.hd * (Nd * C2 / (4 * kap) + P.lam * P.s / 2 * Nd * (A * A / 2 + gbar * gbar)
                    - Nd * A * F * math.cos(phi - om) / 2 + P.s / 4 * G4
                    + P.s * P.eps ** 2 / 2 * kap ** 2 * Nd * A * A / 2)
        assert abs(P.energy(f, u, g) - E) < 1e-12 * abs(E)


def test_plap_closed_form_one_mode():
    # 1D-varying data: plap(u)_i = (G_{i+1/2}^3 - G_{i-1/2}^3)/h with
    # G_{i+1/2} = (u_{i+1} - u_i)/h exactly (Sec. 5.1 with constant y).
    P = Problem(2, 16, 2.0, p=4.0)
    th = 2 * math.pi * 3 / P.n
    i = np.arange(P.n)
    Gp = -(2 / P.h) * math.sin(th / 2) * np.sin(th * (i + 0.5) + 0.4)
    Gm = -(2 / P.h) * math.sin(th / 2) * np.sin(th * (i - 0.5) + 0.4)
    expect = (Gp ** 3 - Gm ** 3) / P.h
    u = np.tile(np.cos(th * i + 0.4), (P.n, 1))
    assert np.abs(P.plap(u) - expect[None, :]).max() < 1e-10 * np.abs(expect).max()


@pytest.mark.parametrize("dim,n,p", [(2, 12, 4.0), (2, 9, 3.0), (3, 6, 4.0), (3, 5, 2.5), (2, 8, 6.0)])
def test_gradient_and_hessian_by_central_differences(dim, n, p):
    P = Problem(dim, n, 2.0, p=p, s=0.05, eps=0.3)
    f = rand(P.shape, 3)
    u = rand(P.shape, 4)
    xi = rand(P.shape, 5)
    tau = 1e-4
    # (delta E_h[u], xi)_2 = (N_h[u] - f, xi)_2  (Sec. 5.3)
    dE = (P.energy(f, u + tau * xi) - P.energy(f, u - tau * xi)) / (2 * tau)
    grad = -P.residual(f, u)
    assert abs(dE - P.ip(grad, xi)) < 1e-7 * (abs(dE) + 1)
    # second variation: central difference of the gradient equals H xi
    dg = (-P.residual(f, u + tau * xi) + P.residual(f, u - tau * xi)) / (2 * tau)
    Hxi = P.hessvec(u, xi)
    assert np.abs(dg - Hxi).max() < 1e-6 * np.abs(Hxi).max()
    # symmetric: (H xi, eta) = (xi, H eta)
    eta = rand(P.shape, 6)
    a, b = P.ip(Hxi, eta), P.ip(xi, P.hessvec(u, eta))
    assert abs(a - b) < 1e-11 * abs(a)


def test_sixth_order_gradient_by_central_differences():
    P = Problem(2, 10, 2.0, order=6, p=4.0, s=0.05, eps=0.3, lam=0.7)
    f = rand(P.shape, 3)
    g = rand(P.shape, 4)
    gbar = g.mean()
    u = rand(P.shape, 5)
    u += gbar - u.mean()
    xi = rand(P.shape, 6)
    xi -= xi.mean()  # mean-zero direction
    tau = 1e-4
    dE = (P.energy(f, u + tau * xi, g) - P.energy(f, u - tau * xi, g)) / (2 * tau)
    rho = P.residual(f, u, g)
    assert abs(rho.mean()) < 1e-12
    assert abs(dE + P.ip(rho, xi)) < 1e-7 * (abs(dE) + 1)


def test_preconditioner_solves_its_equation():
    for order in (4, 6):
        P = Problem(2, 12, 2.0, order=order, p=4.0, s=0.05, eps=0.3, lam=0.5)
        r = rand(P.shape, 9)
        if order == 6:
            r -= r.mean()
        d = P.precond(r)
        # L_h d = d - s Delta d + s eps^2 Delta^2 d (+ T_h d) ; order 6: s lam d
        Ld = -P.s * P.lap(d) + P.s * P.eps ** 2 * P.lap(P.lap(d))
        if order == 4:
            Ld += d
        else:
            Ld += P.s * P.lam * d + P.T(d)
            assert abs(d.mean()) < 1e-14
        assert np.abs(Ld - r).max() < 1e-11
        # symmetric (L1)
        r2 = rand(P.shape, 10)
        if order == 6:
            r2 -= r2.mean()
        assert abs(P.ip(P.precond(r), r2) - P.ip(r, P.precond(r2))) < 1e-12
        # T_h inverts -Delta_h on mean-zero functions
        z = rand(P.shape, 12)
        z -= z.mean()
        assert np.abs(-P.lap(P.T(z)) - z).max() < 1e-10


# --------------------------------------------------------------------------
# line search (Sec. 6.1)
# --------------------------------------------------------------------------

def test_cubic_coefficients_reproduce_q():
    for order in (4, 6):
        P = Problem(2, 10, 2.0, order=order, p=4.0, s=0.05, eps=0.3, lam=0.5)
        f = rand(P.shape, 1)
        g = rand(P.shape, 2) if order == 6 else None
        u = rand(P.shape, 3) * 0.3
        if order == 6:
            u += g.mean() - u.mean()
        r = P.residual(f, u, g)
        d = P.precond(r)
        c = P.ls_coeffs4(u, d, r)
        assert c[0] < 0 and c[1] > 0 and c[3] >= 0
        for alpha in (0.0, 0.3, 1.0, 2.7):
            q_direct = -P.ip(P.residual(f, u + alpha * d, g), d) / P.hd
            q_cubic = c[0] + alpha * (c[1] + alpha * (c[2] + alpha * c[3]))
            assert abs(q_direct - q_cubic) < 1e-10 * (abs(c[0]) + abs(c[1]) + abs(c[3]) * 20)
            # the general-p evaluator agrees with the cubic (values and slope)
            q, dq = P.q_eval(f, u, d, alpha, g)
            assert abs(q - q_cubic) < 1e-10 * (abs(c[0]) + abs(c[1]) + abs(c[3]) * 20)
            dq_cubic = c[1] + alpha * (2 * c[2] + 3 * c[3] * alpha)
            assert abs(dq - dq_cubic) < 1e-9 * abs(dq_cubic)


def test_root_rule_on_known_cubics():
    # x^3 + x - 1 = 0 has the single real root (Cardano)
    r = (0.5 + math.sqrt(31 / 108)) ** (1 / 3) + (0.5 - math.sqrt(31 / 108)) ** (1 / 3) * 1.0
    r = np.cbrt(0.5 + math.sqrt(31 / 108)) + np.cbrt(0.5 - math.sqrt(31 / 108))
    x, _ = oracle.root_cubic([-1.0, 1.0, 0.0, 1.0])
    assert abs(x - r) < 1e-15
    # linear: root -c0/c1 exactly
    x, _ = oracle.root_cubic([-3.0, 2.0, 0.0, 0.0])
    assert x == 1.5
    # stiff: tiny linear term, large cubic
    c = [-1e-6, 1e-8, 3e-3, 10.0]
    x, ev = oracle.root_cubic(c)
    roots = np.roots(c[::-1])
    real = roots[np.abs(roots.imag) < 1e-12].real
    assert abs(x - real.max()) < 1e-13 * abs(x)
    assert ev < 200


# --------------------------------------------------------------------------
# the PSD loop: exact p = 2 solutions, linear theory, manufactured solutions
# --------------------------------------------------------------------------

def _kgrid(P):
    ks = np.meshgrid(*([np.arange(P.n)] * P.dim), indexing="ij")[::-1]
    th = [2 * np.pi * k / P.n for k in ks]
    kappa = sum(4 / P.h ** 2 * np.sin(t / 2) ** 2 for t in th)
    kv = np.zeros_like(kappa)
    for a in range(P.dim):
        term = 4 / P.h ** 2 * np.sin(th[a] / 2) ** 2
        for b in range(P.dim):
            if b != a:
                term = term * np.cos(th[b] / 2) ** 2
        kv = kv + term
    return kappa, kv


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 8)])
def test_p2_exact_fourier_solution_order4(dim, n):
    P = Problem(dim, n, 3.2, p=2.0, s=0.01, eps=0.1)
    f = psd_inputs.small_field(dim, n, P.L, 5)
    kappa, kv = _kgrid(P)
    u_exact = np.fft.ifftn(np.fft.fftn(f) / (1 + P.s * kv + P.s * P.eps ** 2 * kappa ** 2)).real
    out = P.solve(f, tol=1e-13, max_iter=200, history=True)
    assert np.abs(out["u"] - u_exact).max() < 1e-12 * np.abs(u_exact).max()
    # linear PSD: c2 = c3 = 0 and the A-norm error contracts by (K-1)/(K+1),
    # K <= 1 + sqrt(s)/(2 eps)  (Sec. 2.1 classical bound)
    K = 1 + math.sqrt(P.s) / (2 * P.eps)
    rate = (K - 1) / (K + 1)
    u = np.zeros_like(f)
    prev = None
    for k in range(6):
        e = u - u_exact
        eA = math.sqrt(P.ip(P.N4(e), e))
        if prev is not None:
            assert eA <= rate * prev * (1 + 1e-9)
        prev = eA
        r = P.residual(f, u)
        d = P.precond(r)
        # q is linear at p = 2: q(alpha) = q(0) + alpha q'(0)
        q0, dq0 = P.q_eval(f, u, d, 0.0)
        q1, dq1 = P.q_eval(f, u, d, 1.0)
        qscale = 1e-14 * np.abs(d).sum() * (1 + np.abs(f).max()) + 1e-10 * (abs(q0) + dq0)
        assert abs(q1 - (q0 + dq0)) < qscale and abs(dq1 - dq0) < 1e-10 * dq0
        alpha_lin = P.ip(d, r) / P.ip(d, P.N4(d))
        alpha = out["hist"][k, 0]
        # q(alpha) is evaluated from its definition, whose absolute rounding is
        # ~ eps * sum|d| * max|f|; divided by q' this bounds the error in alpha
        dalpha = 1e-14 * np.abs(d).sum() * (1 + np.abs(f).max()) / dq0
        assert abs(alpha - alpha_lin) < 1e-12 * alpha_lin + dalpha
        u = u + alpha * d


def test_p2_exact_fourier_solution_order6():
    P = Problem(2, 32, 3.2, order=6, p=2.0, s=0.02, eps=0.1, lam=1.0)
    f = psd_inputs.small_field(2, P.n, P.L, 6) + 0.2
    g = psd_inputs.small_field(2, P.n, P.L, 7) - 0.1
    kappa, kv = _kgrid(P)
    F, Gh = np.fft.fftn(f), np.fft.fftn(g)
    U = np.zeros_like(F)
    W = np.zeros_like(F)
    nz = kappa > 0
    U[nz] = (F[nz] + Gh[nz] / kappa[nz]) / (P.s * P.lam + P.s * kv[nz] + P.s * P.eps ** 2 * kappa[nz] ** 2 + 1 / kappa[nz])
    U[~nz] = Gh[~nz]
    W[nz] = (Gh[nz] - U[nz]) / kappa[nz]
    W[~nz] = P.s * P.lam * Gh[~nz] - F[~nz]
    u_exact, w_exact = np.fft.ifftn(U).real, np.fft.ifftn(W).real
    out = P.solve(f, g=g, tol=1e-13, max_iter=300)
    assert np.abs(out["u"] - u_exact).max() < 1e-12 * np.abs(u_exact).max()
    assert np.abs(out["w"] - w_exact).max() < 1e-11 * np.abs(w_exact).max()


def test_manufactured_solution_paper():
    # Sec. 6.1 complexity test on [0,1]^2: u~ = (1/2pi) sin(2 pi x) cos(2 pi y) cos(s),
    # f = N_h[I_h u~], u0 = u~(.,0) + s^2 sin(4 pi x) sin(6 pi y); stop at gamma_k <= 1e-8.
    n = 64
    P = Problem(2, n, 1.0, p=4.0, s=0.01, eps=0.03)
    X, Y = cell_coords(P)
    ut = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * math.cos(P.s) / (2 * np.pi)
    f = P.N4(ut)
    u0 = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) / (2 * np.pi) + P.s ** 2 * np.sin(4 * np.pi * X) * np.sin(6 * np.pi * Y)
    out = P.solve(f, u0=u0, tol=1e-12, max_iter=200, history=True)
    assert np.abs(out["u"] - ut).max() <= 1e-8
    # gamma_k falls below 1e-8 at some k
    assert out["iters"] < 200


@pytest.mark.parametrize("order", [4, 6])
def test_manufactured_solution_generic(order):
    P = Problem(2, 24, 3.0, order=order, p=4.0, s=0.02, eps=0.1, lam=1.0)
    u_true = psd_inputs.small_field(2, P.n, P.L, 21, amp=0.8)
    if order == 4:
        f = P.N4(u_true)
        out = P.solve(f, tol=1e-12, max_iter=300)
        assert np.abs(out["u"] - u_true).max() < 1e-11
    else:
        w_true = psd_inputs.small_field(2, P.n, P.L, 22, amp=0.5) + 0.3
        gbar = 0.25
        u_true = u_true + gbar
        g = u_true - P.lap(w_true)
        # f = s lam u - s plap(u) + s eps^2 Delta^2 u - w
        f = P.s * P.lam * u_true - P.s * P.plap(u_true) + P.s * P.eps ** 2 * P.lap(P.lap(u_true)) - w_true
        out = P.solve(f, g=g, tol=1e-12, max_iter=300)
        assert np.abs(out["u"] - u_true).max() < 1e-11
        assert np.abs(out["w"] - w_true).max() < 1e-10
        r1, r2 = P.mixed_residuals(f, g, out["u"], out["w"])
        assert np.abs(r1).max() < 1e-10 and np.abs(r2).max() < 1e-10


# --------------------------------------------------------------------------
# per-step invariants and conservation (Sec. 2.3, Sec. 3, Sec. 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,p", [(2, 32, 4.0), (2, 24, 3.0), (3, 10, 4.0)])
def test_descent_orthogonality_and_decay(dim, n, p):
    P = Problem(dim, n, 12.8 * n / 64, p=p, s=0.01, eps=0.1)
    f = psd_inputs.small_field(dim, n, P.L, 31, K=4)
    out = P.solve(f, tol=1e-12, max_iter=200, history=True)
    H = out["hist"]
    alphas, E = H[:, 0], H[:, 3]
    assert (alphas > 0).all()
    E0 = P.energy(f, np.zeros_like(f))
    Es = np.concatenate([[E0], E])
    assert (np.diff(Es) <= 1e-15 * abs(Es).max()).all()
    # geometric decay of the energy gap (Sec. 2.3 theorem): ratios below 1
    gap = Es - Es[-1]
    m = gap > 1e-13 * abs(Es[-1])
    ratios = gap[1:][m[1:]] / gap[:-1][m[1:]]
    assert (ratios < 1).all()
    # orthogonality (Sec. 2.2): after each exact line search (r_{k+1}, d_k) = 0
    u = np.zeros_like(f)
    for k in range(3):
        r = P.residual(f, u)
        d = P.precond(r)
        if p == 4.0:
            alpha, _ = oracle.root_cubic(P.ls_coeffs4(u, d, r))
            c = P.ls_coeffs4(u, d, r)
            dE_pred = P.hd * (c[0] * alpha + c[1] * alpha ** 2 / 2 + c[2] * alpha ** 3 / 3 + c[3] * alpha ** 4 / 4)
            dE = P.energy(f, u + alpha * d) - P.energy(f, u)
            assert abs(dE - dE_pred) < 1e-10 * abs(dE)
        else:
            alpha = H[k, 0]
        rn = P.residual(f, u + alpha * d)
        assert abs(P.ip(rn, d)) < 1e-9 * abs(P.ip(r, d))
        u = u + alpha * d
    # conservation (Sec. 3): mean(u*) = mean(f)
    assert abs(out["u"].mean() - f.mean()) < 1e-13


def test_sixth_order_conservation():
    P = Problem(2, 32, 12.8 / 2, order=6, p=4.0, s=0.02, eps=0.1, lam=1.0)
    f = psd_inputs.small_field(2, P.n, P.L, 41) + 0.1
    g = psd_inputs.small_field(2, P.n, P.L, 42) - 0.2
    out = P.solve(f, g=g, tol=1e-11, max_iter=300)
    assert abs(out["u"].mean() - g.mean()) < 1e-13
    assert abs(out["w"].mean() - (P.s * P.lam * g.mean() - f.mean())) < 1e-13
    r1, r2 = P.mixed_residuals(f, g, out["u"], out["w"])
    assert np.abs(r1).max() < 1e-10 and np.abs(r2).max() < 1e-10


def test_iteration_trends():
    # Sec. 6.1 trends: more iterations for smaller eps, larger s, larger p
    n = 32
    base = dict(dim=2, n=n, L=1.0, p=4.0, s=0.01, eps=0.06)
    f = psd_inputs.small_field(2, n, 1.0, 51, K=4) * 0.2
    it = lambda **kw: Problem(**{**base, **kw}).solve(f, tol=1e-9, max_iter=500)["iters"]
    assert it(eps=0.03) >= it(eps=0.12)
    assert it(s=0.05) >= it(s=0.002)
    assert it(p=6.0) >= it(p=2.0)


def test_mean_mismatch_rejected_order6():
    P = Problem(2, 8, 1.0, order=6, p=4.0, s=0.02, eps=0.1, lam=1.0)
    f = rand(P.shape, 1)
    g = rand(P.shape, 2) + 1.0
    with pytest.raises(RuntimeError):
        P.solve(f, u0=np.zeros(P.shape), g=g)


# --------------------------------------------------------------------------
# adjoint (second variation, Sec. 5.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n", [(2, 8), (3, 4)])
def test_adjoint_matches_dense_hessian_solve(dim, n):
    P = Problem(dim, n, 2.0, p=4.0, s=0.05, eps=0.3)
    u = rand(P.shape, 1) * 0.5
    gu = rand(P.shape, 2)
    m = n ** dim
    H = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        H[:, j] = P.hessvec(u, e.reshape(P.shape)).ravel()
    assert np.abs(H - H.T).max() < 1e-10 * np.abs(H).max()
    lam_dense = oracle.cholesky_solve(H, gu.ravel())
    assert np.allclose(lam_dense, np.linalg.solve(H, gu.ravel()), rtol=1e-10, atol=1e-12)
    out = P.adjoint(u, gu, rtol=1e-14)
    assert np.abs(out["dJdf"].ravel() - lam_dense).max() < 1e-10 * np.abs(lam_dense).max()


def test_adjoint_matches_finite_differences():
    P = Problem(2, 16, 3.2, p=4.0, s=0.01, eps=0.1)
    f = psd_inputs.small_field(2, P.n, P.L, 61)
    ut = psd_inputs.small_field(2, P.n, P.L, 62)

    def J(Pp, ff):
        u = Pp.solve(ff, tol=1e-14, max_iter=500)["u"]
        return 0.5 * Pp.hd * ((u - ut) ** 2).sum(), u

    J0, u = J(P, f)
    gu = P.hd * (u - ut)
    adj = P.adjoint(u, gu, rtol=1e-14)
    tau = 1e-4
    dirn = rand(P.shape, 63)
    fd_f = (J(P, f + tau * dirn)[0] - J(P, f - tau * dirn)[0]) / (2 * tau)
    assert abs(fd_f - (adj["dJdf"] * dirn).sum()) < 1e-6 * abs(fd_f)
    fd_s = (J(P.replace(s=P.s + tau * P.s), f)[0] - J(P.replace(s=P.s - tau * P.s), f)[0]) / (2 * tau * P.s)
    assert abs(fd_s - adj["dJds"]) < 1e-6 * abs(fd_s)
    fd_e = (J(P.replace(eps=P.eps + tau * P.eps), f)[0] - J(P.replace(eps=P.eps - tau * P.eps), f)[0]) / (2 * tau * P.eps)
    assert abs(fd_e - adj["dJdeps"]) < 1e-6 * abs(fd_e)


# --------------------------------------------------------------------------
# convex-splitting time stepping (Sec. 6.1 thin film, Sec. 6.2 SPFC)
# --------------------------------------------------------------------------
def _init_thinfilm(n, L=3.2):
    # the periodic initial data of the Sec. 6.1 convergence test, at cell centres
    x = (np.arange(n) + 0.5) * L / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    return (0.1 * np.sin(2 * np.pi * X / L) ** 2 * np.sin(4 * np.pi * (Y - 1.4) / L)
            - 0.1 * np.cos(2 * np.pi * (X - 2.0) / L) * np.sin(2 * np.pi * Y / L))


def test_thinfilm_step_p2_closed_form():
    # p = 2: N_h = I - s Delta_h^v + s eps^2 Delta_h^2 and f = u^n - s Delta_h^v u^n are
    # diagonal in Fourier space: u^ <- (1 + s kv) u^ / (1 + s kv + s eps^2 k^2) per step
    n, L, nsteps = 32, 3.2, 5
    P = Problem(2, n, L, p=2.0, s=(L / n) ** 2 / 10 * 20, eps=0.1)
    u0 = _init_thinfilm(n, L) + 0.02 * psd_inputs.white_noise((n, n), 5)
    u, its = oracle.thinfilm_steps(P, u0, nsteps, tol=1e-13)
    kappa, kv = _kgrid(P)
    U = np.fft.fftn(u0) * ((1 + P.s * kv) / (1 + P.s * kv + P.s * P.eps ** 2 * kappa ** 2)) ** nsteps
    exact = np.fft.ifftn(U).real
    assert np.abs(u - exact).max() < 1e-12 * np.abs(exact).max()
    assert all(k > 0 for k in its)


def test_spfc_step_p2_closed_form():
    # p = 2 version of the SPFC step: (s g0 + s kv + s eps^2 k^2) u^ - w^ = s g1 k u^n^,
    # u^ + k w^ = u^n^  =>  u^ = u^n^ (s g1 k + 1/k) / (s g0 + s kv + s eps^2 k^2 + 1/k),
    # k != 0; the mean is kept
    n, L, nsteps, g0, g1 = 32, 20.0, 4, 0.5, 2.0
    P = Problem(2, n, L, order=6, p=2.0, s=0.05, eps=1.0, lam=g0)
    u0 = 0.05 * (2 * np.random.default_rng(11).random((n, n)) - 1) + 0.1
    u, w, its = oracle.spfc_steps(P, u0, g1, nsteps, tol=1e-13)
    kappa, kv = _kgrid(P)
    U = np.fft.fftn(u0)
    nz = kappa > 0
    fac = np.ones_like(kappa)
    fac[nz] = (P.s * g1 * kappa[nz] + 1 / kappa[nz]) / (P.s * g0 + P.s * kv[nz] + P.s * P.eps ** 2 * kappa[nz] ** 2
                                                  + 1 / kappa[nz])
    exact = np.fft.ifftn(U * fac ** nsteps).real
    assert np.abs(u - exact).max() < 1e-11 * np.abs(exact).max()


def _thinfilm_energy(P, u):
    # F_h = 1/p ||grad u||_p^p - 1/2 ||grad u||^2 + eps^2/2 ||Delta_h u||^2 with the vertex
    # gradient (its concave part is the one the scheme treats explicitly)
    G2 = (P.vgrad(u) ** 2).sum(axis=0)
    return P.hd * ((G2 ** (P.p / 2)).sum() / P.p - 0.5 * G2.sum() + 0.5 * P.eps ** 2 * (P.lap(u) ** 2).sum())


@pytest.mark.parametrize("p,sfac", [(4.0, 0.1), (4.0, 10.0), (6.0, 1.0)])
def test_thinfilm_energy_decreases(p, sfac):
    # convex splitting (Sec. 6.1): the discrete energy decreases at every step, for any s
    n, L = 32, 3.2
    P = Problem(2, n, L, p=p, s=sfac * (L / n) ** 2, eps=0.1)
    u = _init_thinfilm(n, L)
    E = [_thinfilm_energy(P, u)]
    for _ in range(20):
        u, _ = oracle.thinfilm_steps(P, u, 1, tol=1e-12)
        E.append(_thinfilm_energy(P, u))
    E = np.array(E)
    assert (np.diff(E) <= 1e-13 * np.abs(E).max()).all()
    assert E[-1] < E[0]


def test_spfc_energy_decreases():
    # SPFC energy (Sec. 6.2) with the 5-point gradient in the concave term the scheme
    # treats explicitly: g0/2 ||u||^2 - g1/2 ||D u||^2 + eps^2/2 ||Delta_h u||^2 + 1/4 ||grad u||_4^4
    n, L, g0, g1 = 32, 25.0, 0.5, 2.0
    P = Problem(2, n, L, order=6, p=4.0, s=0.05, eps=1.0, lam=g0)
    u = 0.05 * (2 * np.random.default_rng(12).random((n, n)) - 1)

    def energy(v):
        G2 = (P.vgrad(v) ** 2).sum(axis=0)
        return P.hd * (0.5 * g0 * (v * v).sum() + 0.5 * g1 * (v * P.lap(v)).sum()
                       + 0.5 * P.eps ** 2 * (P.lap(v) ** 2).sum() + 0.25 * (G2 * G2).sum())
    E = [energy(u)]
    for _ in range(15):
        u, _, _ = oracle.spfc_steps(P, u, g1, 1, tol=1e-12)
        E.append(energy(u))
    E = np.array(E)
    assert (np.diff(E) <= 1e-13 * np.abs(E).max()).all()
    assert E[-1] < E[0]


def test_interp_coarse_to_fine_exact_for_linear_in_cell_index():
    # bilinear interpolation reproduces functions linear along each axis away from the
    # periodic seam, and constants everywhere
    c = np.full((8, 8), 3.5)
    assert np.allclose(oracle.interp_coarse_to_fine(c), 3.5, atol=0, rtol=0)
    xc = (np.arange(8) + 0.5) * 2.0          # coarse centres, h_c = 2
    xf = (np.arange(16) + 0.5) * 1.0         # fine centres
    fine = oracle.interp_coarse_to_fine(np.tile(xc, (8, 1)))
    assert np.abs(fine[:, 1:-1] - xf[None, 1:-1]).max() < 1e-14


# --------------------------------------------------------------------------
# variable-metric search direction (Remark in Sec. 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,p", [(2, 10, 4.0), (2, 9, 3.0), (3, 6, 4.0)])
def test_variable_metric_operator_is_spd(dim, n, p):
    P = Problem(dim, n, 2.0, p=p, s=0.05, eps=0.3)
    u = rand(P.shape, 1)
    a, b = rand(P.shape, 2), rand(P.shape, 3)
    La, Lb = oracle.apply_Lk(P, u, a), oracle.apply_Lk(P, u, b)
    assert abs(P.ip(La, b) - P.ip(a, Lb)) < 1e-11 * abs(P.ip(La, b))
    # dense check: symmetric positive definite on a tiny grid (Cholesky succeeds)
    N = P.n ** dim
    A = np.stack([oracle.apply_Lk(P, u, np.eye(N)[k].reshape(P.shape)).ravel() for k in range(N)], axis=1)
    assert np.abs(A - A.T).max() < 1e-10 * np.abs(A).max()
    x = oracle.cholesky_solve(A, a.ravel())
    assert np.abs(A @ x - a.ravel()).max() < 1e-10 * np.abs(a).max()


def test_variable_metric_is_newton_at_p2():
    # p = 2: the frozen coefficient is 1, L_k = N_h, so one direction solves the
    # equation and the exact line search returns alpha = 1
    P = Problem(2, 32, 6.4, p=2.0, s=0.01, eps=0.1)
    f = psd_inputs.small_field(2, 32, 6.4, 8, K=5)
    u = rand(P.shape, 4)
    assert np.abs(oracle.apply_Lk(P, u, f) - P.N4(f)).max() < 1e-12 * np.abs(P.N4(f)).max()
    out = oracle.solve_variable_metric(P, f, tol=1e-11, inner_rtol=1e-14, inner_iters=300)
    assert out["iters"] == 1 and abs(out["alphas"][0] - 1.0) < 1e-10


@pytest.mark.parametrize("p", [4.0, 3.0])
def test_variable_metric_reaches_the_unique_minimiser(p):
    # strictly convex energy (Sec. 3): both metrics converge to the same u*, the
    # energy decreases at every step, and the frozen-coefficient metric needs
    # fewer outer iterations
    n, L = 32, 6.4
    P = Problem(2, n, L, p=p, s=0.01, eps=0.1)
    f = psd_inputs.small_field(2, n, L, 9, K=5)
    ref = P.solve(f, tol=1e-12, max_iter=400)
    out = oracle.solve_variable_metric(P, f, tol=1e-12, inner_rtol=1e-13, inner_iters=300)
    assert np.abs(out["u"] - ref["u"]).max() <= 1e-11 * np.abs(ref["u"]).max()
    assert out["iters"] < ref["iters"]
    # energies along a fixed-count run
    u = np.zeros_like(f)
    E = [P.energy(f, u)]
    for _ in range(4):
        step = oracle.solve_variable_metric(P, f, u0=u, tol=0.0, max_iter=1, inner_iters=8)
        u = step["u"]
        E.append(P.energy(f, u))
    assert (np.diff(E) < 0).all()


# --------------------------------------------------------------------------
# adjoint of the sixth-order solve (Sec. 4, 5.4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_adjoint6_matches_finite_differences(dim, n):
    L, s, eps, lam = 3.2, 0.05, 0.3, 0.7
    f = psd_inputs.small_field(dim, n, L, 31, K=3) + 0.2
    g = psd_inputs.small_field(dim, n, L, 32, K=3) - 0.1
    ut = psd_inputs.small_field(dim, n, L, 33, K=3)
    hd = (L / n) ** dim

    def solve(ff, gg, ss, ee, ll):
        P = Problem(dim, n, L, order=6, p=4.0, s=ss, eps=ee, lam=ll)
        return P.solve(ff, g=gg, tol=1e-13, max_iter=3000)["u"]

    def J(ff, gg, ss, ee, ll):
        u = solve(ff, gg, ss, ee, ll)
        return 0.5 * hd * ((u - ut) ** 2).sum()

    P = Problem(dim, n, L, order=6, p=4.0, s=s, eps=eps, lam=lam)
    u = solve(f, g, s, eps, lam)
    adj = oracle.adjoint6(P, u, hd * (u - ut))
    tau = 1e-5
    df, dg = rand(P.shape, 34), rand(P.shape, 35)
    checks = [
        ((J(f + tau * df, g, s, eps, lam) - J(f - tau * df, g, s, eps, lam)) / (2 * tau), (adj["dJdf"] * df).sum()),
        ((J(f, g + tau * dg, s, eps, lam) - J(f, g - tau * dg, s, eps, lam)) / (2 * tau), (adj["dJdg"] * dg).sum()),
        ((J(f, g, s + tau, eps, lam) - J(f, g, s - tau, eps, lam)) / (2 * tau), adj["dJds"]),
        ((J(f, g, s, eps + tau, lam) - J(f, g, s, eps - tau, lam)) / (2 * tau), adj["dJdeps"]),
        ((J(f, g, s, eps, lam + tau) - J(f, g, s, eps, lam - tau)) / (2 * tau), adj["dJdlam"]),
    ]
    for fd, an in checks:
        assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12


def test_adjoint6_hessian_is_spd_on_mean_zero():
    P = Problem(2, 8, 1.6, order=6, p=4.0, s=0.05, eps=0.3, lam=0.7)
    u = rand(P.shape, 41)
    N = P.n ** 2
    # basis of the mean-zero space: e_k - mean
    E = np.eye(N) - 1.0 / N
    A = np.stack([oracle.hessvec6(P, u, E[k].reshape(P.shape)).ravel() for k in range(N)], axis=1)
    assert np.abs(A - A.T).max() < 1e-10 * np.abs(A).max()
    B = A[:N - 1, :N - 1]     # restriction to N-1 independent mean-zero directions stays SPD
    x = oracle.cholesky_solve(B + 0.0, np.ones(N - 1))
    assert np.all(np.isfinite(x))
