"""Tolerances shared by the GPU parity tests, derived from the arithmetic.

Step sizes.  The GPU and the oracle follow the same iterate sequence; they
differ by rounding only.  The residual r = f - N_h[u] is a difference of
terms as large as R = max|u| + s max|div_h(...)| + s eps^2 max|Delta_h^2 u|,
so each side carries an absolute error of a few units of 2^-52 R in r, hence
in d = L_h^{-1} r and in the coefficients of q (Sec. 6.1), whose root alpha_k
is (to first order) -q(0)/q'(0) = (r, d)/q'(0).  Its relative error is
therefore about eps_mach R / ||r_{k-1}||: tight while the residual is large,
loose near the tolerance.  On top of that, the coefficients of q are sums
over the N cells, which the oracle adds one after the other and the GPU in a
tree: their relative difference behaves like sqrt(N) eps_mach (random-walk
model of the rounding).  The bound used is

    |alpha_gpu - alpha_oracle|
        <= (SUM_K sqrt(N) eps_mach + ALPHA_K eps_mach R / ||r_{k-1}||_inf) alpha_oracle

with ||r_{k-1}||_inf the oracle's residual before update k.
"""
from __future__ import annotations

import numpy as np

EPS_MACH = 2.0 ** -52
ALPHA_K = 64.0
SUM_K = 16.0


def rounding_scale(O, u, w=None) -> float:
    """R = max|u| + s max|div_h(|grad u|^{p-2} grad u)| + s eps^2 max|Delta_h^2 u|
    (oracle operators).  Order 6 (Sec. 5.4): s lam max|u| in place of max|u|,
    plus max|w| for the T_h term."""
    lin = O.s * O.lam * np.abs(u).max() + np.abs(w).max() if O.order == 6 else np.abs(u).max()
    return float(lin + O.s * np.abs(O.plap(u)).max()
                 + O.s * O.eps ** 2 * np.abs(O.lap(O.lap(u))).max())


def alpha_tolerance(res_before, alpha_ref, scale, ncell):
    """Per-update absolute tolerance of alpha_k (see the module docstring)."""
    res_before = np.asarray(res_before, dtype=np.float64)
    floor = SUM_K * np.sqrt(ncell) * EPS_MACH
    return (floor + ALPHA_K * EPS_MACH * scale / res_before) * np.abs(alpha_ref)


def check_alphas(alpha_gpu, alpha_ref, res_ref, res0, scale, ncell, log=print):
    """Compare the common prefix of two step-size histories with the per-k
    bound; res_ref[k] is the oracle residual after update k, res0 before
    the first, ncell the number of cells.  Returns the worst ratio
    |diff| / bound."""
    k = min(len(alpha_gpu), len(alpha_ref))
    assert k > 0, "empty step-size history"
    a_g = np.asarray(alpha_gpu[:k], dtype=np.float64)
    a_o = np.asarray(alpha_ref[:k], dtype=np.float64)
    before = np.concatenate([[res0], np.asarray(res_ref[:k - 1], dtype=np.float64)])
    tol = alpha_tolerance(before, a_o, scale, ncell)
    diff = np.abs(a_g - a_o)
    ratio = diff / tol
    # per-step ratios to each term of the model
    rel = diff / np.abs(a_o)
    log(f"  alpha: {k} steps, worst |diff|/bound {ratio.max():.3g}; per step "
        f"rel/(sqrt(N) eps) {np.array2string(rel / (np.sqrt(ncell) * EPS_MACH), precision=2)}, "
        f"rel/(eps R/r) {np.array2string(rel / (EPS_MACH * scale / before), precision=2)}")
    assert (diff <= tol).all(), (diff, tol)
    return float(ratio.max())
