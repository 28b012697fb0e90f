"""Imaginary-axis stability optimisation of the free weights (oracle, test
infrastructure only).

App. B, eqs. (problem1), (cvx_subproblem), (reformulated_problem): maximise the
step h such that |R(h*lambda)| <= 1 on a contour Lambda, where R = sum c_i P_i
and the order constraints hold exactly.  For a fixed h the inner problem
min_c max_{lambda in Lambda} (|R(h lambda)| - 1) is convex; its optimum
r(h, Lambda) is used inside a bisection over h.

App. B ("Implementing Order Constraints"): the constraints are enforced
exactly by the dep/free split, so R is affine in c_free alone:
R = R_0 + sum_j c_free_j G_j.

Readings taken here (the paper uses CVX / OPTISB, which are not available):
* Lambda is the imaginary segment [0, i] (R has real coefficients, so the
  lower half mirrors it) sampled at ``n_samples`` equispaced points, and h is
  the bisected end point Y of the covered segment [0, iY].
* The modulus constraint |w| <= 1 + t is replaced by the ``n_gon`` half-planes
  Re(e^{-i phi_k} w) <= 1 + t of the circumscribed regular polygon, which makes
  the inner problem a linear programme (solved with HiGHS).  The polygon lets
  |w| reach (1 + t) / cos(pi / n_gon) between its tangent points, so the LP
  may overstate Y slightly; the exact ISB below is what counts.
* A weight vector is only accepted once its exact ISB (stability.isb) has
  been computed from rationals; the LP only proposes it.
* The bisection optimum is tangency-limited: |R| touches 1 at interior points,
  and any polygon or sampling overshoot there ends the exact ISB early.  To
  obtain a usable vector, ``robust`` re-solves the inner problem slightly
  below the bisected Y with the slack weighted by (y/Y)^(p+2) (the order at
  which |R| - 1 can leave zero at the origin), which pushes |R| strictly below
  1 away from the origin.
"""
from fractions import Fraction

import numpy as np
from scipy.optimize import linprog

from . import weights as W
from .stability import gbs_poly_imag_closed_form


def _affine_parts(p, steps, free_idx):
    """Exact decomposition c = a + B c_free (dependent entries from eq.
    cdep_computation, free entries the identity)."""
    m = len(steps)
    nf = len(free_idx)
    base = W.weights(p, steps, free_idx, [0] * nf)
    cols = []
    for j in range(nf):
        e = [0] * nf
        e[j] = 1
        cj = W.weights(p, steps, free_idx, e)
        cols.append([cj[i] - base[i] for i in range(m)])
    return base, cols


def _seq_values(steps, y):
    """P_{n_i}(i y) for every sequence, via the closed form (stable for
    large degree).  Shape (m, len(y))."""
    y = np.asarray(y, dtype=np.float64)
    return np.array([gbs_poly_imag_closed_form(n, y / n) for n in steps])


def minimax(p, steps, free_idx, Y, n_samples=600, n_gon=128, weighted=False):
    """Inner problem for a fixed Y: returns (t, c_free) with
    t = min over c_free of max_s (|R(i y_s)| - 1) / w_s (polygon-approximated),
    w_s = 1, or (y_s / Y)^(p+2) when ``weighted``."""
    base, cols = _affine_parts(p, steps, free_idx)
    ys = np.linspace(Y / n_samples, Y, n_samples)
    pv = _seq_values(steps, ys)                                 # (m, S)
    r0 = np.array([float(x) for x in base]) @ pv                # (S,)
    g = np.array([[float(x) for x in col] for col in cols]) @ pv  # (nf, S)
    nf = len(free_idx)
    phi = 2 * np.pi * np.arange(n_gon) / n_gon
    # Re(e^{-i phi_k} w) <= 1 + t   for every sample and direction
    rot = np.exp(-1j * phi)[:, None]                            # (K, 1)
    a_c = (rot[:, :, None] * g.T[None, :, :]).real              # (K, S, nf)
    a_c = a_c.reshape(-1, nf)
    rhs = (1.0 - (rot * r0[None, :]).real).reshape(-1)
    w = (ys / Y) ** (p + 2) if weighted else np.ones_like(ys)
    a_t = -(np.ones((n_gon, 1)) * w[None, :]).reshape(-1, 1)
    a_ub = np.hstack([a_c, a_t])
    cost = np.zeros(nf + 1)
    cost[-1] = 1.0
    res = linprog(cost, A_ub=a_ub, b_ub=rhs, bounds=[(None, None)] * (nf + 1),
                  method="highs")
    if res.status != 0:
        return np.inf, None
    return res.x[-1], res.x[:nf]


def optimise(p, steps, free_idx, y_hi=None, tol=1e-4, n_samples=600, n_gon=128,
             feas_tol=1e-12):
    """Bisection over Y (eq. reformulated_problem).  Returns (Y, c_free)."""
    if y_hi is None:
        y_hi = float(max(steps) + 1)          # ISB_n <= 1 for explicit schemes
    lo, hi = 0.0, y_hi
    best = None
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        t, cf = minimax(p, steps, free_idx, mid, n_samples, n_gon)
        if t <= feas_tol:
            lo, best = mid, cf
        else:
            hi = mid
    return lo, best


def robust(p, steps, free_idx, y_star, shrink=1e-3, n_samples=2000, n_gon=256):
    """Weighted-slack inner problem at Y = (1 - shrink) * y_star."""
    t, cf = minimax(p, steps, free_idx, (1 - shrink) * y_star, n_samples, n_gon,
                    weighted=True)
    return t, cf


def rationalise(c_free, max_den=10 ** 6):
    """Nearest fractions with bounded denominators (a stand-in for the paper's
    small-integer search, Sect. 3.8)."""
    return [Fraction(float(x)).limit_denominator(max_den) for x in c_free]
