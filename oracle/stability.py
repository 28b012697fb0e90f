"""Stability polynomials and the imaginary stability boundary (oracle, test
infrastructure only).

App. A: applying a one-step method to y' = lambda*y over one step gives
y_1 = R(xi) y_0 with xi = H*lambda; the stability domain is |R(xi)| <= 1.
App. B: the extrapolated polynomial is R(xi) = sum_i c_i P_i(xi), with P_i the
polynomial of the i-th GBS sequence.
Sect. 2.2: the ISB is the largest Y such that [-iY, iY] lies in the stability
domain (0 if no stretch of the axis is covered); ISB_n divides it by the
function evaluations per step per core, which for folded sequences is
N_max + 1 (Sect. 3.6: N+1 evaluations for the longest sequence, the pairs
folded onto one core add up to the same count).
"""
from fractions import Fraction

import numpy as np


# ---------------------------------------------------------------- polynomials
def _padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def _pscale(a, s):
    return [s * x for x in a]


def gbs_poly(n):
    """Coefficients (ascending powers of xi, exact Fractions) of P_N(xi): the
    GBS sequence of eq. (GBS) applied to y' = lambda*y over a macro step H with
    N substeps, so each substep multiplies f by z = xi/N."""
    if n <= 0 or n % 2:
        raise ValueError("N must be a positive even integer")
    z = [Fraction(0), Fraction(1, n)]          # z = xi / N as a polynomial in xi

    def times_z(a):
        out = [Fraction(0)] * (len(a) + 1)
        for i, x in enumerate(a):
            out[i + 1] += x * z[1]
        return out

    ys = [[Fraction(1)]]                         # y_0 = 1
    ys.append(_padd(ys[0], times_z(ys[0])))      # FE: y_1 = y_0 + z y_0
    for k in range(1, n + 1):                    # LF: y_{k+1} = y_{k-1} + 2 z y_k
        ys.append(_padd(ys[k - 1], _pscale(times_z(ys[k]), 2)))
    # averaging: y* = (y_{N-1} + 2 y_N + y_{N+1}) / 4
    avg = _padd(_padd(ys[n - 1], _pscale(ys[n], 2)), ys[n + 1])
    return _pscale(avg, Fraction(1, 4))


def extrapolated_poly(steps, c):
    """R(xi) = sum_i c_i P_{n_i}(xi) (App. B), exact if c are Fractions."""
    r = [Fraction(0)]
    for n, ci in zip(steps, c):
        r = _padd(r, _pscale(gbs_poly(n), Fraction(ci)))
    return r


def poly_eval(coeffs, x):
    """Evaluate an ascending-coefficient polynomial (Horner), any numeric x."""
    acc = 0
    for a in reversed(coeffs):
        acc = acc * x + a
    return acc


def gbs_poly_imag_closed_form(n, theta):
    """P_N(i*N*theta) for even N, from the characteristic roots of the
    leap-frog recurrence on the imaginary axis (derived, not from the paper):
    with z = i*theta the roots are e^{i phi} and -e^{-i phi}, cos(phi) =
    sqrt(1 - theta^2) (any branch), e^{i phi} = cos(phi) + i*theta, and
        P_N = [(1+cos phi)^2 e^{iN phi} - (1-cos phi)^2 e^{-iN phi}] / (4 cos phi).
    Works for numpy complex or mpmath mpc input."""
    try:
        import mpmath
        if isinstance(theta, (mpmath.mpf, mpmath.mpc)):
            cphi = mpmath.sqrt(1 - theta * theta)
            e = cphi + 1j * theta
            en = e ** n
            return ((1 + cphi) ** 2 * en - (1 - cphi) ** 2 / en) / (4 * cphi)
    except ImportError:  # pragma: no cover
        pass
    theta = np.asarray(theta, dtype=np.complex128)
    cphi = np.sqrt(1 - theta * theta)
    e = cphi + 1j * theta
    en = e ** n
    return ((1 + cphi) ** 2 * en - (1 - cphi) ** 2 / en) / (4 * cphi)


# ------------------------------------------------------------------------ ISB
def _abs2_minus_one(r):
    """|R(iy)|^2 - 1 as a polynomial in u = y^2 with exact coefficients.
    R(iy) = A(y) + i B(y) with A = sum_{k even} r_k (-1)^{k/2} y^k and
    B = sum_{k odd} r_k (-1)^{(k-1)/2} y^k; A^2 + B^2 has only even powers."""
    deg = len(r) - 1
    a = [Fraction(0)] * (deg + 1)
    b = [Fraction(0)] * (deg + 1)
    for k, rk in enumerate(r):
        if k % 2 == 0:
            a[k] = Fraction(rk) * (-1) ** (k // 2)
        else:
            b[k] = Fraction(rk) * (-1) ** ((k - 1) // 2)
    sq = [Fraction(0)] * (2 * deg + 1)
    for i in range(deg + 1):
        if a[i] == 0 and b[i] == 0:
            continue
        for j in range(deg + 1):
            sq[i + j] += a[i] * a[j] + b[i] * b[j]
    sq[0] -= 1
    assert all(sq[k] == 0 for k in range(1, len(sq), 2))
    return [sq[k] for k in range(0, len(sq), 2)]


def isb(r, digits=30):
    """Exact imaginary stability boundary of the real polynomial R (ascending
    coefficients, Fractions or ints).

    Let G(u) = |R(i sqrt u)|^2 - 1 and Q(u) = G(u) / u^m with the largest
    power of u divided out.  If Q(0) > 0, |R| > 1 just off the origin and
    ISB = 0.  Otherwise the axis is covered up to the first positive root of
    Q of odd multiplicity (a root of even multiplicity only touches |R| = 1),
    found by exact real-root isolation.  Returns a float."""
    import sympy
    g = _abs2_minus_one(r)
    if all(x == 0 for x in g):
        return float("inf")
    m = next(i for i, x in enumerate(g) if x != 0)
    q = g[m:]
    if q[0] > 0:
        return 0.0
    u = sympy.Symbol("u")
    poly = sympy.Poly([sympy.Rational(x.numerator, x.denominator) for x in reversed(q)],
                      u, domain="QQ")
    best = None
    _, factors = poly.sqf_list()
    for fac, mult in factors:
        if mult % 2 == 0:
            continue
        for (lo, hi), _k in fac.intervals(eps=sympy.Rational(1, 10 ** digits)):
            if hi <= 0:
                continue
            if lo <= 0 < hi:
                # refine until the interval excludes 0 (a root at u=0 was divided out)
                lo2, hi2 = fac.refine_root(lo, hi, eps=sympy.Rational(1, 10 ** (2 * digits)))
                lo, hi = lo2, hi2
                if hi <= 0:
                    continue
            mid = (sympy.Rational(lo) + sympy.Rational(hi)) / 2
            if best is None or mid < best:
                best = mid
    if best is None:
        return float("inf")
    return float(sympy.sqrt(best).evalf(digits))


def isb_n(steps, r):
    """ISB normalised by N_max + 1 function evaluations per core."""
    return isb(r) / (max(steps) + 1)


def taylor_errors(r, upto):
    """e_k = r_k - 1/k! for k = 0..upto (exact): order p means e_k = 0, k <= p."""
    out = []
    fact = 1
    for k in range(upto + 1):
        if k:
            fact *= k
        rk = Fraction(r[k]) if k < len(r) else Fraction(0)
        out.append(rk - Fraction(1, fact))
    return out


def rk4_poly():
    """Classical RK4 stability polynomial (all 4-stage order-4 RK methods share
    it, App. A): the degree-4 Taylor polynomial of exp."""
    return [Fraction(1), Fraction(1), Fraction(1, 2), Fraction(1, 6), Fraction(1, 24)]
