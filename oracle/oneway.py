"""The paper's numerical experiment (Sect. 4.1), oracle side (test
infrastructure only).

The periodic one-way wave equation u_t + u_x = 0 on [0,1) with
u(x, 0) = (1 - cos 2 pi x) / 2, discretised in space by the Fourier
derivative on M points (operators.SpectralAdvection1D), run once around
the interval (t = 1) near the stability limit, lambda = dt/dx = 0.99 ISB/pi
(pi M is the spectral radius of the Fourier derivative), and compared with
the analytic solution u(x, 1) = u(x, 0).

Readings (the paper leaves them open):
* one revolution in an integer number of macro steps: n = ceil(pi M /
  (0.99 ISB)), H = 1/n, i.e. at or just below 0.99 of the limit;
* the error is the maximum over the M grid points of |u_n - u(., 1)|;
* "truncation to double precision" of the weights is read as keeping 16
  significant decimal digits (round_sig): that reading reproduces both printed
  floors, 1e-14 (order 8) and 1e-12 (order 12), while rounding to the nearest
  binary double leaves the order-12 floor near 1e-13.

Two evaluations of the same experiment:
* run / run_rk4: the literal FP64 time steppers (gbs.integrate, rk4.integrate)
  on the FFT derivative;
* error_closed_form: the fully discrete solution in extended precision
  (mpmath).  The initial data holds Fourier modes 0 and +-1 only, on which
  the Fourier derivative is exact (multiplication by 0 and -+2 pi i), so
  after n steps mode k is multiplied by R(-2 pi i k H)^n, R the stability
  polynomial of the method (App. A/B) built exactly from the weights given.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np

from . import gbs as G
from . import operators as OP
from . import rk4 as RK
from . import stability as S


def initial(m):
    x = np.arange(m) / m
    return (0.5 * (1.0 - np.cos(2.0 * np.pi * x))).reshape(1, m)


def macro_steps(m, isb, frac=0.99):
    """(n, H): one revolution in n steps at or below frac * ISB / (pi M)."""
    n = math.ceil(math.pi * m / (frac * isb))
    return n, 1.0 / n


def run(m, steps, c, n):
    """Literal FP64 extrapolated GBS over one revolution in n macro steps;
    returns (u_n, max error against the analytic solution)."""
    u0 = initial(m)
    u = G.integrate(OP.SpectralAdvection1D(m), 0.0, u0, 1.0 / n, n, steps, c)
    return u, float(np.max(np.abs(u - u0)))


def run_rk4(m, n):
    u0 = initial(m)
    u = RK.integrate(OP.SpectralAdvection1D(m), 0.0, u0, 1.0 / n, n)
    return u, float(np.max(np.abs(u - u0)))


def error_closed_form(m, poly, n, dps=60):
    """Max over grid points of |u_n - u(., 1)| for a method with stability
    polynomial ``poly`` (ascending exact coefficients in xi = H lambda) and
    n steps of H = 1/n, evaluated at ``dps`` decimal digits."""
    with mp.workdps(dps):
        coef = [mp.mpf(Fraction(a).numerator) / Fraction(a).denominator for a in poly]
        r0 = S.poly_eval(coef, mp.mpf(0)) ** n
        g = S.poly_eval(coef, -2j * mp.pi / n) ** n          # mode +1: lambda = -2 pi i
        # u_n = r0/2 - (g e^{2 pi i x} + conj) / 4 against u_0 = 1/2 - cos(2 pi x)/2
        err = max(abs((r0 - 1) / 2 - mp.re((g - 1) * mp.expjpi(2 * mp.mpf(i) / m)) / 2)
                  for i in range(m))
        return float(err)


def solution_closed_form(m, poly, n, dps=60):
    """u_n at the M grid points (extended precision, rounded to FP64 at the
    end) for a method with stability polynomial ``poly`` and n steps."""
    with mp.workdps(dps):
        coef = [mp.mpf(Fraction(a).numerator) / Fraction(a).denominator for a in poly]
        r0 = S.poly_eval(coef, mp.mpf(0)) ** n
        g = S.poly_eval(coef, -2j * mp.pi / n) ** n
        return np.array([[float(r0 / 2 - mp.re(g * mp.expjpi(2 * mp.mpf(i) / m)) / 2)
                          for i in range(m)]])


def gbs_poly(steps, c):
    """R(xi) = sum_j c_j P_{N_j}(xi) with the weights taken exactly as given
    (Fractions, or floats at their binary values)."""
    return S.extrapolated_poly(steps, [Fraction(x) for x in c])


def round_sig(c, digits):
    """Weights rounded to ``digits`` significant decimal digits, exactly."""
    out = []
    for x in c:
        x = Fraction(x)
        if x == 0:
            out.append(x)
            continue
        with mp.workdps(digits + 30):
            s = mp.nstr(mp.mpf(x.numerator) / x.denominator, digits, min_fixed=1, max_fixed=0)
        out.append(Fraction(s))
    return out
