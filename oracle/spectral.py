"""Closed-form fully discrete propagator for constant coefficients (oracle,
test infrastructure only).

For a linear, source-free f(t, y) = A y the macro step of eq. (GBS) plus the
combination is y_out = R(A) y_0 with R = sum_i c_i P_i (App. B), and P_i built
from the substep h_i (App. A: the step applied to y' = lambda y).  With
periodic centred differences A is diagonalised by the discrete Fourier
transform:

* the centred first derivative acts on exp(i theta j) as multiplication by
  (i/dx) s(theta), s(theta) = 2 sum_k a_k sin(k theta);
* the acoustic symbol A_k = [[0, -c^2 i s^T], [-i s, 0]] (s the vector of
  per-axis symbols) satisfies A_k (A_k^2 + w^2) = 0 with w = c |s|, so any
  function g of it is g(A_k) = I + beta A_k + gamma A_k^2 once g(0) = 1, with
  beta = Im g(i w) / w and gamma = (1 - Re g(i w)) / w^2 (g real on the real
  axis).  Here g = R^n.

R^n is evaluated in extended precision (numpy longdouble) from the exact
weights actually used (the FP64-rounded c, taken at their exact binary
values) and the FP64 substeps h_i = fl(H / N_i), so the result is the fully
discrete solution to FFT rounding, for any n.
"""
from fractions import Fraction

import numpy as np

from .operators import centred_first_derivative_weights
from .stability import gbs_poly


def symbol(m, dx, r):
    """s(theta_k)/dx for the m Fourier modes of a periodic axis."""
    theta = 2 * np.pi * np.fft.fftfreq(m)
    a = centred_first_derivative_weights(r)
    s = np.zeros(m)
    for k, ak in enumerate(a, start=1):
        s += 2 * float(ak) * np.sin(k * theta)
    return s / dx


def _z_coeffs(n):
    """Coefficients of P_N in z = h*lambda (P_N was built in xi = N z)."""
    return [q * Fraction(n) ** k for k, q in enumerate(gbs_poly(n))]


def amplification(lam, H, steps, c, n_macro=1):
    """R(lambda)^n for an array of complex eigenvalues lambda, longdouble."""
    lam = np.asarray(lam).astype(np.clongdouble)
    tot = np.zeros(lam.shape, dtype=np.clongdouble)
    for n, ci in zip(steps, c):
        h = np.longdouble(float(H) / n)          # the FP64 substep, exactly
        z = h * lam
        acc = np.zeros(lam.shape, dtype=np.clongdouble)
        for q in reversed(_z_coeffs(n)):
            acc = acc * z + np.longdouble(q.numerator) / np.longdouble(q.denominator)
        cf = Fraction(float(ci))                   # exact binary value of the FP64 weight
        tot += acc * (np.longdouble(cf.numerator) / np.longdouble(cf.denominator))
    return tot ** n_macro


def advection1d(u0, H, steps, c, n_macro, r=2):
    """u_t = -u_x on M points: y_n = IFFT(R(-i s/dx)^n FFT(y_0))."""
    u0 = np.asarray(u0, dtype=np.float64)
    m = u0.shape[-1]
    lam = -1j * symbol(m, 1.0 / m, r)
    g = amplification(lam, H, steps, c, n_macro)
    uh = np.fft.fft(u0, axis=-1)
    return np.real(np.fft.ifft(uh * g.astype(np.complex128), axis=-1))


def acoustic(y0, c2, H, steps, c, n_macro, r=2):
    """Constant-c acoustic system, y0 of shape (1+d, *grid)."""
    return _acoustic_g(y0, c2, lambda iw: amplification(iw, H, steps, c, n_macro), r)


def rk4_amplification(lam, h, n_steps):
    """(1 + z + z^2/2 + z^3/6 + z^4/24)^n, z = h lambda, longdouble."""
    z = np.longdouble(float(h)) * np.asarray(lam).astype(np.clongdouble)
    one = np.longdouble(1)
    r = one + z * (one + z * (one / 2 + z * (one / 6 + z / 24)))
    return r ** n_steps


def acoustic_rk4(y0, c2, h, n_steps, r=2):
    """n_steps classical RK4 steps of size h, constant-c acoustic system."""
    return _acoustic_g(y0, c2, lambda iw: rk4_amplification(iw, h, n_steps), r)


def acoustic_exact(y0, c2, t, r=2):
    """The semi-discrete solution exp(t A) y0 (constant c)."""
    return _acoustic_g(y0, c2, lambda iw: np.exp(np.longdouble(float(t)) * iw), r)


def _acoustic_g(y0, c2, g_of, r):
    """g(A) y0 for g(0) = 1 real on the real axis, given g at i w."""
    y0 = np.asarray(y0, dtype=np.float64)
    grid = y0.shape[1:]
    d = len(grid)
    axes = tuple(range(1, d + 1))
    yh = np.fft.fftn(y0, axes=axes)
    # per-axis symbols, field k (0 = x) on array axis d - k
    svec = []
    for k in range(d):
        n = grid[d - 1 - k]
        s = symbol(n, 1.0 / n, r)
        shape = [1] * d
        shape[d - 1 - k] = n
        svec.append(np.broadcast_to(s.reshape(shape), grid))
    s2 = sum(sk * sk for sk in svec)
    w = np.sqrt(c2 * s2)
    g = g_of(1j * w.astype(np.longdouble))                     # g(i w)
    wl = w.astype(np.longdouble)
    safe = np.where(wl > 0, wl, np.longdouble(1))
    beta = np.where(wl > 0, g.imag / safe, 0).astype(np.float64)
    gamma = np.where(wl > 0, (1 - g.real) / (safe * safe), 0).astype(np.float64)

    def apply_a(v):
        out = np.empty_like(v)
        out[0] = -c2 * sum(1j * svec[k] * v[1 + k] for k in range(d))
        for k in range(d):
            out[1 + k] = -1j * svec[k] * v[0]
        return out

    a1 = apply_a(yh)
    a2 = apply_a(a1)
    out = yh + beta * a1 + gamma * a2
    return np.real(np.fft.ifftn(out, axes=axes))
