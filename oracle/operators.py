"""Method-of-lines right-hand sides (oracle, test infrastructure only).

The paper's time stepper acts on y' = f(t, y) obtained from a spatial
discretisation (Sect. 2.1; App. A: for wave-type PDEs the eigenvalues of the
discrete spatial operator lie near the imaginary axis).  The operators here
are periodic centred finite differences on [0,1)^d with grid spacing dx = 1/M,
grid point i at x_i = i*dx, arrays indexed [..., z, y, x] with x fastest.

First-derivative weights come from the Taylor conditions for an antisymmetric
stencil, solved exactly:  D u_i = (1/dx) sum_{k=1..r} a_k (u_{i+k} - u_{i-k})
with sum_k 2 k a_k = 1 and sum_k k^(2l+1) a_k = 0 for l = 1..r-1, which makes
D exact for polynomials of degree <= 2r.
"""
from fractions import Fraction

import numpy as np

from .weights import _solve


def centred_first_derivative_weights(r):
    """Exact a_1..a_r of the order-2r centred first derivative."""
    a = [[Fraction(k) ** (2 * l + 1) for k in range(1, r + 1)] for l in range(r)]
    b = [Fraction(1, 2)] + [Fraction(0)] * (r - 1)
    return _solve(a, b)


def d1(u, axis, dx, r):
    """Periodic centred first derivative of order 2r along ``axis``."""
    a = centred_first_derivative_weights(r)
    out = np.zeros_like(u, dtype=np.float64)
    for k, ak in enumerate(a, start=1):
        out += float(ak) * (np.roll(u, -k, axis=axis) - np.roll(u, k, axis=axis))
    return out / dx


class Source:
    """Point source added to the pressure equation: f_p[idx] += weight * s(t),
    with s the Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
    tau = t - delay.  ``idx`` is a tuple of grid indices of the p field."""

    def __init__(self, idx, f0, delay, weight):
        self.idx, self.f0, self.delay, self.weight = tuple(idx), f0, delay, weight

    def amplitude(self, t):
        a = (np.pi * self.f0 * (t - self.delay)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)


class Advection1D:
    """u_t = -u_x (the paper's one-way wave equation, Sect. 4.1), FD order 2r.
    State shape (1, M)."""

    def __init__(self, m, r=2):
        self.m, self.r, self.dx = m, r, 1.0 / m

    def __call__(self, t, y):
        return -d1(y, axis=-1, dx=self.dx, r=self.r)

    def matvec_T(self, w):
        """A^T w for the linear map f(t, y) = A y."""
        return d1(w, axis=-1, dx=self.dx, r=self.r)


class Acoustic:
    """First-order acoustic system in d = 2 or 3 dimensions:
        p_t = -c^2 div v (+ sources),   v_t = -grad p,
    state fields (p, v_x, v_y[, v_z]); ``c2`` is a scalar or a field of the
    grid's shape.  Stencil order 2r (r = 2: FD4, r = 4: FD8).  ``spacing``:
    the grid spacing per axis in the order of ``shape`` (default 1/n, the
    periodic unit box; a window cut from a larger grid keeps that grid's
    spacing)."""

    def __init__(self, shape, c2=1.0, r=2, sources=(), spacing=None):
        self.shape = tuple(shape)                    # (Y, X) or (Z, Y, X)
        self.d = len(self.shape)
        self.r = r
        self.dx = ([1.0 / n for n in self.shape] if spacing is None
                   else [float(h) for h in spacing])  # per axis, same order as shape
        self.c2 = c2
        self.sources = list(sources)

    def _axes(self):
        # spatial field k (0 = x, 1 = y, 2 = z) lives on array axis -(k+1)
        return [-(k + 1) for k in range(self.d)]

    def div(self, v):
        out = np.zeros(self.shape)
        for k, ax in enumerate(self._axes()):
            out += d1(v[k], axis=ax, dx=self.dx[ax], r=self.r)
        return out

    def __call__(self, t, y):
        p, v = y[0], y[1:]
        f = np.empty_like(y, dtype=np.float64)
        f[0] = -self.c2 * self.div(v)
        for s in self.sources:
            f[0][s.idx] += s.weight * s.amplitude(t)
        for k, ax in enumerate(self._axes()):
            f[1 + k] = -d1(p, axis=ax, dx=self.dx[ax], r=self.r)
        return f

    def linear(self, y):
        """The source-free part A y."""
        save, self.sources = self.sources, []
        try:
            return self(0.0, y)
        finally:
            self.sources = save

    def matvec_T(self, w):
        """A^T w.  With D^T = -D for the periodic centred stencil and
        A = [[0, -C D_x, -C D_y, ...], [-D_x, 0, ...], ...], C = diag(c^2):
        (A^T w)_p = sum_k D_k w_{v_k},  (A^T w)_{v_k} = D_k (c^2 w_p)."""
        out = np.empty_like(w, dtype=np.float64)
        cw = self.c2 * w[0]
        out[0] = 0.0
        for k, ax in enumerate(self._axes()):
            out[0] += d1(w[1 + k], axis=ax, dx=self.dx[ax], r=self.r)
            out[1 + k] = d1(cw, axis=ax, dx=self.dx[ax], r=self.r)
        return out


class SpectralAdvection1D:
    """u_t = -u_x with the Fourier (spectral) first derivative on M points of
    [0,1), the spatial operator of the paper's experiment (Sect. 4.1): the
    derivative of the trigonometric interpolant, i.e. multiplication of DFT
    mode k by 2 pi i k, |k| < M/2; for even M the mode k = M/2 is set to zero
    (its interpolant cos(pi M x) has zero derivative at every grid point).
    State shape (1, M)."""

    def __init__(self, m):
        self.m = m
        k = np.fft.fftfreq(m, 1.0 / m)
        if m % 2 == 0:
            k[m // 2] = 0.0
        self.ik = 2j * np.pi * k

    def derivative(self, u):
        return np.real(np.fft.ifft(self.ik * np.fft.fft(u, axis=-1), axis=-1))

    def __call__(self, t, y):
        return -self.derivative(y)

    def matvec_T(self, w):
        """A^T w: the derivative is skew-symmetric."""
        return self.derivative(w)
