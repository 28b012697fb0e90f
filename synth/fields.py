"""Seeded initial data, wave-speed fields, sources and receivers.

All grids are periodic on [0,1)^d with point i at x_i = i/M; arrays are
indexed [field][z][y][x] with x fastest, the layout the library expects.
"""
import numpy as np


def advection_modes(m, n_modes=8, kmax=16, seed=0):
    """Sum of ``n_modes`` Fourier modes with distinct wavenumbers drawn from
    1..kmax and N(0,1) cosine and sine amplitudes.  Shape (1, m)."""
    rng = np.random.default_rng(seed)
    ks = rng.choice(np.arange(1, kmax + 1), size=n_modes, replace=False)
    a = rng.standard_normal(n_modes)
    b = rng.standard_normal(n_modes)
    x = np.arange(m) / m
    u = np.zeros(m)
    for k, ak, bk in zip(ks, a, b):
        u += ak * np.cos(2 * np.pi * k * x) + bk * np.sin(2 * np.pi * k * x)
    return u.reshape(1, m)


def oneway_initial(m):
    """u(x, 0) = (1 - cos 2 pi x) / 2 at x_i = i / m, shape (1, m): the
    initial data of the one-way wave experiment (Sect. 4.1)."""
    x = np.arange(m) / m
    return (0.5 * (1.0 - np.cos(2.0 * np.pi * x))).reshape(1, m)


def acoustic2d_pulse_modes(n, n_modes=32, kmax=16, width=0.02, seed=0):
    """Pressure = Gaussian pulse exp(-|x - x0|^2 / (2 w^2)) at x0 = (1/2, 1/2)
    (periodic distance) plus ``n_modes`` plane waves with distinct nonzero
    integer wavevectors in [-kmax, kmax]^2, N(0,1) amplitudes and uniform
    phases; velocity zero.  Shape (3, n, n)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) / n
    dxp = np.minimum(np.abs(x - 0.5), 1 - np.abs(x - 0.5))
    p = np.exp(-(dxp[None, :] ** 2 + dxp[:, None] ** 2) / (2 * width ** 2))
    cand = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
            if (kx, ky) != (0, 0)]
    pick = rng.choice(len(cand), size=n_modes, replace=False)
    amp = rng.standard_normal(n_modes)
    phase = rng.uniform(0, 2 * np.pi, n_modes)
    for (i, a, ph) in zip(pick, amp, phase):
        kx, ky = cand[i]
        p += a * np.cos(2 * np.pi * (kx * x[None, :] + ky * x[:, None]) + ph)
    y = np.zeros((3, n, n))
    y[0] = p
    return y


def gaussian_random_field(shape, ell=0.1, seed=0):
    """Periodic stationary Gaussian field with covariance ~ exp(-r^2/(2 ell^2))
    and unit variance: seeded white noise filtered in Fourier space by the
    square root of the Gaussian spectral density exp(-ell^2 |k|^2 / 2),
    k = 2 pi * integer wavevector."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    filt = np.exp(-0.25 * ell ** 2 * k2)
    g = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    g -= g.mean()
    return g / g.std()


def lognormal_speed(shape, sigma=0.2, ell=0.1, seed=0):
    """c = exp(sigma g) with g from gaussian_random_field."""
    return np.exp(sigma * gaussian_random_field(shape, ell, seed))


def ricker_source_2d(n, c_mean=1.0, cells_per_wavelength=10.0):
    """One Ricker point source at (1/2, 1/2): peak frequency f0 = c / (10 dx),
    delay 1.5 / f0, weight 1 / dx^2 on the p equation.  Returns a dict with the
    grid index (iy, ix), f0, delay and weight."""
    dx = 1.0 / n
    f0 = c_mean / (cells_per_wavelength * dx)
    return dict(idx=(n // 2, n // 2), f0=f0, delay=1.5 / f0, weight=1.0 / dx ** 2)


def edge_receivers_2d(n, count=128, row=None):
    """``count`` receivers along the row y-index ``row`` (default n/32), at
    x-indices spread evenly (n/count apart, offset half a spacing)."""
    row = n // 32 if row is None else row
    step = n // count
    xs = step * np.arange(count) + step // 2
    return np.stack([np.full(count, row), xs], axis=1)


def batch_sizes(count=64, choices=(256, 512, 768, 1024), seed=0):
    """Seeded uniform draw of per-instance square grid sizes."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.array(choices), size=count)]


def bandlimited_lognormal_speed(n, d=3, kmax=12, sigma=0.2, ell=0.1, seed=0):
    """c = exp(sigma g) on an n^d grid, g a periodic Gaussian field made of
    the integer wavevectors |k_i| <= kmax only: complex N(0,1) coefficients
    (seeded, drawn on the (2 kmax + 1)^d cube independently of n) times the
    square root of the spectral density exp(-ell^2 |2 pi k|^2 / 2), real part
    of the inverse FFT, then centred and scaled to unit variance.  For
    n > 2 kmax the grid resolves every product of two modes, so the mean and
    variance, and hence the field values at coincident points, do not depend
    on n: the field on a grid of n / m points per axis is the n-point field
    sampled every m-th point (up to FFT rounding).  ell = 0.1 puts the
    truncated spectrum below 1e-6 of its peak at kmax = 12."""
    rng = np.random.default_rng(seed)
    m = 2 * kmax + 1
    coef = rng.standard_normal((m,) * d) + 1j * rng.standard_normal((m,) * d)
    ks = np.arange(-kmax, kmax + 1)
    k2 = np.zeros((m,) * d)
    for ax in range(d):
        sh = [1] * d
        sh[ax] = m
        k2 = k2 + (2 * np.pi * ks.reshape(sh)) ** 2
    coef = coef * np.exp(-0.25 * ell ** 2 * k2)
    if n <= 2 * kmax:
        raise ValueError("the grid must resolve the field's modes (n > 2 kmax)")
    full = np.zeros((n,) * d, dtype=np.complex128)
    idx = np.ix_(*([ks % n] * d))
    full[idx] = coef
    g = np.real(np.fft.ifftn(full)) * float(n) ** d
    g -= g.mean()
    g /= g.std()
    return np.exp(sigma * g)


def ricker_source_3d(n, points, c_mean=1.0, cells_per_wavelength=10.0):
    """Ricker point sources at the given grid points (z, y, x): peak
    frequency f0 = c / (10 dx), delay 1.5 / f0, weight 1 / dx^3."""
    dx = 1.0 / n
    f0 = c_mean / (cells_per_wavelength * dx)
    return dict(points=list(points), f0=f0, delay=1.5 / f0, weight=1.0 / dx ** 3)


def plane_receivers_3d(n, count=128, z=None):
    """``count`` receivers on the plane z = n/32 (default): a 16 x (count/16)
    lattice of (y, x) points spread evenly.  Returns [(z, y, x)]."""
    z = n // 32 if z is None else z
    nyr = 16 if count >= 16 else count
    nxr = count // nyr
    ys = (n // nyr) * np.arange(nyr) + n // (2 * nyr)
    xs = (n // nxr) * np.arange(nxr) + n // (2 * nxr)
    return [(z, int(y), int(x)) for y in ys for x in xs]
