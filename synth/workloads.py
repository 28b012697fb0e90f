"""Workload definitions: grid sizes, macro step H, number of macro steps.

H follows the rule "a fixed fraction of the stability limit":
H = frac * ISB / rho with rho = c_max * sigma * sqrt(d) / dx the spectral
radius of the centred-difference operator (sigma = max over theta of the
1-D symbol s(theta)).  The two constants below are rounded in the safe
direction; a test recomputes both with the oracle.
"""
import math

from . import schemes

ISB_ORDER8_K6 = 8.0165        # imaginary stability boundary of ORDER8_K6 (exact 8.016569...)
ISB_SQUARE4 = 3.3635          # of SQUARE4_2_4 (exact 3.36358...)
SIGMA_FD4 = 1.3722221         # max of (8 sin t - sin 2t)/6      (exact 1.37222201...)
SIGMA_FD8 = 1.7305985         # same for the 8th-order stencil  (exact 1.73059838...)


def stable_H(isb, c_max, dx, d, sigma, frac=0.8):
    return frac * isb * dx / (c_max * sigma * math.sqrt(d))


# 1-D advection, M = 256, FD4, square order 4, t = 1 in 131 macro steps
# (131 is the smallest count with H = 1/n below 0.8 of the limit).
CONFIG_ADVECTION1D = dict(name="advection1d_m256_square4", m=256, r=2,
                          scheme=schemes.SQUARE4_2_4, H=1.0 / 131, n_macro=131)

# 2-D acoustic, 2048^2, constant c = 1, FD4, order 8 over {2..12}, 500 macro steps.
CONFIG_ACOUSTIC2D = dict(name="acoustic2d_2048_fd4_order8_k6", n=2048, r=2, c2=1.0,
                         scheme=schemes.ORDER8_K6,
                         H=stable_H(ISB_ORDER8_K6, 1.0, 1.0 / 2048, 2, SIGMA_FD4),
                         n_macro=500)


# 64 independent 2-D acoustic instances, square sizes drawn from
# {256, 512, 768, 1024}, log-normal c (sigma 0.2, correlation length 0.1,
# seed 1000 + instance), order 8 over {2..12}, H at 0.8 of each instance's
# limit, 100 macro steps.
CONFIG_BATCH = dict(name="batch64_acoustic2d_lognormal_order8_k6", count=64,
                    sizes=(256, 512, 768, 1024), size_seed=0, field_seed=1000, sigma=0.2,
                    ell=0.1, r=2, scheme=schemes.ORDER8_K6, n_macro=100)


def batch_instances(cfg=CONFIG_BATCH):
    """[(n, c (speed field), H)] for the batch workload."""
    from . import fields
    out = []
    for i, n in enumerate(fields.batch_sizes(cfg["count"], cfg["sizes"], cfg["size_seed"])):
        c = fields.lognormal_speed((n, n), sigma=cfg["sigma"], ell=cfg["ell"],
                                   seed=cfg["field_seed"] + i)
        H = stable_H(ISB_ORDER8_K6, float(c.max()), 1.0 / n, 2, SIGMA_FD4)
        out.append((n, c, H))
    return out


# Differentiation: 2-D acoustic 1024^2, log-normal c^2 (seed 40), one Ricker
# source at the centre, 128 receivers on the row n/32, 400 macro steps,
# checkpoints every 20; data from c^2 * exp(0.1 g') (seed 41).
CONFIG_ADJOINT = dict(name="adjoint_acoustic2d_1024_order8_k6", n=1024, r=2, n_macro=400,
                      checkpoint_every=20, speed_seed=40, data_seed=41, receivers=128,
                      scheme=schemes.ORDER8_K6)

# 3-D acoustic 384^3, FD8, band-limited log-normal c (seed 50; the 96^3
# parity grid samples the same field every 4th point), 8 right-hand sides
# each with one Ricker point source at seeded positions on the 96-point
# lattice, FP32 stepping with the FP64 combination, 100 macro steps; the
# gradient: 128 receivers per right-hand side on the plane z = n/32, data from
# c^2 exp(0.1 g') (g' seed 52), checkpoints every 20 macro steps.
CONFIG_3D = dict(name="acoustic3d_384_fd8_order8_k6_rhs8", n=384, r=4, n_rhs=8, n_macro=100,
                 speed_seed=50, source_seed=51, data_seed=52, kmax=12, receivers=128,
                 checkpoint_every=20, scheme=schemes.ORDER8_K6)


def sources_3d(n, count=8, seed=51, lattice=96):
    """``count`` distinct seeded points (z, y, x) of the ``lattice``-point grid,
    in [lattice/8, 7 lattice/8) per axis, scaled to an n-point grid (n a
    multiple of ``lattice``)."""
    import numpy as np
    if n % lattice:
        raise ValueError("n must be a multiple of the lattice size")
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < count:
        p = tuple(int(v) for v in rng.integers(lattice // 8, lattice - lattice // 8, size=3))
        if p not in pts:
            pts.append(p)
    m = n // lattice
    return [(z * m, y * m, x * m) for z, y, x in pts]
