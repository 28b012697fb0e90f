"""Classical fourth-order Runge-Kutta on the same operators (oracle, test
infrastructure only): the comparison method of the paper's Sect. 3.8 and
App. A, whose stability polynomial is the degree-4 Taylor polynomial of exp
(ISB 2 sqrt 2).

    k1 = f(t, y), k2 = f(t + h/2, y + h/2 k1), k3 = f(t + h/2, y + h/2 k2),
    k4 = f(t + h, y + h k3),  y_new = y + h/6 (k1 + 2 k2 + 2 k3 + k4).
"""
import numpy as np


def rk4_step(f, t, y, h):
    y = np.asarray(y) * 1.0
    k1 = f(t, y)
    k2 = f(t + 0.5 * h, y + (0.5 * h) * k1)
    k3 = f(t + 0.5 * h, y + (0.5 * h) * k2)
    k4 = f(t + h, y + h * k3)
    return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def integrate(f, t0, y0, h, n_steps):
    """n_steps steps of size h from (t0, y0); step i starts at t0 + i h."""
    y = np.asarray(y0) * 1.0
    for i in range(n_steps):
        y = rk4_step(f, t0 + i * h, y, h)
    return y
