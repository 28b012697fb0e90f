"""The extrapolated GBS macro step, literally (oracle, test infrastructure
only).

Sect. 2.1, eq. (GBS): over a macro step H with N substeps h = H/N,
    y_1 = y_0 + h f(t_0, y_0)                          (forward Euler)
    y_{n+1} = y_{n-1} + 2h f(t_n, y_n),  n = 1..N      (leap-frog)
    y*_N = (y_{N-1} + 2 y_N + y_{N+1}) / 4             (averaging)
with t_n = t_0 + n h.  Sect. 3.2: m such sequences with step counts n_i run
independently and are combined as y_out = sum_i c_i y*_i.  Sect. 3.6: the first
evaluation f(t_0, y_0) is the same for every sequence and is computed once.

The combination is accumulated in FP64 in ascending order of N.
"""
import numpy as np


def sequence(f, t0, y0, f0, h, n):
    """One GBS sequence with n substeps of size h; f0 = f(t0, y0).
    Returns y*_n."""
    y_prev = y0
    y_cur = y0 + h * f0
    y_prevprev = None
    for k in range(1, n + 1):
        y_next = y_prev + 2.0 * h * f(t0 + k * h, y_cur)
        y_prevprev, y_prev, y_cur = y_prev, y_cur, y_next
    # now y_prevprev = y_{n-1}, y_prev = y_n, y_cur = y_{n+1}
    return (y_prevprev + 2.0 * y_prev + y_cur) / 4.0


def macro_step(f, t0, y0, H, steps, c):
    """One extrapolated macro step.  ``steps`` and ``c`` are parallel lists;
    c are floats (the FP64-rounded weights)."""
    y0 = np.asarray(y0) * 1.0            # FP64 (or complex128 for scalar tests)
    f0 = f(t0, y0)
    order = sorted(range(len(steps)), key=lambda i: steps[i])
    out = None
    for i in order:
        n = steps[i]
        ys = sequence(f, t0, y0, f0, H / n, n)
        term = c[i] * ys
        out = term if out is None else out + term
    return out


def integrate(f, t0, y0, H, n_macro, steps, c, callback=None):
    """n_macro macro steps from (t0, y0); callback(n, t, y) after each."""
    y = np.asarray(y0) * 1.0
    t = t0
    for n in range(1, n_macro + 1):
        y = macro_step(f, t, y, H, steps, c)
        t = t0 + n * H
        if callback is not None:
            callback(n, t, y)
    return y
