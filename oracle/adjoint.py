"""Discrete adjoint of the extrapolated GBS step for the acoustic system
(oracle, test infrastructure only).

The paper defines only the forward step (Sect. 2.1, eq. GBS; Sect. 3.2, the
combination).  For f(t, y) = A y + s(t) e_src, with A linear in the state
and, through C = diag(c^2), linear in the coefficient field, the exact
transpose of one macro step is obtained by running each sequence's
recurrence backwards:

  forward  y_1 = y_0 + h F_0,  F_0 = f(t_0, y_0)          (shared by all j)
           y_{n+1} = y_{n-1} + 2h f(t_n, y_n),  n = 1..N
           y* = (y_{N-1} + 2 y_N + y_{N+1}) / 4,  y_out = sum_j c_j y*_j
  adjoint  w = c_j ybar_out;  l_{N+1} = w/4, l_N = w/2, l_{N-1} = w/4
           for n = N..1:  l_{n-1} += l_{n+1};  l_n += 2h A^T l_{n+1}
           ybar_0 += l_0 + l_1;   Fbar_0 += h_j l_1
  and finally ybar_0 += A^T Fbar_0 (the shared first evaluation).

The coefficient gradient collects, for every application of A to a state
y_n with factor a (2h for leap-frog, h_j for the shared first evaluation),
a * l_p ⊙ (-div v_n), with l_p the pressure part of the adjoint of the
level that the application produced.

Misfit (receiver residuals at macro-step ends n = 1..n_macro):
  L = 1/2 sum_n sum_r (p_n(x_r) - d_{n,r})^2,
with x_r a grid point of the pressure field in any dimension; a run of
several independent right-hand sides (sharing c^2) sums L and dL/dc^2 over
them (misfit_gradient_rhs).
"""
import numpy as np


def _levels(op, t0, y0, f0, h, n):
    """All levels y_0 .. y_{N+1} of one sequence."""
    ys = [y0, y0 + h * f0]
    for k in range(1, n + 1):
        ys.append(ys[k - 1] + 2.0 * h * op(t0 + k * h, ys[k]))
    return ys


def macro_step_adjoint(op, t0, y0, H, steps, c, ybar_out, want_c2=True):
    """Returns (ybar_0, g_c2) for one macro step started at (t0, y0)."""
    y0 = np.asarray(y0, dtype=np.float64)
    f0 = op(t0, y0)
    ybar0 = np.zeros_like(y0)
    fbar0 = np.zeros_like(y0)
    g = np.zeros(op.shape) if want_c2 else None
    for n, cj in zip(steps, c):
        h = H / n
        ys = _levels(op, t0, y0, f0, h, n)
        lam = [np.zeros_like(y0) for _ in range(n + 2)]
        w = cj * ybar_out
        lam[n + 1] += 0.25 * w
        lam[n] += 0.5 * w
        lam[n - 1] += 0.25 * w
        for k in range(n, 0, -1):
            lam[k - 1] += lam[k + 1]
            lam[k] += 2.0 * h * op.matvec_T(lam[k + 1])
            if want_c2:
                g += 2.0 * h * lam[k + 1][0] * (-op.div(ys[k][1:]))
        ybar0 += lam[0] + lam[1]
        fbar0 += h * lam[1]
    ybar0 += op.matvec_T(fbar0)
    if want_c2:
        g += fbar0[0] * (-op.div(y0[1:]))
    return ybar0, g


def _at(receivers):
    """Index tuple of the receivers' grid points: receivers is an (R, d) array
    whose rows are grid indices in array order ((iy, ix) or (iz, iy, ix))."""
    receivers = np.asarray(receivers, dtype=np.int64)
    return tuple(receivers[:, k] for k in range(receivers.shape[1]))


def misfit(op, t0, y0, H, steps, c, n_macro, receivers, data):
    """Forward run; returns (L, states) with states[n] = y after n macro steps
    (states[0] = y0).  receivers: (R, d) grid indices of the pressure field;
    data: (n_macro, R)."""
    from .gbs import macro_step
    at = _at(receivers)
    ys = [np.asarray(y0, dtype=np.float64)]
    L = 0.0
    for n in range(1, n_macro + 1):
        ys.append(macro_step(op, t0 + (n - 1) * H, ys[-1], H, steps, c))
        res = ys[-1][0][at] - data[n - 1]
        L += 0.5 * float(np.sum(res * res))
    return L, ys


def misfit_gradient(op, t0, y0, H, steps, c, n_macro, receivers, data):
    """Returns (L, dL/dy0, dL/dc2) by the reverse sweep over stored macro-step
    boundary states."""
    L, ys = misfit(op, t0, y0, H, steps, c, n_macro, receivers, data)
    at = _at(receivers)
    ybar = np.zeros_like(ys[0])
    g = np.zeros(op.shape)
    for n in range(n_macro, 0, -1):
        res = ys[n][0][at] - data[n - 1]
        np.add.at(ybar[0], at, res)
        ybar, gn = macro_step_adjoint(op, t0 + (n - 1) * H, ys[n - 1], H, steps, c, ybar)
        g += gn
    return L, ybar, g


def misfit_gradient_rhs(ops, t0, y0s, H, steps, c, n_macro, receivers, data):
    """Several independent right-hand sides r (each its own operator ops[r],
    i.e. its own sources, all with the same c^2; initial state y0s[r];
    receivers[r], data[r] as in misfit_gradient).  Returns
    (sum_r L_r, [dL/dy0_r], sum_r dL_r/dc2)."""
    L, gys, g = 0.0, [], None
    for op, y0, rec, d in zip(ops, y0s, receivers, data):
        Lr, gy, gc = misfit_gradient(op, t0, y0, H, steps, c, n_macro, rec, d)
        L += Lr
        gys.append(gy)
        g = gc if g is None else g + gc
    return L, gys, g
