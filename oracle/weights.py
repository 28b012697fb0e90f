"""Extrapolation weights in exact rational arithmetic (oracle, test
infrastructure only).

Paper, Sect. 3.2, eq. (vander): for m sequences with step counts n_i and
substeps h_i = H / n_i, the weights c satisfy the p/2 order constraints

    sum_i c_i h_i^(2k) = [k == 0],      k = 0 .. p/2 - 1.

Dividing row k by H^(2k) gives the same system in n_i^(-2k), so the weights do
not depend on H.  The matrix has p/2 rows and m columns (the paper states both
"p/2 x m" and "m x p/2"; the rows are the order constraints).

Paper, Sect. 3.7, eqs. (order_constraints) and (cdep_computation): with m > p/2
the step counts are split into p/2 dependent and m - p/2 free ones; the free
weights are chosen and the dependent ones follow from

    c_dep = V_dep^{-1} (b - V_free c_free),

computed exactly and only then rounded to floating point.
"""
from fractions import Fraction


def vandermonde(p, steps):
    """Rows k = 0..p/2-1, columns i: n_i^(-2k) as exact Fractions (eq. vander)."""
    if p <= 0 or p % 2:
        raise ValueError("order p must be a positive even integer")
    return [[Fraction(1, n ** (2 * k)) for n in steps] for k in range(p // 2)]


def _solve(a, b):
    """Gaussian elimination with exact Fractions; a is square."""
    n = len(a)
    m = [list(row) + [rhs] for row, rhs in zip(a, b)]
    for col in range(n):
        piv = next((r for r in range(col, n) if m[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular order-constraint system")
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col] / m[col][col]
                m[r] = [x - f * y for x, y in zip(m[r], m[col])]
    return [m[i][n] / m[i][i] for i in range(n)]


def check_steps(steps):
    """Step counts must be positive, even (Sect. 2.1: only then do the odd
    powers of h vanish from the error expansion) and distinct (Sect. 3.2: the
    matrix is invertible only for distinct n_i)."""
    if any(int(n) != n or n <= 0 or n % 2 for n in steps):
        raise ValueError("step counts must be positive even integers")
    if len(set(steps)) != len(steps):
        raise ValueError("step counts must be distinct")


def weights(p, steps, free_idx=(), c_free=()):
    """Exact weights for order p.

    steps    : the m step counts n_i (any order).
    free_idx : positions in ``steps`` whose weights are given (the n_free set).
    c_free   : their values (anything Fraction() accepts: int, str, Fraction,
               or a float, which is taken at its exact binary value).
    Returns a list of m Fractions, c[i] belonging to steps[i].
    """
    check_steps(steps)
    free_idx = list(free_idx)
    if len(free_idx) != len(c_free):
        raise ValueError("free_idx and c_free differ in length")
    m = len(steps)
    dep = [i for i in range(m) if i not in free_idx]
    if len(dep) != p // 2:
        raise ValueError("need exactly p/2 dependent step counts, got %d" % len(dep))
    v = vandermonde(p, steps)
    cf = [Fraction(x) for x in c_free]
    rhs = [Fraction(int(k == 0)) for k in range(p // 2)]
    for k in range(p // 2):
        for j, i in enumerate(free_idx):
            rhs[k] -= v[k][i] * cf[j]
    vdep = [[v[k][i] for i in dep] for k in range(p // 2)]
    cdep = _solve(vdep, rhs)
    c = [Fraction(0)] * m
    for j, i in enumerate(dep):
        c[i] = cdep[j]
    for j, i in enumerate(free_idx):
        c[i] = cf[j]
    return c


def weights_square_closed_form(steps):
    """Square case m = p/2: the Lagrange form of the inverse Vandermonde
    matrix in x_i = n_i^(-2) evaluated at x = 0 gives
    c_i = prod_{j != i} n_i^2 / (n_i^2 - n_j^2)."""
    check_steps(steps)
    c = []
    for i, ni in enumerate(steps):
        w = Fraction(1)
        for j, nj in enumerate(steps):
            if j != i:
                w *= Fraction(ni * ni, ni * ni - nj * nj)
        c.append(w)
    return c


def to_fp64(c):
    """Round each exact weight to the nearest double (Python's int/int
    division is correctly rounded, ties to even)."""
    return [x.numerator / x.denominator for x in c]
