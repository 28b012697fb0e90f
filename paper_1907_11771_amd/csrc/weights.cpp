// Host-side scheme arithmetic: exact order-constraint weights and the
// imaginary stability boundary of the extrapolated polynomial.
//
// Weights (Sect. 3.2, eq. vander; Sect. 3.7, eqs. order_constraints and
// cdep_computation): p/2 constraints sum_i c_i n_i^(-2k) = [k == 0]; the
// dependent weights are solved for exactly, then each weight is rounded once
// to the nearest double.
//
// Stability (App. A, App. B): R(xi) = sum_j c_j P_j(xi) where P_j is one GBS
// sequence applied to y' = lambda y.  The sign of |R(iy)|^2 - 1 next to the
// origin (where it is O(y^(p+2)) and below any floating-point resolution) is
// taken exactly from the lowest non-zero coefficient of that polynomial; the
// first crossing away from the origin is then located in long double by
// running the sequences' recurrences on y' = i y.
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <vector>

#include "bigrat.hpp"
#include "internal.hpp"

namespace gbs {

namespace {

BigInt big_pow(int64_t base, int e) {
  BigInt r(1), b(base);
  for (int i = 0; i < e; ++i) r = r * b;
  return r;
}

}  // namespace

int check_steps(int32_t m, const int32_t* steps) {
  if (m <= 0 || !steps) return fail(GBS_EINVAL, "step counts: null or empty");
  for (int i = 0; i < m; ++i) {
    if (steps[i] <= 0 || steps[i] % 2)
      return fail(GBS_ESTEPS, "step count %d is not a positive even integer", steps[i]);
    for (int j = 0; j < i; ++j)
      if (steps[i] == steps[j]) return fail(GBS_ESTEPS, "step count %d appears twice", steps[i]);
  }
  return GBS_OK;
}

int exact_weights(int32_t p, int32_t m, const int32_t* steps, int32_t n_free,
                  const int32_t* free_idx, const Rational* c_free, std::vector<Rational>& c) {
  if (p <= 0 || p % 2) return fail(GBS_EORDER, "order p = %d must be a positive even integer", p);
  int st = check_steps(m, steps);
  if (st) return st;
  const int rows = p / 2;
  if (m - n_free != rows)
    return fail(GBS_ESTEPS, "need exactly p/2 = %d dependent step counts, have %d", rows, m - n_free);
  std::vector<int> is_free(m, -1);
  for (int j = 0; j < n_free; ++j) {
    if (!free_idx || free_idx[j] < 0 || free_idx[j] >= m || is_free[free_idx[j]] >= 0)
      return fail(GBS_EINVAL, "free_idx[%d] invalid or repeated", j);
    is_free[free_idx[j]] = j;
  }
  std::vector<int> dep;
  for (int i = 0; i < m; ++i)
    if (is_free[i] < 0) dep.push_back(i);
  // V[k][i] = n_i^(-2k); augmented dependent system [V_dep | b - V_free c_free]
  std::vector<std::vector<Rational>> a(rows, std::vector<Rational>(rows + 1));
  for (int k = 0; k < rows; ++k) {
    Rational rhs(k == 0 ? 1 : 0);
    for (int i = 0; i < m; ++i) {
      Rational v(BigInt(1), big_pow(steps[i], 2 * k));
      if (is_free[i] >= 0) rhs = rhs - v * c_free[is_free[i]];
    }
    for (int d = 0; d < rows; ++d) a[k][d] = Rational(BigInt(1), big_pow(steps[dep[d]], 2 * k));
    a[k][rows] = rhs;
  }
  for (int col = 0; col < rows; ++col) {
    int piv = -1;
    for (int r = col; r < rows; ++r)
      if (!a[r][col].is_zero()) { piv = r; break; }
    if (piv < 0) return fail(GBS_ESINGULAR, "order-constraint system is singular");
    std::swap(a[col], a[piv]);
    for (int r = 0; r < rows; ++r) {
      if (r == col || a[r][col].is_zero()) continue;
      Rational f = a[r][col] / a[col][col];
      for (int q = col; q <= rows; ++q) a[r][q] = a[r][q] - f * a[col][q];
    }
  }
  c.assign(m, Rational());
  for (int d = 0; d < rows; ++d) c[dep[d]] = a[d][rows] / a[d][d];
  for (int i = 0; i < m; ++i)
    if (is_free[i] >= 0) c[i] = c_free[is_free[i]];
  return GBS_OK;
}

// Ascending coefficients of P_N(xi): y_0 = 1, y_1 = (1 + z), y_{n+1} =
// y_{n-1} + 2 z y_n, y* = (y_{N-1} + 2 y_N + y_{N+1}) / 4, with z = xi / N.
std::vector<Rational> seq_poly(int n) {
  using Poly = std::vector<Rational>;
  Rational z(BigInt(1), BigInt(n));
  auto add = [](const Poly& x, const Poly& y) {
    Poly r(std::max(x.size(), y.size()));
    for (size_t i = 0; i < r.size(); ++i) {
      if (i < x.size()) r[i] = r[i] + x[i];
      if (i < y.size()) r[i] = r[i] + y[i];
    }
    return r;
  };
  auto times = [&](const Poly& x, const Rational& s, int shift) {
    Poly r(x.size() + shift);
    for (size_t i = 0; i < x.size(); ++i) r[i + shift] = x[i] * s;
    return r;
  };
  Poly ym1{Rational(1)};
  Poly y = add(ym1, times(ym1, z, 1));
  Poly prev = ym1;
  std::vector<Poly> last(3);
  for (int k = 1; k <= n; ++k) {
    Poly nx = add(prev, times(y, z * Rational(2), 1));
    if (k == n) { last[0] = prev; last[1] = y; last[2] = nx; }
    prev = y;
    y = nx;
  }
  Poly avg = add(add(last[0], times(last[1], Rational(2), 0)), last[2]);
  return times(avg, Rational(BigInt(1), BigInt(4)), 0);
}

// Sign of |R(iy)|^2 - 1 next to the origin, exactly: the lowest non-zero
// coefficient of G(u) = |R(i sqrt u)|^2 - 1 (R real, so G has even powers of
// y only).  Returns +1, -1, or 0 when G vanishes identically.
int origin_sign(const std::vector<Rational>& r) {
  const int deg = (int)r.size() - 1;
  std::vector<Rational> a(deg + 1), b(deg + 1);
  for (int k = 0; k <= deg; ++k) {
    if (k % 2 == 0) a[k] = ((k / 2) % 2) ? -r[k] : r[k];
    else b[k] = (((k - 1) / 2) % 2) ? -r[k] : r[k];
  }
  // coefficients of y^e, e = 0, 2, 4, ... in increasing order; stop at the
  // first non-zero one
  for (int e = 0; e <= 2 * deg; e += 2) {
    Rational g = e == 0 ? Rational(-1) : Rational(0);
    for (int i = 0; i <= std::min(e, deg); ++i) {
      const int j = e - i;
      if (j > deg) continue;
      if (!a[i].is_zero() && !a[j].is_zero()) g = g + a[i] * a[j];
      if (!b[i].is_zero() && !b[j].is_zero()) g = g + b[i] * b[j];
    }
    if (!g.is_zero()) return g.sign();
  }
  return 0;
}

// |R(iy)|^2 - 1 in long double, with R(iy) = sum_j c_j P_j(iy) and P_j run
// as the GBS recurrence itself on y' = i y (z = i y / N_j); *bound is a
// rounding bound for the result.
long double g_numeric(int k, const int32_t* steps, const std::vector<long double>& c,
                      long double y, long double* bound) {
  using C = std::complex<long double>;
  C R(0, 0);
  long double mag = 0;
  int nmax = 0;
  for (int j = 0; j < k; ++j) {
    const int n = steps[j];
    nmax = std::max(nmax, n);
    const C z(0, y / n);
    C ym1(1, 0), yc = ym1 + z * ym1, ynm1, yn, yn1;
    C prev = ym1, cur = yc;
    for (int s = 1; s <= n; ++s) {
      C nx = prev + 2.0L * z * cur;
      if (s == n) { ynm1 = prev; yn = cur; yn1 = nx; }
      prev = cur;
      cur = nx;
    }
    const C ps = 0.25L * (ynm1 + 2.0L * yn + yn1);
    R += c[j] * ps;
    mag += fabsl(c[j]) * (std::abs(ynm1) + 2 * std::abs(yn) + std::abs(yn1)) * 0.25L;
  }
  *bound = 64 * (nmax + 2) * std::numeric_limits<long double>::epsilon() * mag * (1 + mag);
  return std::norm(R) - 1;
}

double isb_of(int k, const int32_t* steps, const std::vector<Rational>& c) {
  std::vector<Rational> r;
  int nmax = 0;
  for (int j = 0; j < k; ++j) {
    std::vector<Rational> pj = seq_poly(steps[j]);
    if (r.size() < pj.size()) r.resize(pj.size());
    for (size_t i = 0; i < pj.size(); ++i) r[i] = r[i] + c[j] * pj[i];
    nmax = std::max(nmax, (int)steps[j]);
  }
  const int s0 = origin_sign(r);
  if (s0 == 0) return std::numeric_limits<double>::infinity();
  if (s0 > 0) return 0.0;
  std::vector<long double> cl(k);
  for (int j = 0; j < k; ++j) cl[j] = (long double)c[j].to_double();
  // Scan y in (0, Y] for the first value clearly above |R| = 1 (values
  // within the rounding bound, e.g. near the origin where |R| - 1 =
  // O(y^(p+2)), or at a tangential contact, count as covered), then bisect.
  // The degree of R is N_max + 1, and no polynomial of degree s with
  // R = 1 + xi + O(xi^2) covers more than [-i s, i s], so Y = 2 (N_max + 2)
  // is a safe end of the scan.
  const long double ymax = 2.0L * (nmax + 2);
  const int n_scan = 100000;
  long double prev = 0;
  for (int i = 1; i <= n_scan; ++i) {
    const long double y = ymax * i / n_scan;
    long double bd;
    if (g_numeric(k, steps, cl, y, &bd) > bd) {
      long double lo = prev, hi = y;
      for (int it = 0; it < 100; ++it) {
        const long double mid = 0.5L * (lo + hi);
        long double bm;
        if (g_numeric(k, steps, cl, mid, &bm) > bm) hi = mid; else lo = mid;
      }
      return (double)lo;
    }
    prev = y;
  }
  return (double)ymax;
}

// max over theta in [0, pi] of s(theta) = 2 sum_k a_k sin(k theta) for the
// order-4 and order-8 centred stencils: dense scan, then golden section.  For
// the Fourier derivative the symbol is theta itself (mode k: 2 pi k = theta n
// with theta = 2 pi k / n), whose bound over the modes is pi.
double stencil_sigma(int fd_order) {
  if (fd_order == GBS_FD_SPECTRAL) return 3.14159265358979323846;
  const double a4[2] = {2.0 / 3.0, -1.0 / 12.0};
  const double a8[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
  const double* a = fd_order == 8 ? a8 : a4;
  const int r = fd_order == 8 ? 4 : 2;
  auto s = [&](double t) {
    double v = 0;
    for (int k = 0; k < r; ++k) v += 2 * a[k] * std::sin((k + 1) * t);
    return v;
  };
  const double pi = 3.14159265358979323846;
  int best = 0;
  double bv = -1;
  const int n = 100000;
  for (int i = 0; i <= n; ++i) {
    double v = s(pi * i / n);
    if (v > bv) { bv = v; best = i; }
  }
  double lo = pi * std::max(best - 1, 0) / n, hi = pi * std::min(best + 1, n) / n;
  const double g = 0.6180339887498949;
  for (int it = 0; it < 200; ++it) {
    double m1 = hi - g * (hi - lo), m2 = lo + g * (hi - lo);
    if (s(m1) < s(m2)) lo = m1; else hi = m2;
  }
  return s(0.5 * (lo + hi));
}

}  // namespace gbs

using namespace gbs;

extern "C" int gbs_weights(int32_t p, int32_t m, const int32_t* steps, int32_t n_free,
                           const int32_t* free_idx, const int64_t* c_free_num,
                           const int64_t* c_free_den, double* c_out, double* isb_out) {
  try {
    if (!steps || !c_out || m <= 0 || n_free < 0 || n_free > m)
      return fail(GBS_EINVAL, "gbs_weights: bad arguments");
    if (n_free > 0 && (!free_idx || !c_free_num || !c_free_den))
      return fail(GBS_EINVAL, "gbs_weights: free weights missing");
    std::vector<Rational> cf(n_free);
    for (int j = 0; j < n_free; ++j) {
      if (c_free_den[j] <= 0) return fail(GBS_EINVAL, "gbs_weights: denominator must be > 0");
      cf[j] = Rational(BigInt(c_free_num[j]), BigInt(c_free_den[j]));
    }
    std::vector<Rational> c;
    int st = exact_weights(p, m, steps, n_free, free_idx, cf.data(), c);
    if (st) return st;
    for (int i = 0; i < m; ++i) c_out[i] = c[i].to_double();
    if (isb_out) *isb_out = isb_of(m, steps, c);
    return GBS_OK;
  } catch (const std::exception& e) {
    return fail(GBS_EINVAL, "gbs_weights: %s", e.what());
  }
}

extern "C" int gbs_isb(int32_t k, const int32_t* steps, const double* weights, double* isb_out) {
  try {
    if (!steps || !weights || !isb_out || k <= 0) return fail(GBS_EINVAL, "gbs_isb: bad arguments");
    int st = check_steps(k, steps);
    if (st) return st;
    std::vector<Rational> c(k);
    for (int j = 0; j < k; ++j) c[j] = Rational::from_double(weights[j]);
    *isb_out = isb_of(k, steps, c);
    return GBS_OK;
  } catch (const std::exception& e) {
    return fail(GBS_EINVAL, "gbs_isb: %s", e.what());
  }
}
