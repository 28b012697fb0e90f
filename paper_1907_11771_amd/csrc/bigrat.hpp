// Exact rational arithmetic for the host side of the library: arbitrary
// precision integers (32-bit limbs) and reduced fractions, with correctly
// rounded conversion to double.  Used once per plan to solve the order
// constraints exactly (weights are rounded to FP64 only at the end) and to
// form the exact |R(iy)|^2 - 1 polynomial for the stability check.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace gbs {

class BigInt {
 public:
  BigInt() = default;
  BigInt(int64_t v) {  // NOLINT(implicit)
    neg_ = v < 0;
    uint64_t m = neg_ ? (uint64_t)(-(v + 1)) + 1u : (uint64_t)v;
    while (m) { mag_.push_back((uint32_t)m); m >>= 32; }
  }
  static BigInt from_u64(uint64_t m) {
    BigInt r;
    while (m) { r.mag_.push_back((uint32_t)m); m >>= 32; }
    return r;
  }

  bool is_zero() const { return mag_.empty(); }
  bool negative() const { return neg_ && !is_zero(); }
  int sign() const { return is_zero() ? 0 : (neg_ ? -1 : 1); }
  BigInt abs() const { BigInt r = *this; r.neg_ = false; return r; }
  BigInt operator-() const { BigInt r = *this; if (!r.is_zero()) r.neg_ = !r.neg_; return r; }

  size_t bit_length() const {
    if (mag_.empty()) return 0;
    uint32_t top = mag_.back();
    size_t b = 0;
    while (top) { ++b; top >>= 1; }
    return (mag_.size() - 1) * 32 + b;
  }
  bool bit(size_t i) const {
    size_t w = i / 32;
    return w < mag_.size() && ((mag_[w] >> (i % 32)) & 1u);
  }
  bool is_even() const { return mag_.empty() || !(mag_[0] & 1u); }

  friend int cmp_mag(const BigInt& a, const BigInt& b) {
    if (a.mag_.size() != b.mag_.size()) return a.mag_.size() < b.mag_.size() ? -1 : 1;
    for (size_t i = a.mag_.size(); i-- > 0;)
      if (a.mag_[i] != b.mag_[i]) return a.mag_[i] < b.mag_[i] ? -1 : 1;
    return 0;
  }
  friend int cmp(const BigInt& a, const BigInt& b) {
    int sa = a.sign(), sb = b.sign();
    if (sa != sb) return sa < sb ? -1 : 1;
    int m = cmp_mag(a, b);
    return sa >= 0 ? m : -m;
  }

  friend BigInt operator+(const BigInt& a, const BigInt& b) {
    if (a.negative() == b.negative()) {
      BigInt r = add_mag(a, b);
      r.neg_ = a.negative();
      return r;
    }
    if (cmp_mag(a, b) >= 0) { BigInt r = sub_mag(a, b); r.neg_ = a.negative(); r.trim(); return r; }
    BigInt r = sub_mag(b, a);
    r.neg_ = b.negative();
    r.trim();
    return r;
  }
  friend BigInt operator-(const BigInt& a, const BigInt& b) { return a + (-b); }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.is_zero() || b.is_zero()) return r;
    r.mag_.assign(a.mag_.size() + b.mag_.size(), 0u);
    for (size_t i = 0; i < a.mag_.size(); ++i) {
      uint64_t carry = 0;
      for (size_t j = 0; j < b.mag_.size(); ++j) {
        uint64_t cur = (uint64_t)a.mag_[i] * b.mag_[j] + r.mag_[i + j] + carry;
        r.mag_[i + j] = (uint32_t)cur;
        carry = cur >> 32;
      }
      size_t k = i + b.mag_.size();
      while (carry) {
        uint64_t cur = (uint64_t)r.mag_[k] + carry;
        r.mag_[k] = (uint32_t)cur;
        carry = cur >> 32;
        ++k;
      }
    }
    r.neg_ = a.negative() != b.negative();
    r.trim();
    return r;
  }

  BigInt shl(size_t n) const {
    if (is_zero()) return *this;
    BigInt r;
    size_t w = n / 32, s = n % 32;
    r.mag_.assign(mag_.size() + w + 1, 0u);
    for (size_t i = 0; i < mag_.size(); ++i) {
      uint64_t v = (uint64_t)mag_[i] << s;
      r.mag_[i + w] |= (uint32_t)v;
      r.mag_[i + w + 1] |= (uint32_t)(v >> 32);
    }
    r.neg_ = neg_;
    r.trim();
    return r;
  }
  BigInt shr(size_t n) const {
    size_t w = n / 32, s = n % 32;
    BigInt r;
    if (w >= mag_.size()) return r;
    r.mag_.assign(mag_.size() - w, 0u);
    for (size_t i = w; i < mag_.size(); ++i) {
      uint64_t v = mag_[i];
      if (i + 1 < mag_.size()) v |= (uint64_t)mag_[i + 1] << 32;
      r.mag_[i - w] = (uint32_t)(v >> s);
    }
    r.neg_ = neg_;
    r.trim();
    return r;
  }

  // Truncating division; quotient sign = product of signs, remainder takes
  // the sign of the dividend.  Bitwise long division with the running
  // remainder shifted in place.
  static void divmod(const BigInt& a, const BigInt& b, BigInt& q, BigInt& r) {
    if (b.is_zero()) throw std::domain_error("BigInt division by zero");
    q = BigInt();
    r = BigInt();
    if (cmp_mag(a, b) < 0) { r = a; return; }
    const std::vector<uint32_t>& bm = b.mag_;
    const size_t nl = bm.size() + 1;
    std::vector<uint32_t> rem(nl, 0u);
    size_t nb = a.bit_length();
    q.mag_.assign((nb + 31) / 32, 0u);
    for (size_t i = nb; i-- > 0;) {
      uint32_t carry = a.bit(i) ? 1u : 0u;
      for (size_t k = 0; k < nl; ++k) {
        uint32_t nc = rem[k] >> 31;
        rem[k] = (rem[k] << 1) | carry;
        carry = nc;
      }
      // rem >= b ?
      int c = 0;
      if (rem[nl - 1]) c = 1;
      else {
        for (size_t k = bm.size(); k-- > 0;) {
          if (rem[k] != bm[k]) { c = rem[k] > bm[k] ? 1 : -1; break; }
        }
      }
      if (c >= 0) {
        int64_t borrow = 0;
        for (size_t k = 0; k < nl; ++k) {
          int64_t d = (int64_t)rem[k] - borrow - (k < bm.size() ? (int64_t)bm[k] : 0);
          borrow = d < 0;
          if (d < 0) d += ((int64_t)1 << 32);
          rem[k] = (uint32_t)d;
        }
        q.mag_[i / 32] |= 1u << (i % 32);
      }
    }
    q.trim();
    q.neg_ = a.negative() != b.negative();
    r.mag_ = rem;
    r.neg_ = a.negative();
    r.trim();
  }
  friend BigInt operator/(const BigInt& a, const BigInt& b) { BigInt q, r; divmod(a, b, q, r); return q; }

  // Binary (Stein) gcd of the magnitudes.
  static BigInt gcd(BigInt a, BigInt b) {
    a = a.abs();
    b = b.abs();
    if (a.is_zero()) return b;
    if (b.is_zero()) return a;
    size_t shift = 0;
    while (a.is_even() && b.is_even()) { a = a.shr(1); b = b.shr(1); ++shift; }
    while (a.is_even()) a = a.shr(1);
    while (!b.is_zero()) {
      while (b.is_even()) b = b.shr(1);
      if (cmp_mag(a, b) > 0) std::swap(a, b);
      b = sub_mag(b, a);
    }
    return a.shl(shift);
  }

  // Low 64 bits of the magnitude.
  uint64_t low64() const {
    uint64_t v = 0;
    if (mag_.size() > 0) v |= mag_[0];
    if (mag_.size() > 1) v |= (uint64_t)mag_[1] << 32;
    return v;
  }

 private:
  static BigInt add_mag(const BigInt& a, const BigInt& b) {
    BigInt r;
    size_t n = std::max(a.mag_.size(), b.mag_.size());
    r.mag_.assign(n + 1, 0u);
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
      uint64_t s = carry;
      if (i < a.mag_.size()) s += a.mag_[i];
      if (i < b.mag_.size()) s += b.mag_[i];
      r.mag_[i] = (uint32_t)s;
      carry = s >> 32;
    }
    r.mag_[n] = (uint32_t)carry;
    r.trim();
    return r;
  }
  // requires |a| >= |b|
  static BigInt sub_mag(const BigInt& a, const BigInt& b) {
    BigInt r;
    r.mag_.assign(a.mag_.size(), 0u);
    int64_t borrow = 0;
    for (size_t i = 0; i < a.mag_.size(); ++i) {
      int64_t d = (int64_t)a.mag_[i] - borrow - (i < b.mag_.size() ? (int64_t)b.mag_[i] : 0);
      borrow = d < 0;
      if (d < 0) d += ((int64_t)1 << 32);
      r.mag_[i] = (uint32_t)d;
    }
    r.trim();
    return r;
  }
  void trim() {
    while (!mag_.empty() && mag_.back() == 0u) mag_.pop_back();
    if (mag_.empty()) neg_ = false;
  }

  bool neg_ = false;
  std::vector<uint32_t> mag_;
};

class Rational {
 public:
  Rational() : num_(0), den_(1) {}
  Rational(int64_t v) : num_(v), den_(1) {}  // NOLINT(implicit)
  Rational(BigInt n, BigInt d) : num_(std::move(n)), den_(std::move(d)) { normalise(); }

  // The exact value of a finite double.
  static Rational from_double(double x) {
    if (!std::isfinite(x)) throw std::domain_error("non-finite weight");
    if (x == 0.0) return Rational();
    int e;
    double m = std::frexp(x, &e);             // x = m * 2^e, 0.5 <= |m| < 1
    int64_t mi = (int64_t)std::ldexp(m, 53);  // exact
    e -= 53;
    BigInt n(mi), d(1);
    if (e >= 0) n = n.shl((size_t)e); else d = d.shl((size_t)(-e));
    return Rational(n, d);
  }

  const BigInt& num() const { return num_; }
  const BigInt& den() const { return den_; }
  bool is_zero() const { return num_.is_zero(); }
  int sign() const { return num_.sign(); }

  friend Rational operator+(const Rational& a, const Rational& b) {
    return Rational(a.num_ * b.den_ + b.num_ * a.den_, a.den_ * b.den_);
  }
  friend Rational operator-(const Rational& a, const Rational& b) {
    return Rational(a.num_ * b.den_ - b.num_ * a.den_, a.den_ * b.den_);
  }
  friend Rational operator*(const Rational& a, const Rational& b) {
    return Rational(a.num_ * b.num_, a.den_ * b.den_);
  }
  friend Rational operator/(const Rational& a, const Rational& b) {
    if (b.is_zero()) throw std::domain_error("rational division by zero");
    return Rational(a.num_ * b.den_, a.den_ * b.num_);
  }
  Rational operator-() const { return Rational(-num_, den_); }
  friend bool operator==(const Rational& a, const Rational& b) {
    return cmp(a.num_, b.num_) == 0 && cmp(a.den_, b.den_) == 0;
  }

  // Nearest double, ties to even (normal range; results below the normal
  // range are formed with one extra rounding by ldexp).
  double to_double() const {
    if (num_.is_zero()) return 0.0;
    BigInt a = num_.abs();
    const BigInt& b = den_;
    long s = 54 - ((long)a.bit_length() - (long)b.bit_length());
    BigInt q, r;
    for (int it = 0; it < 4; ++it) {
      BigInt aa = s >= 0 ? a.shl((size_t)s) : a;
      BigInt bb = s >= 0 ? b : b.shl((size_t)(-s));
      BigInt::divmod(aa, bb, q, r);
      size_t bl = q.bit_length();
      if (bl == 54) break;
      s += bl < 54 ? 1 : -1;
    }
    uint64_t qq = q.low64();            // 54 bits: 53 + guard
    uint64_t mant = qq >> 1;
    bool guard = qq & 1u, sticky = !r.is_zero();
    if (guard && (sticky || (mant & 1u))) ++mant;
    double v = std::ldexp((double)mant, (int)(1 - s));
    return num_.negative() ? -v : v;
  }

  std::string str() const;

 private:
  void normalise() {
    if (den_.is_zero()) throw std::domain_error("zero denominator");
    if (den_.negative()) { num_ = -num_; den_ = -den_; }
    if (num_.is_zero()) { den_ = BigInt(1); return; }
    BigInt g = BigInt::gcd(num_, den_);
    if (!(cmp(g, BigInt(1)) == 0)) { num_ = num_ / g; den_ = den_ / g; }
  }
  BigInt num_, den_;
};

}  // namespace gbs
