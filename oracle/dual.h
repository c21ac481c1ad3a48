/*
 * dual.h -- forward-mode dual numbers for the oracle (test infrastructure).
 *
 * Dual<K> carries a value and K directional derivatives; every operation
 * applies the chain rule exactly, so running the oracle's step on Dual<K>
 * gives the exact tangent (Jacobian-vector product) of the discrete step in K
 * directions at once.  Comparisons look at the value only: a non-smooth
 * operation (min, max, abs, a branch) is differentiated along the branch the
 * value takes.
 */
#pragma once
#include <cmath>

template <int K> struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { for (int k = 0; k < K; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0.0; }  // NOLINT: implicit from a constant
  Dual& operator+=(const Dual& b) { v += b.v; for (int k = 0; k < K; ++k) d[k] += b.d[k]; return *this; }
  Dual& operator-=(const Dual& b) { v -= b.v; for (int k = 0; k < K; ++k) d[k] -= b.d[k]; return *this; }
  Dual& operator*=(const Dual& b) { *this = *this * b; return *this; }
  Dual& operator/=(const Dual& b) { *this = *this / b; return *this; }
  friend Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
  friend Dual operator+(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
  }
  friend Dual operator-(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
  }
  friend Dual operator*(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v * b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
  }
  friend Dual operator/(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
  }
  friend Dual operator+(const Dual& a, double b) { return a + Dual(b); }
  friend Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
  friend Dual operator-(const Dual& a, double b) { return a - Dual(b); }
  friend Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
  friend Dual operator*(const Dual& a, double b) {
    Dual r; r.v = a.v * b; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b; return r;
  }
  friend Dual operator*(double a, const Dual& b) { return b * a; }
  friend Dual operator/(const Dual& a, double b) { return a / Dual(b); }
  friend Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
  friend bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
  friend bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
  friend bool operator<=(const Dual& a, const Dual& b) { return a.v <= b.v; }
  friend bool operator>=(const Dual& a, const Dual& b) { return a.v >= b.v; }
  friend bool operator==(const Dual& a, const Dual& b) { return a.v == b.v; }
  friend bool operator!=(const Dual& a, const Dual& b) { return a.v != b.v; }
  friend bool operator<(const Dual& a, double b) { return a.v < b; }
  friend bool operator>(const Dual& a, double b) { return a.v > b; }
  friend bool operator<=(const Dual& a, double b) { return a.v <= b; }
  friend bool operator>=(const Dual& a, double b) { return a.v >= b; }
  friend bool operator<(double a, const Dual& b) { return a < b.v; }
  friend bool operator>(double a, const Dual& b) { return a > b.v; }
  /* elementary functions: value and derivative from the mathematics */
  friend Dual chain(const Dual& a, double f, double df) {
    Dual r; r.v = f; for (int k = 0; k < K; ++k) r.d[k] = df * a.d[k]; return r;
  }
  friend Dual sqrt(const Dual& a) { const double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
  friend Dual exp(const Dual& a) { const double e = std::exp(a.v); return chain(a, e, e); }
  friend Dual tanh(const Dual& a) { const double t = std::tanh(a.v); return chain(a, t, 1.0 - t * t); }
  friend Dual cosh(const Dual& a) { return chain(a, std::cosh(a.v), std::sinh(a.v)); }
  friend Dual pow(const Dual& a, double p) {
    return chain(a, std::pow(a.v, p), p * std::pow(a.v, p - 1.0));
  }
  friend Dual pow(const Dual& a, const Dual& p) {  // a^p = exp(p log a)
    const double f = std::pow(a.v, p.v);
    Dual r; r.v = f;
    for (int k = 0; k < K; ++k) r.d[k] = f * (p.v * a.d[k] / a.v + std::log(a.v) * p.d[k]);
    return r;
  }
};
