/*
 * flops.h -- an operation-counting scalar for the oracle (test and
 * measurement infrastructure).
 *
 * Flop carries a double and computes every value exactly as double does (the
 * step run on Flop gives the double step bit for bit); each arithmetic
 * operation also bumps a per-thread counter:
 *   add (+, -), mul, div, sqrt, trans (exp, tanh, cosh, pow, log), cmp.
 * The floating-point operation count of a stage is add + mul + div + sqrt +
 * trans (a fused multiply-add would count as two: the oracle has none).
 *
 * Structural zeros: a value built from the constant 0 (the unused entries of
 * a 3x3 tensor in 1-D or 2-D, an accumulator's start) is marked, and the
 * marking follows products (0 * x), sums of two marked values and quotients
 * with a marked numerator.  Operations with a marked operand that an
 * implementation would not execute are not counted: 0 * x, 0 / x, 0 + x,
 * x - 0, 0 - x (a negation).  State and parameter values are never marked,
 * whatever their value.
 */
#pragma once
#include <cmath>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { FC_ADD = 0, FC_MUL, FC_DIV, FC_SQRT, FC_TRANS, FC_CMP, FC_N };

struct alignas(64) FlopSlot {
  long long c[8];
};
extern FlopSlot g_flop_slots[256];

inline void flop_bump(int k) {
#ifdef _OPENMP
  g_flop_slots[omp_get_thread_num() & 255].c[k] += 1;
#else
  g_flop_slots[0].c[k] += 1;
#endif
}

struct Flop {
  double v;
  bool z;  // structural zero
  Flop() : v(0.0), z(true) {}
  Flop(double x) : v(x), z(x == 0.0) {}  // NOLINT: implicit from a constant
  static Flop data(double x) {
    Flop r(x);
    r.z = false;
    return r;
  }
  Flop& operator+=(const Flop& b) { *this = *this + b; return *this; }
  Flop& operator-=(const Flop& b) { *this = *this - b; return *this; }
  Flop& operator*=(const Flop& b) { *this = *this * b; return *this; }
  Flop& operator/=(const Flop& b) { *this = *this / b; return *this; }
  friend Flop operator-(const Flop& a) { Flop r(-a.v); r.z = a.z; return r; }
  friend Flop operator+(const Flop& a, const Flop& b) {
    if (!a.z && !b.z) flop_bump(FC_ADD);
    Flop r(a.v + b.v);
    r.z = a.z && b.z;
    return r;
  }
  friend Flop operator-(const Flop& a, const Flop& b) {
    if (!a.z && !b.z) flop_bump(FC_ADD);
    Flop r(a.v - b.v);
    r.z = a.z && b.z;
    return r;
  }
  friend Flop operator*(const Flop& a, const Flop& b) {
    if (!a.z && !b.z) flop_bump(FC_MUL);
    Flop r(a.v * b.v);
    r.z = a.z || b.z;
    return r;
  }
  friend Flop operator/(const Flop& a, const Flop& b) {
    if (!a.z) flop_bump(FC_DIV);
    Flop r(a.v / b.v);
    r.z = a.z;
    return r;
  }
  friend Flop operator+(const Flop& a, double b) { return a + Flop(b); }
  friend Flop operator+(double a, const Flop& b) { return Flop(a) + b; }
  friend Flop operator-(const Flop& a, double b) { return a - Flop(b); }
  friend Flop operator-(double a, const Flop& b) { return Flop(a) - b; }
  friend Flop operator*(const Flop& a, double b) { return a * Flop(b); }
  friend Flop operator*(double a, const Flop& b) { return Flop(a) * b; }
  friend Flop operator/(const Flop& a, double b) { return a / Flop(b); }
  friend Flop operator/(double a, const Flop& b) { return Flop(a) / b; }
  friend bool operator<(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v < b.v; }
  friend bool operator>(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v > b.v; }
  friend bool operator<=(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v <= b.v; }
  friend bool operator>=(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v >= b.v; }
  friend bool operator==(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v == b.v; }
  friend bool operator!=(const Flop& a, const Flop& b) { flop_bump(FC_CMP); return a.v != b.v; }
  friend bool operator<(const Flop& a, double b) { return a < Flop(b); }
  friend bool operator>(const Flop& a, double b) { return a > Flop(b); }
  friend bool operator<=(const Flop& a, double b) { return a <= Flop(b); }
  friend bool operator>=(const Flop& a, double b) { return a >= Flop(b); }
  friend bool operator<(double a, const Flop& b) { return Flop(a) < b; }
  friend bool operator>(double a, const Flop& b) { return Flop(a) > b; }
  static Flop unary(double v, int kind) {
    flop_bump(kind);
    return Flop::data(v);
  }
  friend Flop sqrt(const Flop& a) { return unary(std::sqrt(a.v), FC_SQRT); }
  friend Flop exp(const Flop& a) { return unary(std::exp(a.v), FC_TRANS); }
  friend Flop tanh(const Flop& a) { return unary(std::tanh(a.v), FC_TRANS); }
  friend Flop cosh(const Flop& a) { return unary(std::cosh(a.v), FC_TRANS); }
  friend Flop log(const Flop& a) { return unary(std::log(a.v), FC_TRANS); }
  friend Flop pow(const Flop& a, double p) { return unary(std::pow(a.v, p), FC_TRANS); }
  friend Flop pow(const Flop& a, const Flop& p) { return unary(std::pow(a.v, p.v), FC_TRANS); }
};
