// Forward-mode scalar for local Jacobians: a value and its gradient with
// respect to N local inputs.  Value parts are computed by the same double
// operations as the time step, so branch decisions (comparisons act on
// values) are the ones the step took; the gradient follows that branch.
#pragma once
#include "mmfv_math.h"

namespace mmfv {

// the overloads for Dn below must not hide the double versions
using ::fabs;
using ::fmax;
using ::fmin;
using ::sqrt;

template <int N>
struct Dn {
  double v;
  double d[N];
  MMD Dn() {}
  MMD Dn(double x) : v(x) {
    for (int i = 0; i < N; i++) d[i] = 0.0;
  }
};

// input i of N with value x
template <int N>
MMD Dn<N> dn_seed(double x, int i) {
  Dn<N> r(x);
  r.d[i] = 1.0;
  return r;
}

template <int N>
MMD Dn<N> operator-(const Dn<N>& a) {
  Dn<N> r;
  r.v = -a.v;
  for (int i = 0; i < N; i++) r.d[i] = -a.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator+(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator-(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator*(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator/(const Dn<N>& a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a.v / b.v;
  double ib = 1.0 / b.v;
  for (int i = 0; i < N; i++) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N>
MMD Dn<N> operator+(const Dn<N>& a, double b) {
  Dn<N> r = a;
  r.v = a.v + b;
  return r;
}
template <int N>
MMD Dn<N> operator+(double a, const Dn<N>& b) {
  Dn<N> r = b;
  r.v = a + b.v;
  return r;
}
template <int N>
MMD Dn<N> operator-(const Dn<N>& a, double b) {
  Dn<N> r = a;
  r.v = a.v - b;
  return r;
}
template <int N>
MMD Dn<N> operator-(double a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a - b.v;
  for (int i = 0; i < N; i++) r.d[i] = -b.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator*(const Dn<N>& a, double b) {
  Dn<N> r;
  r.v = a.v * b;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b;
  return r;
}
template <int N>
MMD Dn<N> operator*(double a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a * b.v;
  for (int i = 0; i < N; i++) r.d[i] = a * b.d[i];
  return r;
}
template <int N>
MMD Dn<N> operator/(const Dn<N>& a, double b) {
  Dn<N> r;
  r.v = a.v / b;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] / b;
  return r;
}
template <int N>
MMD Dn<N> operator/(double a, const Dn<N>& b) {
  Dn<N> r;
  r.v = a / b.v;
  double s = -r.v / b.v;
  for (int i = 0; i < N; i++) r.d[i] = s * b.d[i];
  return r;
}

#define MMFV_DN_CMP(op)                                                              \
  template <int N>                                                                    \
  MMD bool operator op(const Dn<N>& a, const Dn<N>& b) { return a.v op b.v; }        \
  template <int N>                                                                    \
  MMD bool operator op(const Dn<N>& a, double b) { return a.v op b; }                \
  template <int N>                                                                    \
  MMD bool operator op(double a, const Dn<N>& b) { return a op b.v; }
MMFV_DN_CMP(<)
MMFV_DN_CMP(>)
MMFV_DN_CMP(<=)
MMFV_DN_CMP(>=)
MMFV_DN_CMP(==)
MMFV_DN_CMP(!=)
#undef MMFV_DN_CMP

template <int N>
MMD Dn<N> sqrt(const Dn<N>& a) {
  Dn<N> r;
  r.v = ::sqrt(a.v);
  double s = 0.5 / r.v;
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * s;
  return r;
}
template <int N>
MMD Dn<N> fabs(const Dn<N>& a) {
  return a.v < 0.0 ? -a : a;
}
// x^e for a constant exponent: d(x^e) = e x^(e-1) dx
template <int N>
MMD Dn<N> pow(const Dn<N>& a, double e) {
  Dn<N> r;
  r.v = ::pow(a.v, e);
  double s = e * ::pow(a.v, e - 1.0);
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * s;
  return r;
}
// the selected operand supplies the gradient (the first one on a tie)
template <int N>
MMD Dn<N> fmin(const Dn<N>& a, const Dn<N>& b) {
  return b.v < a.v ? b : a;
}
template <int N>
MMD Dn<N> fmax(const Dn<N>& a, const Dn<N>& b) {
  return b.v > a.v ? b : a;
}

}  // namespace mmfv
