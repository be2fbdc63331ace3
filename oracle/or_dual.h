/*
 * or_dual.h -- scalar with one directional derivative, for the tangent build
 * of the oracle (forward-mode differentiation of the discrete step).
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself.
 *
 * The value part of every operation is the plain double operation on the
 * value parts, in the same order, so a computation on or_dual reproduces the
 * double computation bit for bit and takes the same branches; comparisons
 * look at values only.  The derivative part follows the textbook rules
 * (sum, product, quotient, square root).  At the kinks of |x|, min and max
 * the branch that the value comparison takes supplies the derivative, so the
 * result is the derivative along the branch pattern of the forward run.
 */
#ifndef OR_DUAL_H
#define OR_DUAL_H
#include <math.h>

struct or_dual {
  double v, d;
  or_dual() = default;
  or_dual(double x) : v(x), d(0.0) {}
  or_dual(double x, double dx) : v(x), d(dx) {}
};

static inline double or_value(const or_dual& a) { return a.v; }
static inline double or_value(double a) { return a; }

static inline or_dual operator-(const or_dual& a) { return or_dual(-a.v, -a.d); }
static inline or_dual operator+(const or_dual& a, const or_dual& b) {
  return or_dual(a.v + b.v, a.d + b.d);
}
static inline or_dual operator-(const or_dual& a, const or_dual& b) {
  return or_dual(a.v - b.v, a.d - b.d);
}
static inline or_dual operator*(const or_dual& a, const or_dual& b) {
  return or_dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
static inline or_dual operator/(const or_dual& a, const or_dual& b) {
  double q = a.v / b.v;
  return or_dual(q, (a.d - q * b.d) / b.v);
}
static inline or_dual operator+(const or_dual& a, double b) { return or_dual(a.v + b, a.d); }
static inline or_dual operator+(double a, const or_dual& b) { return or_dual(a + b.v, b.d); }
static inline or_dual operator-(const or_dual& a, double b) { return or_dual(a.v - b, a.d); }
static inline or_dual operator-(double a, const or_dual& b) { return or_dual(a - b.v, -b.d); }
static inline or_dual operator*(const or_dual& a, double b) { return or_dual(a.v * b, a.d * b); }
static inline or_dual operator*(double a, const or_dual& b) { return or_dual(a * b.v, a * b.d); }
static inline or_dual operator/(const or_dual& a, double b) { return or_dual(a.v / b, a.d / b); }
static inline or_dual operator/(double a, const or_dual& b) {
  double q = a / b.v;
  return or_dual(q, -q * b.d / b.v);
}
static inline or_dual& operator+=(or_dual& a, const or_dual& b) { return a = a + b; }
static inline or_dual& operator-=(or_dual& a, const or_dual& b) { return a = a - b; }
static inline or_dual& operator*=(or_dual& a, const or_dual& b) { return a = a * b; }
static inline or_dual& operator/=(or_dual& a, const or_dual& b) { return a = a / b; }

#define OR_DUAL_CMP(op)                                                                   \
  static inline bool operator op(const or_dual& a, const or_dual& b) { return a.v op b.v; } \
  static inline bool operator op(const or_dual& a, double b) { return a.v op b; }           \
  static inline bool operator op(double a, const or_dual& b) { return a op b.v; }
OR_DUAL_CMP(<)
OR_DUAL_CMP(>)
OR_DUAL_CMP(<=)
OR_DUAL_CMP(>=)
OR_DUAL_CMP(==)
OR_DUAL_CMP(!=)
#undef OR_DUAL_CMP

static inline or_dual sqrt(const or_dual& a) {
  double r = sqrt(a.v);
  return or_dual(r, a.d / (2.0 * r));
}
static inline or_dual fabs(const or_dual& a) { return a.v < 0.0 ? -a : a; }
/* x^e for a constant exponent: d(x^e) = e x^(e-1) dx */
static inline or_dual pow(const or_dual& a, double e) {
  double r = pow(a.v, e);
  return or_dual(r, e * pow(a.v, e - 1.0) * a.d);
}
/* C's fmin/fmax on values; the selected operand supplies the derivative
   (the first one when the values are equal) */
static inline or_dual fmin(const or_dual& a, const or_dual& b) { return b.v < a.v ? b : a; }
static inline or_dual fmax(const or_dual& a, const or_dual& b) { return b.v > a.v ? b : a; }
static inline bool isfinite(const or_dual& a) { return isfinite(a.v); }

#endif
