// Counts the FP64 arithmetic operations of one bulk 2D update as the
// library writes them: the point-wise templates of mmfv_math.h are
// instantiated with a scalar type that counts every add, subtract, multiply,
// divide and square root applied to state-dependent values (operations on
// EOS parameters alone are loop invariants and not counted; comparisons,
// min/max and absolute values are not arithmetic and not counted).
//
// A bulk update of one cell (Eq. discretized_equ with alpha = A = 1) needs
// the primitive state of its cell, two face fluxes (each of its four faces is
// shared with a neighbour), each face eight WENO5 reconstructions (four
// primitive variables, left and right) and one HLLC flux, and the RK
// combination of four components.
#include <cstdio>
#include <cmath>
#include <cstring>

namespace opc {
struct Ops {
  long add = 0, mul = 0, div = 0, sqrt_ = 0;
  long total() const { return add + mul + div + sqrt_; }
};
static Ops ops;
struct C {
  double v;
  C() : v(0.0) {}
  C(double x) : v(x) {}
};
inline C operator+(C a, C b) { ops.add++; return C(a.v + b.v); }
inline C operator-(C a, C b) { ops.add++; return C(a.v - b.v); }
inline C operator*(C a, C b) { ops.mul++; return C(a.v * b.v); }
inline C operator/(C a, C b) { ops.div++; return C(a.v / b.v); }
inline C operator+(C a, double b) { ops.add++; return C(a.v + b); }
inline C operator+(double a, C b) { ops.add++; return C(a + b.v); }
inline C operator-(C a, double b) { ops.add++; return C(a.v - b); }
inline C operator-(double a, C b) { ops.add++; return C(a - b.v); }
inline C operator*(C a, double b) { ops.mul++; return C(a.v * b); }
inline C operator*(double a, C b) { ops.mul++; return C(a * b.v); }
inline C operator/(C a, double b) { ops.div++; return C(a.v / b); }
inline C operator/(double a, C b) { ops.div++; return C(a / b.v); }
inline C operator-(C a) { return C(-a.v); }
inline bool operator<(C a, C b) { return a.v < b.v; }
inline bool operator>(C a, C b) { return a.v > b.v; }
inline bool operator>=(C a, double b) { return a.v >= b; }
inline bool operator>(C a, double b) { return a.v > b; }
inline bool operator<(C a, double b) { return a.v < b; }
inline C sqrt(C a) { ops.sqrt_++; return C(std::sqrt(a.v)); }
inline C fmin(C a, C b) { return b.v < a.v ? b : a; }
inline C fmax(C a, C b) { return b.v > a.v ? b : a; }
inline C fabs(C a) { return C(std::fabs(a.v)); }
// (the Tait pressure's power; not on the stiffened-gas path counted here)
inline C pow(C a, double e) { ops.mul++; return C(std::pow(a.v, e)); }
}  // namespace opc

#define MMD inline
#include "../../paper_1704_00519_amd/csrc/mmfv_math.h"

using opc::C;
using opc::ops;

static long measure(void (*f)()) {
  ops = opc::Ops();
  f();
  return ops.total();
}

static void f_weno() { mmfv::weno5<C>(C(1.0), C(1.1), C(1.3), C(1.2), C(1.0)); }
static const mmfv::Eos kAir = {1.4, 0.0, 0.0, 0.0, false};
static void f_prim() { mmfv::prim_from_U<C>(C(1.0), C(0.2), C(0.1), C(2.6), kAir); }
// subsonic face: S_L < 0 < S_R, so the star state is built (the usual case)
static void f_hllc_star() {
  mmfv::PrimT<C> L{C(1.0), C(0.1), C(0.05), C(1.0)}, R{C(0.9), C(0.05), C(0.0), C(0.9)};
  C F[4];
  mmfv::hllc_flux<C>(L, R, kAir, 2.5, F);
}
static void f_hllc_super() {
  mmfv::PrimT<C> L{C(1.0), C(5.0), C(0.0), C(1.0)}, R{C(1.0), C(5.0), C(0.0), C(1.0)};
  C F[4];
  mmfv::hllc_flux<C>(L, R, kAir, 2.5, F);
}
// RK combination of one component, as the bulk kernel writes it: the
// divergence of the x- and y-face fluxes, then b Q^n + c (Q^(s) + rhs)
// (stage 0 of the RK scheme has b = 0, c = 1 and adds Q^(s) + rhs only)
static bool stage0;
static void f_update() {
  C Fl(1.0), Fr(1.1), Fb(0.9), Ft(1.2), qs(1.0), qn(1.0);
  double lx = 0.1, ly = 0.1, b = 0.75, c = 0.25;
  C rhs = lx * (Fl - Fr);
  rhs = rhs + ly * (Fb - Ft);
  C x = stage0 ? (qs + rhs) : (b * qn + c * (qs + rhs));
  (void)x;
}

int main() {
  long weno = measure(f_weno), prim = measure(f_prim);
  long hllc = measure(f_hllc_star), hllc_sup = measure(f_hllc_super);
  stage0 = true;
  long upd0 = measure(f_update);
  stage0 = false;
  long upd = measure(f_update);
  long face = 8 * weno + hllc;
  // mean over the three stages of SSP-RK3 (one stage-0 combination, two full)
  long per_update3 = 3 * (2 * face + prim) + 4 * (upd0 + 2 * upd);
  std::printf("weno5 %ld\nhllc_star %ld\nhllc_supersonic %ld\nprim %ld\n", weno, hllc, hllc_sup, prim);
  std::printf("update_component_stage0 %ld\nupdate_component %ld\nface %ld\n", upd0, upd, face);
  std::printf("bulk_update_2d_rk3_mean %.4f\n", per_update3 / 3.0);
  return 0;
}
