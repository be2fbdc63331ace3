// Point-wise numerics of the cut-cell step, device side.
//
// Every expression is written in a fixed evaluation order and the library is
// compiled without floating-point contraction, so each operation is rounded
// exactly once as written.  This makes results reproducible bit for bit
// across launch shapes.  FP64 addition, multiplication and square root round
// like the host's IEEE operations; FP64 division is faithful and almost
// always correctly rounded, but not when the exact quotient lies within about
// 1e-16 ulp of a rounding midpoint (such quotients arise between numbers near
// 1), so a host computation of the same expressions can differ in the last
// bit there.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef MMD
#define MMD __device__ __forceinline__
#endif

namespace mmfv {

constexpr int H = 4;       // halo width (WENO5 needs 3, extension 4)
constexpr int MAXM = 8;

struct Params {
  int dim, nx, ny, NX, NY, HY, NC, M;
  double dx, dy, h, bls, idx, idy, amix;
  int kext;
  // pinf: the p_inf of the energy relation (a Tait material's B - p0)
  double gamma[MAXM], pinf[MAXM], igm1[MAXM];
  int bc[4];
  double inflow_W[4];
  int inflow_mat;
  double cfl;
  int tait[MAXM];                 // 1: Tait material (pressure from density)
  double taitB[MAXM], rho0[MAXM];
  int flux;                       // FLUX_HLLC or FLUX_ROE
  int scale_sep;                  // 1: interface scale separation after each step
  int coord;                      // 1: 1D cylindrical, x the radius
  int fs_on, fs_mat;              // material fs_mat: an ambient that is not solved
  double x0;                      // low end of the domain in x
  double fs_p[5];                 // p_hi, p_lo, t0, t1, density of the ambient
  int reinit;                     // 1: redistancing of the level set after each step
  int nband;                      // band width of the level set in cells
};
enum { FLUX_HLLC = 0, FLUX_ROE = 1 };

// EOS of one material, as the point-wise functions take it
struct Eos {
  double g, pinf, B, rho0;
  bool tait;
};
MMD Eos eos_of(const Params& P, int m) {
  Eos e;
  e.g = P.gamma[m];
  e.pinf = P.pinf[m];
  e.B = P.taitB[m];
  e.rho0 = P.rho0[m];
  e.tait = P.tait[m] != 0;
  return e;
}

// ---------------------------------------------------------------------------
// The point-wise functions below are templates on the scalar type T.  The
// time step instantiates them with double; the adjoint instantiates them with
// a value + gradient type (forward-mode over a few local inputs) to obtain
// local Jacobians.  Comparisons act on values, so both take the same branches.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// EOS (Sec. 2.1).  Stiffened gas: p = (gamma-1) rho e - gamma p_inf.  Tait
// (water-like fluids): p = B (rho/rho0)^gamma - B + p0, a function of the
// density alone; its energy relation is that of the stiffened gas with the
// same gamma and p_inf = B - p0 (so rho E is defined and
// c^2 = gamma (p + B - p0)/rho).
// ---------------------------------------------------------------------------
template <class T>
struct PrimT {
  T r, u, v, p;
};
using Prim = PrimT<double>;

template <class T>
MMD PrimT<T> prim_from_U(T U0, T U1, T U2, T U3, const Eos& e) {
  PrimT<T> w;
  w.r = U0;
  w.u = U1 / U0;
  w.v = U2 / U0;
  T ke = 0.5 * w.r * (w.u * w.u + w.v * w.v);
  if (e.tait)
    w.p = e.B * pow(U0 / e.rho0, e.g) - e.pinf;
  else
    w.p = (e.g - 1.0) * (U3 - ke) - e.g * e.pinf;
  return w;
}

template <class T>
MMD T total_energy(T r, T u, T v, T p, double g, double pinf, double igm1) {
  return (p + g * pinf) * igm1 + 0.5 * r * (u * u + v * v);
}

// ---------------------------------------------------------------------------
// HLLC with the two-EOS Roe-averaged wave-speed estimates (Sec. 2.3.2).
// States are (rho, u_normal, u_tangential, p).
// ---------------------------------------------------------------------------
template <class T>
MMD void wave_speeds(const PrimT<T>& L, const Eos& eL, const PrimT<T>& R, const Eos& eR,
                     T& SL, T& SR) {
  double gL = eL.g, piL = eL.pinf, gR = eR.g, piR = eR.pinf;
  T irL = 1.0 / L.r, irR = 1.0 / R.r;
  T porL = L.p * irL, porR = R.p * irR;
  // Tait: Psi = dp/drho = gamma (p + B - p0)/rho, Upsilon = 0
  T psiL = eL.tait ? gL * (L.p + piL) * irL : (L.p + gL * piL) * irL;
  T psiR = eR.tait ? gR * (R.p + piR) * irR : (R.p + gR * piR) * irR;
  double upsL = eL.tait ? 0.0 : gL - 1.0, upsR = eR.tait ? 0.0 : gR - 1.0;
  T cL = sqrt(psiL + upsL * porL);
  T cR = sqrt(psiR + upsR * porR);
  T sL = sqrt(L.r), sR = sqrt(R.r);
  T iw = 1.0 / (sL + sR);
  T psi_t = (sL * psiL + sR * psiR) * iw;
  T ups_t = (sL * upsL + sR * upsR) * iw;
  T u_t = (sL * L.u + sR * R.u) * iw;
  T du = (R.u - L.u) * iw;
  T por_t = (sL * porL + sR * porR) * iw + 0.5 * (sL * sR) * (du * du);
  T c_t = sqrt(psi_t + ups_t * por_t);
  SL = fmin(L.u - cL, u_t - c_t);
  SR = fmax(u_t + c_t, R.u + cR);
}

template <class T>
MMD T contact_speed(const PrimT<T>& L, const PrimT<T>& R, T SL, T SR) {
  T num = ((SR - R.u) * R.r * R.u + (L.u - SL) * L.r * L.u) + (L.p - R.p);
  T den = (SR - R.u) * R.r + (L.u - SL) * L.r;
  return num / den;
}

// HLLC face flux inside one material: F = (mass, normal mom, tangential mom,
// energy).
template <class T>
MMD void hllc_flux(const PrimT<T>& L, const PrimT<T>& R, const Eos& e, double igm1, T F[4]) {
  double g = e.g, pinf = e.pinf;
  T SL, SR;
  wave_speeds(L, e, R, e, SL, SR);
  T SM = contact_speed(L, R, SL, SR);
  // upwind choice: F_L if S_L >= 0, else F*_L if S_M >= 0, else F*_R if
  // S_R > 0, else F_R
  bool left = (SL >= 0.0) || (SM >= 0.0);
  const PrimT<T>& K = left ? L : R;
  T Sk = left ? SL : SR;
  bool star = !(SL >= 0.0) && ((SM >= 0.0) || (SR > 0.0));
  T r = K.r, u = K.u, v = K.v, p = K.p;
  T E = total_energy(r, u, v, p, g, pinf, igm1);
  T ru = r * u;
  F[0] = ru;
  F[1] = ru * u + p;
  F[2] = ru * v;
  F[3] = u * (E + p);
  if (star) {
    T d = Sk - u;
    T mk = r * d;
    T coef = mk / (Sk - SM);
    T Us0 = coef;
    T Us1 = coef * SM;
    T Us2 = coef * v;
    T Us3 = coef * (E / r + (SM - u) * (SM + p / mk));
    F[0] = F[0] + Sk * (Us0 - r);
    F[1] = F[1] + Sk * (Us1 - ru);
    F[2] = F[2] + Sk * (Us2 - r * v);
    F[3] = F[3] + Sk * (Us3 - E);
  }
}

// ---------------------------------------------------------------------------
// Roe flux with characteristic-wise WENO5 (the second face-flux variant,
// stiffened gases only).  Same expressions, in the same order, as the CPU
// reference, so both round alike.
// ---------------------------------------------------------------------------
// conserved (rho, rho u_n, rho u_t, rho E) of a primitive state
template <class T>
MMD void roe_cons(const PrimT<T>& w, const Eos& e, double igm1, T U[4]) {
  U[0] = w.r;
  U[1] = w.r * w.u;
  U[2] = w.r * w.v;
  U[3] = total_energy(w.r, w.u, w.v, w.p, e.g, e.pinf, igm1);
}
// Roe average of two states: normal and tangential velocity, enthalpy and
// sound speed, c^2 = (gamma-1)(H - |u|^2/2)
template <class T>
MMD void roe_average(const PrimT<T>& L, const PrimT<T>& R, const Eos& e, double igm1, T& u,
                     T& v, T& Hr, T& c) {
  T sL = sqrt(L.r), sR = sqrt(R.r);
  T iw = 1.0 / (sL + sR);
  T HL = (total_energy(L.r, L.u, L.v, L.p, e.g, e.pinf, igm1) + L.p) / L.r;
  T HR = (total_energy(R.r, R.u, R.v, R.p, e.g, e.pinf, igm1) + R.p) / R.r;
  u = (sL * L.u + sR * R.u) * iw;
  v = (sL * L.v + sR * R.v) * iw;
  Hr = (sL * HL + sR * HR) * iw;
  c = sqrt((e.g - 1.0) * (Hr - 0.5 * (u * u + v * v)));
}
// left (Lm[k][.]) and right (Rm[.][k]) eigenvectors of the normal flux
// Jacobian: eigenvalues u - c, u, u (shear), u + c
template <class T>
MMD void roe_eig(double g, T u, T v, T Hr, T c, T Lm[4][4], T Rm[4][4]) {
  T q2 = 0.5 * (u * u + v * v);
  T b1 = (g - 1.0) / (c * c), b2 = q2 * b1;
  Rm[0][0] = 1.0; Rm[1][0] = u - c; Rm[2][0] = v; Rm[3][0] = Hr - u * c;
  Rm[0][1] = 1.0; Rm[1][1] = u;     Rm[2][1] = v; Rm[3][1] = q2;
  Rm[0][2] = 0.0; Rm[1][2] = 0.0;   Rm[2][2] = 1.0; Rm[3][2] = v;
  Rm[0][3] = 1.0; Rm[1][3] = u + c; Rm[2][3] = v; Rm[3][3] = Hr + u * c;
  Lm[0][0] = 0.5 * (b2 + u / c); Lm[0][1] = -0.5 * (b1 * u + 1.0 / c);
  Lm[0][2] = -0.5 * (b1 * v); Lm[0][3] = 0.5 * b1;
  Lm[1][0] = 1.0 - b2; Lm[1][1] = b1 * u; Lm[1][2] = b1 * v; Lm[1][3] = -b1;
  Lm[2][0] = -v; Lm[2][1] = 0.0; Lm[2][2] = 1.0; Lm[2][3] = 0.0;
  Lm[3][0] = 0.5 * (b2 - u / c); Lm[3][1] = -0.5 * (b1 * u - 1.0 / c);
  Lm[3][2] = -0.5 * (b1 * v); Lm[3][3] = 0.5 * b1;
}
template <class T>
MMD void roe_mv(const T A[4][4], const T x[4], T y[4]) {
  for (int k = 0; k < 4; k++) y[k] = ((A[k][0] * x[0] + A[k][1] * x[1]) + A[k][2] * x[2]) + A[k][3] * x[3];
}
// normal flux and pressure of a conserved state
template <class T>
MMD void roe_phys(const T U[4], const Eos& e, T F[4], T& p) {
  T rho = U[0], un = U[1] / rho, ut = U[2] / rho;
  p = (e.g - 1.0) * (U[3] - 0.5 * rho * (un * un + ut * ut)) - e.g * e.pinf;
  F[0] = U[1];
  F[1] = U[1] * un + p;
  F[2] = U[1] * ut;
  F[3] = un * (U[3] + p);
}
// u_n -+ c of a conserved state; ok = false if it is not physical
template <class T>
MMD T roe_acoustic(const T U[4], const Eos& e, int sign, bool& ok) {
  T rho = U[0];
  T un = U[1] / rho, ut = U[2] / rho;
  T p = (e.g - 1.0) * (U[3] - 0.5 * rho * (un * un + ut * ut)) - e.g * e.pinf;
  ok = rho > 0.0 && p + e.pinf > 0.0;
  if (!ok) return T(0.0);
  T c = sqrt(e.g * (p + e.pinf) / rho);
  return sign < 0 ? un - c : un + c;
}
// Roe flux with the Harten-Hyman entropy fix on the acoustic fields (the
// speeds on either side of each acoustic wave of the linearised solution)
template <class T>
MMD void roe_flux(const PrimT<T>& WL, const PrimT<T>& WR, const Eos& e, double igm1, T G[4]) {
  T UL[4], UR[4], FL[4], FR[4], pL, pR;
  roe_cons(WL, e, igm1, UL);
  roe_cons(WR, e, igm1, UR);
  roe_phys(UL, e, FL, pL);
  roe_phys(UR, e, FR, pR);
  T u, v, Hr, c, Lm[4][4], Rm[4][4];
  roe_average(WL, WR, e, igm1, u, v, Hr, c);
  roe_eig(e.g, u, v, Hr, c, Lm, Rm);
  T dU[4], a[4];
  for (int k = 0; k < 4; k++) dU[k] = UR[k] - UL[k];
  roe_mv(Lm, dU, a);
  T lam[4] = {u - c, u, u, u + c};
  T Ua[4], Ub[4];
  for (int q = 0; q < 4; q++) {
    Ua[q] = UL[q] + a[0] * Rm[q][0];
    Ub[q] = UR[q] - a[3] * Rm[q][3];
  }
  for (int k = 0; k < 4; k++) {
    T l = fabs(lam[k]);
    if (k == 0 || k == 3) {
      bool oka, okb;
      T la = k == 0 ? roe_acoustic(UL, e, -1, oka) : roe_acoustic(Ub, e, 1, oka);
      T lb = k == 0 ? roe_acoustic(Ua, e, -1, okb) : roe_acoustic(UR, e, 1, okb);
      if (oka && okb) {
        T d1 = lam[k] - la, d2 = lb - lam[k];
        T delta = d1 > d2 ? d1 : d2;
        if (delta > 0.0 && l < delta) l = (lam[k] * lam[k] + delta * delta) / (2.0 * delta);
      }
    }
    a[k] = l * a[k];
  }
  for (int q = 0; q < 4; q++) {
    T d = ((Rm[q][0] * a[0] + Rm[q][1] * a[1]) + Rm[q][2] * a[2]) + Rm[q][3] * a[3];
    G[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * d;
  }
}

template <class T>
MMD T weno5(T v1, T v2, T v3, T v4, T v5);

// characteristic-wise WENO5 at a face from the six stencil states (face
// normal first): returns the primitive states on both sides
template <class T>
MMD void char_weno(const PrimT<T> Ws[6], const Eos& e, double igm1, PrimT<T>& WL,
                   PrimT<T>& WR) {
  T U[6][4], w[6][4];
  for (int q = 0; q < 6; q++) roe_cons(Ws[q], e, igm1, U[q]);
  T u, v, Hr, c, Lm[4][4], Rm[4][4];
  roe_average(Ws[2], Ws[3], e, igm1, u, v, Hr, c);
  roe_eig(e.g, u, v, Hr, c, Lm, Rm);
  for (int q = 0; q < 6; q++) roe_mv(Lm, U[q], w[q]);
  T cl[4], cr[4], UL[4], UR[4];
  for (int k = 0; k < 4; k++) {
    cl[k] = weno5(w[0][k], w[1][k], w[2][k], w[3][k], w[4][k]);
    cr[k] = weno5(w[5][k], w[4][k], w[3][k], w[2][k], w[1][k]);
  }
  roe_mv(Rm, cl, UL);
  roe_mv(Rm, cr, UR);
  T pL, pR, F[4];
  roe_phys(UL, e, F, pL);
  roe_phys(UR, e, F, pR);
  WL.r = UL[0]; WL.u = UL[1] / UL[0]; WL.v = UL[2] / UL[0]; WL.p = pL;
  WR.r = UR[0]; WR.u = UR[1] / UR[0]; WR.v = UR[2] / UR[0]; WR.p = pR;
}

// face flux of the Roe variant from the six stencil states (face-normal
// order, cells i-2 .. i+3 of face i+1/2); all_ok: every stencil cell holds a
// state.  A reconstructed state that is not physical (or a stencil cell
// without a state) falls back to the first-order states of the two face
// cells; the return value is false then.
template <class T>
MMD bool roe_face(const PrimT<T> Ws[6], bool all_ok, const Eos& e, double igm1, T G[4]) {
  PrimT<T> L, R;
  bool ok = all_ok;
  if (ok) {
    char_weno(Ws, e, igm1, L, R);
    if (!(L.r > 0.0) || !(R.r > 0.0) || !(L.p + e.pinf > 0.0) || !(R.p + e.pinf > 0.0))
      ok = false;
  }
  if (!ok) {
    L = Ws[2];
    R = Ws[3];
  }
  roe_flux(L, R, e, igm1, G);
  return ok;
}

// ---------------------------------------------------------------------------
// WENO5-JS (Jiang-Shu), one division per reconstructed value: the nonlinear
// weights d_k/(eps+beta_k)^2 are scaled by the product of the three squared
// denominators and the 1/6 of the candidate stencils joins the same division.
// ---------------------------------------------------------------------------
template <class T>
MMD T weno5(T v1, T v2, T v3, T v4, T v5) {
  T t, u;
  t = v1 - 2.0 * v2 + v3;
  u = v1 - 4.0 * v2 + 3.0 * v3;
  T b0 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v2 - 2.0 * v3 + v4;
  u = v2 - v4;
  T b1 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v3 - 2.0 * v4 + v5;
  u = 3.0 * v3 - 4.0 * v4 + v5;
  T b2 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  T e0 = 1e-6 + b0, e1 = 1e-6 + b1, e2 = 1e-6 + b2;
  e0 = e0 * e0;
  e1 = e1 * e1;
  e2 = e2 * e2;
  T a0 = 0.1 * (e1 * e2);
  T a1 = 0.6 * (e0 * e2);
  T a2 = 0.3 * (e0 * e1);
  T q0 = 2.0 * v1 - 7.0 * v2 + 11.0 * v3;
  T q1 = -v2 + 5.0 * v3 + 2.0 * v4;
  T q2 = 2.0 * v3 + 5.0 * v4 - v5;
  return (a0 * q0 + a1 * q1 + a2 * q2) / (6.0 * (a0 + a1 + a2));
}

// ---------------------------------------------------------------------------
// Cut-cell geometry primitives (Sec. 2.3).  A point is inside material r if
// its local level-set value is positive, or zero while r owns the point (the
// smallest indicator among the cells that define it).
// ---------------------------------------------------------------------------
template <class T>
MMD bool inside(const T& v, int owner, int r) {
  return v > 0.0 || (v == 0.0 && owner == r);
}

template <class T>
MMD T seg_frac(T v0, bool in0, T v1, bool in1) {
  if (in0 && in1) return T(1.0);
  if (!in0 && !in1) return T(0.0);
  T vp = in0 ? v0 : v1, vm = in0 ? v1 : v0;
  if (vp <= 0.0) return T(0.0);
  return vp / (vp - vm);
}

template <class T>
MMD T tri_frac(T a, bool ia, T b, bool ib, T c, bool ic) {
  int n = (int)ia + (int)ib + (int)ic;
  if (n == 3) return T(1.0);
  if (n == 0) return T(0.0);
  if (n == 1) {
    T p = ia ? a : (ib ? b : c);
    T q = ia ? b : a;
    T r = ia ? c : (ib ? c : b);
    if (p <= 0.0) return T(0.0);
    return (p * p) / ((p - q) * (p - r));
  }
  T o = !ia ? a : (!ib ? b : c);
  T p = !ia ? b : a;
  T q = !ia ? c : (!ib ? c : b);
  if (o >= 0.0) return T(1.0);
  return 1.0 - (o * o) / ((o - p) * (o - q));
}

}  // namespace mmfv
