// Point-wise numerics of the cut-cell step, device side.
//
// Every expression is written in a fixed evaluation order and the library is
// compiled without floating-point contraction, so each operation is rounded
// exactly once as written; FP64 division and square root are the correctly
// rounded IEEE operations.  This makes results reproducible bit for bit
// across launch shapes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MMD __device__ __forceinline__

namespace mmfv {

constexpr int H = 4;       // halo width (WENO5 needs 3, extension 4)
constexpr int MAXM = 8;

struct Params {
  int dim, nx, ny, NX, NY, HY, NC, M;
  double dx, dy, h, bls, idx, idy, amix;
  int kext;
  double gamma[MAXM], pinf[MAXM], igm1[MAXM];
  int bc[4];
  double inflow_W[4];
  int inflow_mat;
  double cfl;
};

// ---------------------------------------------------------------------------
// Stiffened-gas EOS (Sec. 2.1): p = (gamma-1) rho e - gamma p_inf.
// ---------------------------------------------------------------------------
struct Prim {
  double r, u, v, p;
};

MMD Prim prim_from_U(double U0, double U1, double U2, double U3, double g,
                     double pinf) {
  Prim w;
  w.r = U0;
  w.u = U1 / U0;
  w.v = U2 / U0;
  double ke = 0.5 * w.r * (w.u * w.u + w.v * w.v);
  w.p = (g - 1.0) * (U3 - ke) - g * pinf;
  return w;
}

MMD double total_energy(double r, double u, double v, double p, double g,
                        double pinf, double igm1) {
  return (p + g * pinf) * igm1 + 0.5 * r * (u * u + v * v);
}

// ---------------------------------------------------------------------------
// HLLC with the two-EOS Roe-averaged wave-speed estimates (Sec. 2.3.2).
// States are (rho, u_normal, u_tangential, p).
// ---------------------------------------------------------------------------
MMD void wave_speeds(const Prim& L, double gL, double piL, const Prim& R,
                     double gR, double piR, double& SL, double& SR) {
  double irL = 1.0 / L.r, irR = 1.0 / R.r;
  double porL = L.p * irL, porR = R.p * irR;
  double psiL = (L.p + gL * piL) * irL, psiR = (R.p + gR * piR) * irR;
  double upsL = gL - 1.0, upsR = gR - 1.0;
  double cL = sqrt(psiL + upsL * porL);
  double cR = sqrt(psiR + upsR * porR);
  double sL = sqrt(L.r), sR = sqrt(R.r);
  double iw = 1.0 / (sL + sR);
  double psi_t = (sL * psiL + sR * psiR) * iw;
  double ups_t = (sL * upsL + sR * upsR) * iw;
  double u_t = (sL * L.u + sR * R.u) * iw;
  double du = (R.u - L.u) * iw;
  double por_t = (sL * porL + sR * porR) * iw + 0.5 * (sL * sR) * (du * du);
  double c_t = sqrt(psi_t + ups_t * por_t);
  SL = fmin(L.u - cL, u_t - c_t);
  SR = fmax(u_t + c_t, R.u + cR);
}

MMD double contact_speed(const Prim& L, const Prim& R, double SL, double SR) {
  double num = ((SR - R.u) * R.r * R.u + (L.u - SL) * L.r * L.u) + (L.p - R.p);
  double den = (SR - R.u) * R.r + (L.u - SL) * L.r;
  return num / den;
}

// HLLC face flux inside one material: F = (mass, normal mom, tangential mom,
// energy).
MMD void hllc_flux(const Prim& L, const Prim& R, double g, double pinf,
                   double igm1, double F[4]) {
  double SL, SR;
  wave_speeds(L, g, pinf, R, g, pinf, SL, SR);
  double SM = contact_speed(L, R, SL, SR);
  // upwind choice: F_L if S_L >= 0, else F*_L if S_M >= 0, else F*_R if
  // S_R > 0, else F_R
  bool left = (SL >= 0.0) || (SM >= 0.0);
  const Prim& K = left ? L : R;
  double Sk = left ? SL : SR;
  bool star = !(SL >= 0.0) && ((SM >= 0.0) || (SR > 0.0));
  double r = K.r, u = K.u, v = K.v, p = K.p;
  double E = total_energy(r, u, v, p, g, pinf, igm1);
  double ru = r * u;
  F[0] = ru;
  F[1] = ru * u + p;
  F[2] = ru * v;
  F[3] = u * (E + p);
  if (star) {
    double d = Sk - u;
    double mk = r * d;
    double coef = mk / (Sk - SM);
    double Us0 = coef;
    double Us1 = coef * SM;
    double Us2 = coef * v;
    double Us3 = coef * (E / r + (SM - u) * (SM + p / mk));
    F[0] = F[0] + Sk * (Us0 - r);
    F[1] = F[1] + Sk * (Us1 - ru);
    F[2] = F[2] + Sk * (Us2 - r * v);
    F[3] = F[3] + Sk * (Us3 - E);
  }
}

// ---------------------------------------------------------------------------
// WENO5-JS (Jiang-Shu), one division per reconstructed value: the nonlinear
// weights d_k/(eps+beta_k)^2 are scaled by the product of the three squared
// denominators and the 1/6 of the candidate stencils joins the same division.
// ---------------------------------------------------------------------------
MMD double weno5(double v1, double v2, double v3, double v4, double v5) {
  double t, u;
  t = v1 - 2.0 * v2 + v3;
  u = v1 - 4.0 * v2 + 3.0 * v3;
  double b0 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v2 - 2.0 * v3 + v4;
  u = v2 - v4;
  double b1 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v3 - 2.0 * v4 + v5;
  u = 3.0 * v3 - 4.0 * v4 + v5;
  double b2 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  double e0 = 1e-6 + b0, e1 = 1e-6 + b1, e2 = 1e-6 + b2;
  e0 = e0 * e0;
  e1 = e1 * e1;
  e2 = e2 * e2;
  double a0 = 0.1 * (e1 * e2);
  double a1 = 0.6 * (e0 * e2);
  double a2 = 0.3 * (e0 * e1);
  double q0 = 2.0 * v1 - 7.0 * v2 + 11.0 * v3;
  double q1 = -v2 + 5.0 * v3 + 2.0 * v4;
  double q2 = 2.0 * v3 + 5.0 * v4 - v5;
  return (a0 * q0 + a1 * q1 + a2 * q2) / (6.0 * (a0 + a1 + a2));
}

// ---------------------------------------------------------------------------
// Cut-cell geometry primitives (Sec. 2.3).  A point is inside material r if
// its local level-set value is positive, or zero while r owns the point (the
// smallest indicator among the cells that define it).
// ---------------------------------------------------------------------------
MMD bool inside(double v, int owner, int r) {
  return v > 0.0 || (v == 0.0 && owner == r);
}

MMD double seg_frac(double v0, bool in0, double v1, bool in1) {
  if (in0 && in1) return 1.0;
  if (!in0 && !in1) return 0.0;
  double vp = in0 ? v0 : v1, vm = in0 ? v1 : v0;
  if (vp <= 0.0) return 0.0;
  return vp / (vp - vm);
}

MMD double tri_frac(double a, bool ia, double b, bool ib, double c, bool ic) {
  int n = (int)ia + (int)ib + (int)ic;
  if (n == 3) return 1.0;
  if (n == 0) return 0.0;
  if (n == 1) {
    double p = ia ? a : (ib ? b : c);
    double q = ia ? b : a;
    double r = ia ? c : (ib ? c : b);
    if (p <= 0.0) return 0.0;
    return (p * p) / ((p - q) * (p - r));
  }
  double o = !ia ? a : (!ib ? b : c);
  double p = !ia ? b : a;
  double q = !ia ? c : (!ib ? c : b);
  if (o >= 0.0) return 1.0;
  return 1.0 - (o * o) / ((o - p) * (o - q));
}

}  // namespace mmfv
