/*
 * mmfv_oracle.c -- plain, slow, single-threaded FP64 CPU reference of one time
 * step of the conservative sharp-interface method for compressible
 * multi-material flows (Pan, Han, Hu & Adams, arXiv:1704.00519).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product library never links or calls it,
 * and the two share no code, headers or generated tables.
 *
 * Every routine below follows a passage of the paper (section / equation
 * named in its comment).  Where the paper is silent or garbled, the reading
 * taken is stated in the comment ("Reading: ...").  The loops are plain nested
 * loops over cells in row-major order; nothing is blocked, fused or reordered
 * beyond what the method states.
 *
 * Conventions
 *   * Uniform Cartesian grid, nx x ny interior cells (ny = 1 in 1D), a frame of
 *     H = 4 halo cells on every side (none in y for 1D).
 *   * Per-material conserved state Q^r = alpha^r U^r with 4 components
 *     (rho, rho u, rho v, rho E); in 1D the rho v component stays exactly 0.
 *   * Stiffened-gas EOS p = (gamma-1) rho e - gamma p_inf (ideal gas: p_inf = 0;
 *     Sec. 2.1 names the stiffened gas but prints no formula).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The arithmetic type of the state and of every computed quantity.  The
 * plain build (C) uses double.  The tangent build compiles this same file as
 * C++ with OR_TANGENT defined, where real carries a value and one directional
 * derivative (forward-mode differentiation); its values are computed by the
 * same double operations in the same order, so both builds take the same
 * branches and produce bitwise the same values.  RV() is the value of a
 * real, CONST_R() a real with the derivative dropped. */
#ifdef OR_TANGENT
#include "or_dual.h"
typedef or_dual real;
#define RV(x) or_value(x)
#define CONST_R(x) or_dual(or_value(x))
#else
typedef double real;
#define RV(x) (x)
#define CONST_R(x) (x)
#endif

#define OR_H 4
#define OR_NV 4
#define OR_MAXM 8

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_ENONPHYS = 4,
       OR_ESTATE = 5 };
enum { BC_TRANSMISSIVE = 0, BC_REFLECTIVE = 1, BC_INFLOW = 2, BC_OUTFLOW = 3 };

/* Plain-old-data configuration, laid out for ctypes. */
typedef struct {
  int32_t dim, nx, ny, n_mat;
  double x0, x1, y0, y1;
  double gamma[OR_MAXM], pinf[OR_MAXM];
  int32_t bc[4]; /* x-lo, x-hi, y-lo, y-hi */
  double inflow_W[4];
  int32_t inflow_mat, rk_order;
  double cfl, alpha_mix;
  int32_t k_ext, band_ls;
  /* Tait materials (Sec. 2.1, Tait's equation for water-like fluids):
     eos = 1 gives p = B (rho/rho0)^gamma - B + p0; eos = 0 the stiffened gas */
  int32_t eos[OR_MAXM];
  double rho0[OR_MAXM], tait_B[OR_MAXM], p0[OR_MAXM];
  int32_t flux;
  /* 1: the interface scale-separation model after every time step
     (Sec. 2.3.3) */
  int32_t scale_sep;
  /* coord = 1: 1D cylindrical (radial) geometry, x the radius (Sec. 3 Case
     II); fs_on = 1: material fs_mat is an ambient that is not solved, and
     its interfaces are free surfaces under the pressure law of fs_p (Case
     II's p(t): p_hi up to t0, then linear to p_lo at t1; reading: p_lo
     afterwards) */
  int32_t coord, fs_on, fs_mat;
  double fs_p[5];  /* p_hi, p_lo, t0, t1, density of the ambient */
  /* 1: redistancing of the regional level set after every time step
     (reading: the paper describes none) */
  int32_t reinit;
} or_config;

typedef struct {
  or_config c;
  int M, NX, NY, HY, NC;
  double dx, dy, h, bls, idx, idy;
  double igm1[OR_MAXM];
  /* p_inf of the energy relation: the stiffened gas's own, B - p0 for a Tait
     material (see energy()) */
  double pinfe[OR_MAXM];
  int tait[OR_MAXM];
  /* regional level set: current stage, time n, next stage */
  real *phi, *phin, *phit;
  int *chi, *chin, *chit;
  /* conserved state [M][4][NC]: current stage, time n, after the RK update */
  real *Q, *Qn, *Qt;
  /* cut-cell geometry [M][NC]; ax[k] is the x-face i+1/2 of cell k,
     ay[k] the y-face j+1/2 */
  real *al, *ax, *ay, *cx, *cy;
  /* primitive state and validity [M][4][NC], [M][NC] */
  real *W, *lw;
  unsigned char *Wv, *lok, *band, *band2;
  int *list;
  real *X;       /* interface exchange [M][4][NC] */
  real *vx, *vy; /* level-set advection velocity v^n */
  unsigned char *vok, *reg; /* velocity set / level-set update region */
  real *lv;       /* velocity extension scratch */
  real *Fx, *Fy; /* face fluxes [M][4][NC] */
  real *mass;    /* [M][NC] scratch for the volume-fraction correction */
  real *cv;      /* corner scratch [NC] */
  int *co;         /* corner owner scratch [NC] */
  unsigned char *xs; /* X_s bitmask [NC] */
  real *mixM;    /* [M][3][4][NC] mixing exchanges */
  int *mixT;       /* [M][3][NC] mixing target cell (-1 = none) */
  real inflow[4];  /* primitive state on inflow sides */
  double t, dt_fixed;
  real dt;         /* step size; its derivative is always zero (frozen) */
  long nstep;
  long n_posfix, n_fluxskip, n_ifskip, n_stranded, n_mixsrc, n_upd;
  long n_absorb, n_relabel, n_oddball;
  /* stranded mixing sources of a stage: cell, material and receiving
     material, in the order found; cells relabelled and their new material */
  int *abk, *abr, *rlk, *rlto;
  long nab, nrl;
  real bnd[OR_MAXM][OR_NV], bnd_c[OR_MAXM][OR_NV];
  real xsum[OR_MAXM][OR_NV], xsum_c[OR_MAXM][OR_NV];
  /* conserved quantities moved between materials of one cell (stranded
     sources, scale separation): received minus given, per material */
  real xfer[OR_MAXM][OR_NV], xfer_c[OR_MAXM][OR_NV];
  double xw;       /* weight in the full step of a change to the stage state */
  double tstage;   /* time of the current stage's input state */
  int err_code;
  long err_cell;
} St;

#define ID(s, i, j) (((j) + (s)->HY) * (s)->NX + (i) + OR_H)
/* the ambient material of a free surface (not solved) */
#define PASSIVE(s, r) ((s)->c.fs_on && (r) == (s)->c.fs_mat)
#define M1(s, a, m, k) ((a)[(size_t)(m) * (s)->NC + (k)])
#define M4(s, a, m, v, k) ((a)[((size_t)(m) * OR_NV + (v)) * (s)->NC + (k)])

static void neumaier(real *sum, real *comp, real x) {
  real t = *sum + x;
  if (fabs(*sum) >= fabs(x))
    *comp += (*sum - t) + x;
  else
    *comp += (x - t) + *sum;
  *sum = t;
}

/* ------------------------------------------------------------------------ */
/* Thermodynamics (Sec. 2.1; general-EOS sound speed, Sec. 2.3.2)            */
/* ------------------------------------------------------------------------ */

/* primitive (rho, u, v, p) from conserved cell averages U (not alpha U).
 * Stiffened gas: p = (gamma-1)(rho E - rho |u|^2/2) - gamma p_inf.  Tait
 * (Sec. 2.1): p = B (rho/rho0)^gamma - B + p0, a function of density alone. */
static void prim(const St *s, int m, const real *U, real *W) {
  double g = s->c.gamma[m], pinf = s->pinfe[m];
  real rho = U[0];
  real u = U[1] / rho;
  real v = U[2] / rho;
  real ke = 0.5 * rho * (u * u + v * v);
  W[0] = rho;
  W[1] = u;
  W[2] = v;
  if (s->tait[m])
    W[3] = s->c.tait_B[m] * pow(rho / s->c.rho0[m], g) - pinf;
  else
    W[3] = (g - 1.0) * (U[3] - ke) - g * pinf;
}

/* total energy density rho E of a primitive state.  Reading for a Tait
 * material (the paper gives no energy relation for it): the internal energy
 * of the stiffened gas with the same gamma and p_inf = B - p0, so that
 * rho E is defined and c^2 = gamma (p + B - p0)/rho as for that gas; the
 * pressure itself never depends on the energy. */
static real energy(const St *s, int m, real rho, real u, real v,
                     real p) {
  double g = s->c.gamma[m], pinf = s->pinfe[m];
  return (p + g * pinf) * s->igm1[m] + 0.5 * rho * (u * u + v * v);
}

/* Wave-speed estimates of the HLLC solver for two states that may obey
 * different EOS (Sec. 2.3.2, the S_L/S_R estimate and the Roe averages of
 * Psi, Upsilon and p/rho).  Stiffened gas: Psi = (p + gamma p_inf)/rho,
 * Upsilon = gamma - 1, so c^2 = Psi + Upsilon p/rho = gamma (p + p_inf)/rho.
 * States are (rho, u_normal, u_tangential, p). */
static void wave_speeds(const real *WL, double gL, double piL, int tL,
                        const real *WR, double gR, double piR, int tR, real *SL,
                        real *SR) {
  real rL = WL[0], uL = WL[1], pL = WL[3];
  real rR = WR[0], uR = WR[1], pR = WR[3];
  real irL = 1.0 / rL, irR = 1.0 / rR;
  real porL = pL * irL, porR = pR * irR;
  /* Tait: Psi = dp/drho = gamma (p + B - p0)/rho, Upsilon = 0 */
  real psiL = tL ? gL * (pL + piL) * irL : (pL + gL * piL) * irL;
  real psiR = tR ? gR * (pR + piR) * irR : (pR + gR * piR) * irR;
  double upsL = tL ? 0.0 : gL - 1.0, upsR = tR ? 0.0 : gR - 1.0;
  real cL = sqrt(psiL + upsL * porL);
  real cR = sqrt(psiR + upsR * porR);
  real sL = sqrt(rL), sR = sqrt(rR);
  real iw = 1.0 / (sL + sR);
  real psi_t = (sL * psiL + sR * psiR) * iw;
  real ups_t = (sL * upsL + sR * upsR) * iw;
  real u_t = (sL * uL + sR * uR) * iw;
  real du = (uR - uL) * iw;
  real por_t = (sL * porL + sR * porR) * iw + 0.5 * (sL * sR) * (du * du);
  real c_t = sqrt(psi_t + ups_t * por_t);
  *SL = fmin(uL - cL, u_t - c_t);
  *SR = fmax(u_t + c_t, uR + cR);
}

/* Contact speed S_M of Toro's HLLC solver (Sec. 2.3.2).  The two momentum
 * terms and the pressure difference are summed separately, so swapping the
 * two states and the sign of the velocities gives exactly -S_M. */
static real contact_speed(const real *WL, const real *WR, real SL,
                            real SR) {
  real rL = WL[0], uL = WL[1], pL = WL[3];
  real rR = WR[0], uR = WR[1], pR = WR[3];
  real num = ((SR - uR) * rR * uR + (uL - SL) * rL * uL) + (pL - pR);
  real den = (SR - uR) * rR + (uL - SL) * rL;
  return num / den;
}

/* HLLC flux (Toro) across a cell face inside one material.  W are
 * (rho, u_n, u_t, p); F = (mass, normal momentum, tangential momentum,
 * energy). */
static void hllc_flux(const St *s, int m, const real *WL, const real *WR,
                      real *F) {
  double g = s->c.gamma[m], pinf = s->pinfe[m];
  int t = s->tait[m];
  real SL, SR;
  wave_speeds(WL, g, pinf, t, WR, g, pinf, t, &SL, &SR);
  real SM = contact_speed(WL, WR, SL, SR);
  const real *Wk;
  real Sk;
  int star;
  if (SL >= 0.0) {
    Wk = WL; Sk = SL; star = 0;
  } else if (SM >= 0.0) {
    Wk = WL; Sk = SL; star = 1;
  } else if (SR > 0.0) {
    Wk = WR; Sk = SR; star = 1;
  } else {
    Wk = WR; Sk = SR; star = 0;
  }
  real r = Wk[0], u = Wk[1], v = Wk[2], p = Wk[3];
  real E = energy(s, m, r, u, v, p);
  real ru = r * u;
  F[0] = ru;
  F[1] = ru * u + p;
  F[2] = ru * v;
  F[3] = u * (E + p);
  if (star) {
    real d = Sk - u;
    real mk = r * d;
    real coef = mk / (Sk - SM);
    real Us0 = coef;
    real Us1 = coef * SM;
    real Us2 = coef * v;
    real Us3 = coef * (E / r + (SM - u) * (SM + p / mk));
    F[0] = F[0] + Sk * (Us0 - r);
    F[1] = F[1] + Sk * (Us1 - ru);
    F[2] = F[2] + Sk * (Us2 - r * v);
    F[3] = F[3] + Sk * (Us3 - E);
  }
}

/* ------------------------------------------------------------------------ */
/* 5th-order WENO-JS (Sec. 3 intro: fluid and level set use 5th-order WENO) */
/* ------------------------------------------------------------------------ */
/* Left-biased value at i+1/2 from (v1..v5) = (f_{i-2}, ..., f_{i+2}).
 * Jiang-Shu smoothness indicators, linear weights (1/10, 6/10, 3/10),
 * eps = 1e-6, power 2.  The nonlinear weights d_k/(eps+beta_k)^2 are
 * multiplied through by the product of the three squared denominators, so
 * the normalised combination needs a single division; the 1/6 of the three
 * candidate stencils is folded into the same division.  Algebraically this is
 * the textbook formula. */
static real weno5(real v1, real v2, real v3, real v4, real v5) {
  real t, u;
  t = v1 - 2.0 * v2 + v3;
  u = v1 - 4.0 * v2 + 3.0 * v3;
  real b0 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v2 - 2.0 * v3 + v4;
  u = v2 - v4;
  real b1 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  t = v3 - 2.0 * v4 + v5;
  u = 3.0 * v3 - 4.0 * v4 + v5;
  real b2 = (13.0 / 12.0) * (t * t) + 0.25 * (u * u);
  real e0 = 1e-6 + b0, e1 = 1e-6 + b1, e2 = 1e-6 + b2;
  e0 = e0 * e0;
  e1 = e1 * e1;
  e2 = e2 * e2;
  real a0 = 0.1 * (e1 * e2);
  real a1 = 0.6 * (e0 * e2);
  real a2 = 0.3 * (e0 * e1);
  real q0 = 2.0 * v1 - 7.0 * v2 + 11.0 * v3;
  real q1 = -v2 + 5.0 * v3 + 2.0 * v4;
  real q2 = 2.0 * v3 + 5.0 * v4 - v5;
  return (a0 * q0 + a1 * q1 + a2 * q2) / (6.0 * (a0 + a1 + a2));
}

/* ------------------------------------------------------------------------ */
/* Boundary frames                                                          */
/* ------------------------------------------------------------------------ */
/* Reading: transmissive/outflow = zero-gradient copy, reflective = mirror
 * with the normal velocity negated, inflow = a fixed state of one material
 * (Case V: inflow/outflow left/right, symmetric top/bottom). */
static int src_lo(int i, int type) { return type == BC_REFLECTIVE ? -1 - i : 0; }
static int src_hi(int i, int n, int type) {
  return type == BC_REFLECTIVE ? 2 * n - 1 - i : n - 1;
}

static void fill_d(St *s, real *f, double sx, double sy) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int j = 0; j < ny; j++)
    for (int i = -OR_H; i < 0; i++) {
      int tl = s->c.bc[0], th = s->c.bc[1];
      f[ID(s, i, j)] = f[ID(s, src_lo(i, tl), j)] * (tl == BC_REFLECTIVE ? sx : 1.0);
      int ih = nx + (-1 - i); /* nx .. nx+3 */
      f[ID(s, ih, j)] = f[ID(s, src_hi(ih, nx, th), j)] * (th == BC_REFLECTIVE ? sx : 1.0);
    }
  if (s->c.dim < 2) return;
  for (int i = -OR_H; i < nx + OR_H; i++)
    for (int j = -OR_H; j < 0; j++) {
      int tl = s->c.bc[2], th = s->c.bc[3];
      f[ID(s, i, j)] = f[ID(s, i, src_lo(j, tl))] * (tl == BC_REFLECTIVE ? sy : 1.0);
      int jh = ny + (-1 - j);
      f[ID(s, i, jh)] = f[ID(s, i, src_hi(jh, ny, th))] * (th == BC_REFLECTIVE ? sy : 1.0);
    }
}

static void fill_i(St *s, int *f) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int j = 0; j < ny; j++)
    for (int i = -OR_H; i < 0; i++) {
      f[ID(s, i, j)] = f[ID(s, src_lo(i, s->c.bc[0]), j)];
      int ih = nx + (-1 - i);
      f[ID(s, ih, j)] = f[ID(s, src_hi(ih, nx, s->c.bc[1]), j)];
    }
  if (s->c.dim < 2) return;
  for (int i = -OR_H; i < nx + OR_H; i++)
    for (int j = -OR_H; j < 0; j++) {
      f[ID(s, i, j)] = f[ID(s, i, src_lo(j, s->c.bc[2]))];
      int jh = ny + (-1 - j);
      f[ID(s, i, jh)] = f[ID(s, i, src_hi(jh, ny, s->c.bc[3]))];
    }
}

/* Primitive-state frame of every material.  On an inflow side the inflow
 * material receives the fixed state; the other materials are copied. */
static void fill_W(St *s) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int m = 0; m < s->M; m++) {
    real *f[4];
    for (int v = 0; v < 4; v++) f[v] = &M4(s, s->W, m, v, 0);
    unsigned char *fv = &M1(s, s->Wv, m, 0);
    /* x sides */
    for (int v = 0; v < 4; v++) {
      double sx = (v == 1) ? -1.0 : 1.0;
      for (int j = 0; j < ny; j++)
        for (int i = -OR_H; i < 0; i++) {
          int tl = s->c.bc[0], th = s->c.bc[1];
          f[v][ID(s, i, j)] = f[v][ID(s, src_lo(i, tl), j)] * (tl == BC_REFLECTIVE ? sx : 1.0);
          int ih = nx + (-1 - i);
          f[v][ID(s, ih, j)] = f[v][ID(s, src_hi(ih, nx, th), j)] * (th == BC_REFLECTIVE ? sx : 1.0);
        }
    }
    for (int j = 0; j < ny; j++)
      for (int i = -OR_H; i < 0; i++) {
        fv[ID(s, i, j)] = fv[ID(s, src_lo(i, s->c.bc[0]), j)];
        int ih = nx + (-1 - i);
        fv[ID(s, ih, j)] = fv[ID(s, src_hi(ih, nx, s->c.bc[1]), j)];
      }
    for (int side = 0; side < 2; side++)
      if (s->c.bc[side] == BC_INFLOW && m == s->c.inflow_mat)
        for (int j = 0; j < ny; j++)
          for (int i = -OR_H; i < 0; i++) {
            int ii = side == 0 ? i : nx + (-1 - i);
            for (int v = 0; v < 4; v++) f[v][ID(s, ii, j)] = s->inflow[v];
            fv[ID(s, ii, j)] = 1;
          }
    if (s->c.dim < 2) continue;
    /* y sides */
    for (int v = 0; v < 4; v++) {
      double sy = (v == 2) ? -1.0 : 1.0;
      for (int i = -OR_H; i < nx + OR_H; i++)
        for (int j = -OR_H; j < 0; j++) {
          int tl = s->c.bc[2], th = s->c.bc[3];
          f[v][ID(s, i, j)] = f[v][ID(s, i, src_lo(j, tl))] * (tl == BC_REFLECTIVE ? sy : 1.0);
          int jh = ny + (-1 - j);
          f[v][ID(s, i, jh)] = f[v][ID(s, i, src_hi(jh, ny, th))] * (th == BC_REFLECTIVE ? sy : 1.0);
        }
    }
    for (int i = -OR_H; i < nx + OR_H; i++)
      for (int j = -OR_H; j < 0; j++) {
        fv[ID(s, i, j)] = fv[ID(s, i, src_lo(j, s->c.bc[2]))];
        int jh = ny + (-1 - j);
        fv[ID(s, i, jh)] = fv[ID(s, i, src_hi(jh, ny, s->c.bc[3]))];
      }
    for (int side = 2; side < 4; side++)
      if (s->c.bc[side] == BC_INFLOW && m == s->c.inflow_mat)
        for (int i = -OR_H; i < nx + OR_H; i++)
          for (int j = -OR_H; j < 0; j++) {
            int jj = side == 2 ? j : ny + (-1 - j);
            for (int v = 0; v < 4; v++) f[v][ID(s, i, jj)] = s->inflow[v];
            fv[ID(s, i, jj)] = 1;
          }
  }
}

static void fill_ls(St *s, real *phi, int *chi) {
  fill_d(s, phi, 1.0, 1.0);
  fill_i(s, chi);
}

/* ------------------------------------------------------------------------ */
/* Multi-region level set (Sec. 2.2)                                        */
/* ------------------------------------------------------------------------ */
/* Construction operator C_r (Eq. construction): +phi inside material r,
 * -phi elsewhere. */
static real lsv(const real *phi, const int *chi, int r, int k) {
  return chi[k] == r ? phi[k] : -phi[k];
}

/* Local material set X_s: the distinct indicators of the 3x3 block around a
 * cell.  Reading: the strict inequalities printed for V_s would select the
 * cell alone; the block of the cell and its 8 neighbours is meant. */
static void local_sets(St *s, const int *chi, unsigned char *xs) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      unsigned char b = 0;
      for (int dj = -two; dj <= two; dj++)
        for (int di = -1; di <= 1; di++) b |= (unsigned char)(1u << chi[ID(s, i + di, j + dj)]);
      xs[ID(s, i, j)] = b;
    }
}

/* ------------------------------------------------------------------------ */
/* Cut-cell geometry (Sec. 2.3: volume fraction alpha, apertures A,          */
/* interface segment Delta Omega)                                           */
/* ------------------------------------------------------------------------ */
/* Reading (tie rule): a point is inside material r if its local level-set
 * value is positive, or zero while r is the smallest indicator among the
 * cells that define the point; this gives every zero a single owner. */
static int inside(real v, int owner, int r) {
  return v > 0.0 || (v == 0.0 && owner == r);
}

/* Fraction of a segment on which the linear interpolant of its end values is
 * inside. */
static real seg_frac(real v0, int in0, real v1, int in1) {
  if (in0 && in1) return 1.0;
  if (!in0 && !in1) return 0.0;
  real vp = in0 ? v0 : v1, vm = in0 ? v1 : v0;
  if (vp <= 0.0) return 0.0;
  return vp / (vp - vm);
}

/* Fraction of a triangle on which the linear interpolant of its vertex values
 * is inside. */
static real tri_frac(real a, int ia, real b, int ib, real c, int ic) {
  int n = ia + ib + ic;
  if (n == 3) return 1.0;
  if (n == 0) return 0.0;
  if (n == 1) {
    real p, q, r;
    if (ia) { p = a; q = b; r = c; }
    else if (ib) { p = b; q = a; r = c; }
    else { p = c; q = a; r = b; }
    if (p <= 0.0) return 0.0;
    return (p * p) / ((p - q) * (p - r));
  }
  real o, p, q;
  if (!ia) { o = a; p = b; q = c; }
  else if (!ib) { o = b; p = a; q = c; }
  else { o = c; p = a; q = b; }
  if (o >= 0.0) return 1.0;
  return 1.0 - (o * o) / ((o - p) * (o - q));
}

/* Volume fractions, face apertures and interface closure vectors of every
 * material, from the regional level set (phi, chi) with filled frame.
 * Reading (geometry; the two-phase formulas of hu2006conservative are not
 * reproduced in the paper): in 2D the local level set is interpolated
 * piecewise linearly on the four triangles spanned by the cell centre and
 * each face; corner values are the mean of the four surrounding cells.  The
 * aperture of a face is the inside fraction of the linear interpolant between
 * its two corners, the volume fraction the inside area fraction of the four
 * triangles.  In 1D the face value is the mean of the two cells.  The
 * interface segment Delta Omega^r times its normal (pointing into r) closes
 * the polygon: c^r = ((A_{i+1/2} - A_{i-1/2}) dy, (A_{j+1/2} - A_{j-1/2}) dx). */
static void geometry(St *s, const real *phi, const int *chi) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int r = 0; r < s->M; r++) {
    real *al = &M1(s, s->al, r, 0), *ax = &M1(s, s->ax, r, 0),
           *ay = &M1(s, s->ay, r, 0), *cx = &M1(s, s->cx, r, 0),
           *cy = &M1(s, s->cy, r, 0);
    if (s->c.dim == 1) {
      for (int i = -1; i < nx; i++) {
        int a = ID(s, i, 0), b = ID(s, i + 1, 0);
        real f = (lsv(phi, chi, r, a) + lsv(phi, chi, r, b)) * 0.5;
        int own = chi[a] < chi[b] ? chi[a] : chi[b];
        s->cv[a] = f;
        s->co[a] = own;
        ax[a] = inside(f, own, r) ? 1.0 : 0.0;
      }
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, 0), kl = ID(s, i - 1, 0);
        real c = lsv(phi, chi, r, k);
        int ic = inside(c, chi[k], r);
        int il = inside(s->cv[kl], s->co[kl], r), ir = inside(s->cv[k], s->co[k], r);
        al[k] = (seg_frac(s->cv[kl], il, c, ic) + seg_frac(c, ic, s->cv[k], ir)) * 0.5;
        cx[k] = ax[k] - ax[kl];
        if (s->c.coord == 1) {
          /* cylindrical: the interface area r_s per cell volume r_i dx, from
             the faces' areas and the volume fraction (alpha dx = r_s - r_{i-1/2}
             for a material on the inner side), so that a uniform pressure
             balances the faces, the geometric source and the exchange */
          double rl = s->c.x0 + i * s->dx, rr = s->c.x0 + (i + 1) * s->dx;
          double ri = s->c.x0 + (i + 0.5) * s->dx;
          cx[k] = ((ax[k] * rr - ax[kl] * rl) - al[k] * s->dx) / ri;
        }
        cy[k] = 0.0;
      }
      continue;
    }
    /* corners (i+1/2, j+1/2) for i, j in [-1, n) */
    for (int j = -1; j < ny; j++)
      for (int i = -1; i < nx; i++) {
        int k00 = ID(s, i, j), k10 = ID(s, i + 1, j), k01 = ID(s, i, j + 1),
            k11 = ID(s, i + 1, j + 1);
        real v = ((lsv(phi, chi, r, k00) + lsv(phi, chi, r, k11)) +
                    (lsv(phi, chi, r, k10) + lsv(phi, chi, r, k01))) * 0.25;
        int own = chi[k00];
        if (chi[k10] < own) own = chi[k10];
        if (chi[k01] < own) own = chi[k01];
        if (chi[k11] < own) own = chi[k11];
        s->cv[k00] = v;
        s->co[k00] = own;
      }
    /* x-faces i+1/2 (i in [-1,nx)), endpoints corners (i, j-1) and (i, j) */
    for (int j = 0; j < ny; j++)
      for (int i = -1; i < nx; i++) {
        int ka = ID(s, i, j - 1), kb = ID(s, i, j);
        ax[kb] = seg_frac(s->cv[ka], inside(s->cv[ka], s->co[ka], r), s->cv[kb],
                          inside(s->cv[kb], s->co[kb], r));
      }
    /* y-faces j+1/2 (j in [-1,ny)), endpoints corners (i-1, j) and (i, j) */
    for (int j = -1; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int ka = ID(s, i - 1, j), kb = ID(s, i, j);
        ay[kb] = seg_frac(s->cv[ka], inside(s->cv[ka], s->co[ka], r), s->cv[kb],
                          inside(s->cv[kb], s->co[kb], r));
      }
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, j);
        int ksw = ID(s, i - 1, j - 1), kse = ID(s, i, j - 1), knw = ID(s, i - 1, j),
            kne = k;
        real c = lsv(phi, chi, r, k);
        int ic = inside(c, chi[k], r);
        real vsw = s->cv[ksw], vse = s->cv[kse], vnw = s->cv[knw], vne = s->cv[kne];
        int isw = inside(vsw, s->co[ksw], r), ise = inside(vse, s->co[kse], r),
            inw = inside(vnw, s->co[knw], r), ine = inside(vne, s->co[kne], r);
        real tl = tri_frac(vsw, isw, vnw, inw, c, ic);
        real tr = tri_frac(vse, ise, vne, ine, c, ic);
        real tb = tri_frac(vsw, isw, vse, ise, c, ic);
        real tt = tri_frac(vnw, inw, vne, ine, c, ic);
        al[k] = ((tl + tr) + (tb + tt)) * 0.25;
        cx[k] = (ax[k] - ax[ID(s, i - 1, j)]) * s->dy;
        cy[k] = (ay[k] - ay[ID(s, i, j - 1)]) * s->dx;
      }
  }
}

/* Volume-fraction correction for a multi-material-cell (Sec. 2.3.1,
 * Eq. vol_corr2): in cells where three or more materials have alpha > 0, the
 * material of least mass alpha*rho (the cell's own indicator excluded, it is
 * not changed) absorbs 1 - sum(alpha).  Reading: ties go to the smaller
 * index; if the lightest would become negative it is set to 0 and the rest
 * passes to the next lightest.  mass[m][k] is the partial density. */
static void vf_correction(St *s, const int *chi, const real *mass) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j), n = 0;
      for (int r = 0; r < s->M; r++)
        if (M1(s, s->al, r, k) > 0.0) n++;
      if (n < 3) continue;
      real sum = 0.0;
      for (int r = 0; r < s->M; r++) sum += M1(s, s->al, r, k);
      real d = 1.0 - sum;
      int used = 0;
      while (d != 0.0) {
        int best = -1;
        for (int r = 0; r < s->M; r++) {
          if (r == chi[k] || (used >> r & 1) || !(M1(s, s->al, r, k) > 0.0)) continue;
          if (best < 0 || M1(s, mass, r, k) < M1(s, mass, best, k)) best = r;
        }
        if (best < 0) break;
        used |= 1 << best;
        real nv = M1(s, s->al, best, k) + d;
        if (nv < 0.0) {
          M1(s, s->al, best, k) = 0.0;
          d = nv;
        } else {
          M1(s, s->al, best, k) = nv;
          d = 0.0;
        }
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Real and ghost primitive states (Sec. 2.3.2: the real state of the       */
/* primary material, the ghost state otherwise)                             */
/* ------------------------------------------------------------------------ */
static void record_err(St *s, int code, int i, int j) {
  long lin = (long)j * s->c.nx + i;
  if (s->err_code == OR_OK || lin < s->err_cell) {
    s->err_code = code;
    s->err_cell = lin;
  }
}

/* Real cells of material r: chi == r and alpha^r > 0; W = prim(Q / alpha).
 * Reading (guards): rho <= 0, p + p_inf <= 0 or a non-finite value there is
 * a non-physical state and stops the run. */
/* Pressure on a free surface at time t (Sec. 3 Case II). */
static double fs_pressure(const St *s, double t) {
  const double *f = s->c.fs_p;
  if (t <= f[2]) return f[0];
  if (t >= f[3]) return f[1];
  return f[0] - (f[0] - f[1]) * (t - f[2]) / (f[3] - f[2]);
}

/* The ambient of a free surface is not solved: its state is the prescribed
 * one (the ambient density, at rest, at the surface pressure of the stage's
 * time) in every cell, and its conserved quantities alpha U of that state. */
static void ambient_state(St *s) {
  int r = s->c.fs_mat, nx = s->c.nx, ny = s->c.ny;
  real W[4] = {s->c.fs_p[4], 0.0, 0.0, fs_pressure(s, s->tstage)};
  real E = energy(s, r, W[0], W[1], W[2], W[3]);
  for (size_t k = 0; k < (size_t)s->NC; k++) {
    for (int v = 0; v < 4; v++) M4(s, s->W, r, v, k) = W[v];
    M1(s, s->Wv, r, k) = 1;
  }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      real a = M1(s, s->al, r, k);
      real U[4] = {W[0], 0.0, 0.0, E};
      for (int v = 0; v < 4; v++) M4(s, s->Q, r, v, k) = a > 0.0 ? a * U[v] : 0.0;
    }
}

static void real_states(St *s) {
  int nx = s->c.nx, ny = s->c.ny;
  memset(s->Wv, 0, (size_t)s->M * s->NC);
  if (s->c.fs_on) ambient_state(s);
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j), r = s->chi[k];
      real a = M1(s, s->al, r, k);
      if (!(a > 0.0) || PASSIVE(s, r)) continue;
      real U[4], W[4];
      for (int v = 0; v < 4; v++) U[v] = M4(s, s->Q, r, v, k) / a;
      prim(s, r, U, W);
      if (!(W[0] > 0.0) || !(W[3] + s->pinfe[r] > 0.0) || !isfinite(W[1]) ||
          !isfinite(W[2]) || !isfinite(W[0]) || !isfinite(W[3]))
        record_err(s, OR_ENONPHYS, i, j);
      for (int v = 0; v < 4; v++) M4(s, s->W, r, v, k) = W[v];
      M1(s, s->Wv, r, k) = 1;
    }
}

/* Ghost states by extrapolation (the paper defers to hu2006conservative).
 * Reading: cells within Chebyshev distance 4 of a real cell of r form its
 * ghost band.  Jacobi sweeps take each ghost cell from its upwind neighbours
 * along the direction of increasing phi^r (central differences), weighted
 * by the gradient components; only neighbours valid after the previous sweep
 * count.  k_ext such sweeps are followed by 4 sweeps that take the mean of
 * the valid 8-neighbours (2-neighbours in 1D) for any cell still empty, which
 * reaches every cell of the band. */
static void extension(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2, R = 4;
  size_t nc = s->NC;
  for (int r = 0; r < s->M; r++) {
    unsigned char *v = &M1(s, s->Wv, r, 0);
    unsigned char *rb = s->band2, *b = s->band;
    /* ghost band: dilation of the real mask by R cells (rows, then columns) */
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        unsigned char h = 0;
        for (int di = -R; di <= R; di++)
          if (i + di >= 0 && i + di < nx) h |= v[ID(s, i + di, j)];
        rb[ID(s, i, j)] = h;
      }
    int n = 0;
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        unsigned char h = 0;
        for (int dj = -R * two; dj <= R * two; dj++)
          if (j + dj >= 0 && j + dj < ny) h |= rb[ID(s, i, j + dj)];
        b[ID(s, i, j)] = h;
        if (h && !v[ID(s, i, j)]) s->list[n++] = ID(s, i, j);
      }
    int sweeps = s->c.k_ext + 4;
    for (int it = 0; it < sweeps; it++) {
      int upwind = it < s->c.k_ext;
      for (int q = 0; q < n; q++) {
        int k = s->list[q];
        int i = k % s->NX - OR_H, j = k / s->NX - s->HY;
        real *out = &s->lw[(size_t)q * 4];
        s->lok[q] = 0;
        if (v[k]) continue;
        if (upwind) {
          real gx = lsv(s->phi, s->chi, r, ID(s, i + 1, j)) - lsv(s->phi, s->chi, r, ID(s, i - 1, j));
          real gy = two ? lsv(s->phi, s->chi, r, ID(s, i, j + 1)) - lsv(s->phi, s->chi, r, ID(s, i, j - 1)) : 0.0;
          int kx = -1, ky = -1;
          if (gx != 0.0) {
            int ii = i + (gx > 0.0 ? 1 : -1);
            if (ii >= 0 && ii < nx && v[ID(s, ii, j)]) kx = ID(s, ii, j);
          }
          if (gy != 0.0) {
            int jj = j + (gy > 0.0 ? 1 : -1);
            if (jj >= 0 && jj < ny && v[ID(s, i, jj)]) ky = ID(s, i, jj);
          }
          if (kx >= 0 && ky >= 0) {
            real wx = fabs(gx), wy = fabs(gy);
            for (int c = 0; c < 4; c++)
              out[c] = (wx * M4(s, s->W, r, c, kx) + wy * M4(s, s->W, r, c, ky)) / (wx + wy);
            s->lok[q] = 1;
          } else if (kx >= 0) {
            for (int c = 0; c < 4; c++) out[c] = M4(s, s->W, r, c, kx);
            s->lok[q] = 1;
          } else if (ky >= 0) {
            for (int c = 0; c < 4; c++) out[c] = M4(s, s->W, r, c, ky);
            s->lok[q] = 1;
          }
        } else {
          /* mean of the valid neighbours, summed in mirror-symmetric pairs:
             rows (-1 + +1) + 0, within a row (-1 + +1) + 0 */
          real row[3][4];
          int cnt = 0;
          for (int dj = -1; dj <= 1; dj++) {
            real a[3][4];
            for (int di = -1; di <= 1; di++) {
              int ii = i + di, jj = j + dj, ok2 = 0;
              if ((di != 0 || dj != 0) && (two || dj == 0) && ii >= 0 && ii < nx &&
                  jj >= 0 && jj < ny && v[ID(s, ii, jj)]) ok2 = 1;
              for (int c = 0; c < 4; c++)
                a[di + 1][c] = ok2 ? M4(s, s->W, r, c, ID(s, ii, jj)) : 0.0;
              cnt += ok2;
            }
            for (int c = 0; c < 4; c++) row[dj + 1][c] = (a[0][c] + a[2][c]) + a[1][c];
          }
          if (cnt > 0) {
            for (int c = 0; c < 4; c++)
              out[c] = ((row[0][c] + row[2][c]) + row[1][c]) / (real)cnt;
            s->lok[q] = 1;
          }
        }
      }
      /* Jacobi: commit after the whole sweep */
      for (int q = 0; q < n; q++) {
        if (!s->lok[q]) continue;
        int k = s->list[q];
        for (int c = 0; c < 4; c++) M4(s, s->W, r, c, k) = s->lw[(size_t)q * 4 + c];
        v[k] = 1;
      }
    }
  }
  (void)nc;
}

static real wave_jump(const St *s, int m, const real *W, real ps);

/* Free surface (Sec. 3 Case II): the ambient's own waves are not solved, so
 * the surface's Riemann problem against the prescribed pressure ps can be far
 * faster than the solved side's sound speed.  Reading: in a cell holding the
 * surface, the step is bounded by max(|u|, |v|) + |du| + c_s for every solved
 * material present, du the velocity jump of its wave to ps and c_s that
 * wave's front speed relative to the material (c for a rarefaction; the
 * stiffened-gas shock speed c sqrt(1 + (g + 1)/(2 g) (ps - p)/(p + pinf))
 * for a shock). */
static real fs_speed(St *s, int k) {
  real ps = fs_pressure(s, s->tstage), smax = 0.0;
  for (int m = 0; m < s->M; m++) {
    if (!(s->xs[k] >> m & 1) || PASSIVE(s, m) || !M1(s, s->Wv, m, k)) continue;
    real W[4] = {M4(s, s->W, m, 0, k), M4(s, s->W, m, 1, k), M4(s, s->W, m, 2, k),
                 M4(s, s->W, m, 3, k)};
    double g = s->c.gamma[m];
    real pb = W[3] + s->pinfe[m];
    real c = sqrt(g * pb / W[0]);
    if (ps > W[3]) c = c * sqrt(1.0 + (g + 1.0) / (2.0 * g) * ((ps - W[3]) / pb));
    real u = fabs(W[1]), v = fabs(W[2]);
    real w = (u > v ? u : v) + fabs(wave_jump(s, m, W, ps)) + c;
    if (w > smax) smax = w;
  }
  return smax;
}

/* CFL time step (Sec. 2.3, Sec. 3: CFL number 0.6).  Reading: one step size
 * per time step from the time-n state, dt = CFL h / max over real cells of
 * max(|u| + c, |v| + c). */
static real cfl_dt(St *s) {
  int nx = s->c.nx, ny = s->c.ny;
  real smax = 0.0;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j), r = s->chi[k];
      if (!M1(s, s->Wv, r, k) || PASSIVE(s, r)) continue;
      real rho = M4(s, s->W, r, 0, k), u = M4(s, s->W, r, 1, k),
             v = M4(s, s->W, r, 2, k), p = M4(s, s->W, r, 3, k);
      real c = sqrt(s->c.gamma[r] * (p + s->pinfe[r]) / rho);
      real a = fabs(u) + c, b = fabs(v) + c;
      real w = a > b ? a : b;
      if (w > smax) smax = w;
      if (s->c.fs_on && (s->xs[k] >> s->c.fs_mat & 1)) {
        w = fs_speed(s, k);
        if (w > smax) smax = w;
      }
    }
  return s->c.cfl * s->h / smax;
}

/* ------------------------------------------------------------------------ */
/* Reduced interface-interaction model (Sec. 2.3.2)                          */
/* ------------------------------------------------------------------------ */
/* In every cell whose local set holds two or more materials only the two
 * heaviest (by partial mass alpha rho = Q_rho) interact: a the heavier, b the
 * other; ties go to the smaller index.  The interface is present when the
 * closure vector c^a of a is non-zero.  Its normal n = c^a/|c^a| points into
 * a (Reading: the closure vector replaces grad phi^a / |grad phi^a|; the two
 * agree to first order, and this choice keeps a uniform pressure exactly in
 * equilibrium).  The Riemann problem takes the lighter material as the left
 * state and the heavier as the right one, each the real state where it is
 * the cell's indicator and its ghost state otherwise.  With the HLLC contact
 * speed S_M and star pressure p* the exchange is
 * X^a = (0, p* c^a_x, p* c^a_y, p* S_M |c^a|), X^b = -X^a, zero for every
 * other material.  Reading: p* is the mean of its two equal forms.  At
 * stage 0 the interface velocity S_M n is kept for the level set. */
/* Velocity jump across the wave of a stiffened-gas state W (rho, u_n, u_t, p)
 * of material m that brings its pressure to ps (Toro's pressure function,
 * pressures shifted by p_inf): a shock for ps > p, a rarefaction otherwise. */
static real wave_jump(const St *s, int m, const real *W, real ps) {
  double g = s->c.gamma[m], pinf = s->pinfe[m];
  real pb = W[3] + pinf, psb = ps + pinf;
  if (ps > W[3]) {
    real A = 2.0 / ((g + 1.0) * W[0]);
    real B = (g - 1.0) / (g + 1.0) * pb;
    return (ps - W[3]) * sqrt(A / (psb + B));
  }
  real c = sqrt(g * pb / W[0]);
  return 2.0 * c / (g - 1.0) * (pow(psb / pb, (g - 1.0) / (2.0 * g)) - 1.0);
}

static void interface_exchange(St *s, int stage) {
  int nx = s->c.nx, ny = s->c.ny;
  memset(s->X, 0, (size_t)s->M * 4 * s->NC * sizeof(real));
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      if (stage == 0) {
        s->vx[k] = 0.0;
        s->vy[k] = 0.0;
        s->vok[k] = 0;
      }
      unsigned b = s->xs[k];
      if ((b & (b - 1)) == 0) continue;
      int a = -1, bb = -1;
      for (int r = 0; r < s->M; r++) {
        if (!(b >> r & 1)) continue;
        if (a < 0 || M4(s, s->Q, r, 0, k) > M4(s, s->Q, a, 0, k)) a = r;
      }
      for (int r = 0; r < s->M; r++) {
        if (!(b >> r & 1) || r == a) continue;
        if (bb < 0 || M4(s, s->Q, r, 0, k) > M4(s, s->Q, bb, 0, k)) bb = r;
      }
      real cxa = M1(s, s->cx, a, k), cya = M1(s, s->cy, a, k);
      if (cxa == 0.0 && cya == 0.0) continue;
      if (!M1(s, s->Wv, a, k) || !M1(s, s->Wv, bb, k)) {
        s->n_ifskip++;
        continue;
      }
      real nrm = sqrt(cxa * cxa + cya * cya);
      real nxv = cxa / nrm, nyv = cya / nrm;
      real WL[4], WR[4];
      WL[0] = M4(s, s->W, bb, 0, k);
      WL[1] = M4(s, s->W, bb, 1, k) * nxv + M4(s, s->W, bb, 2, k) * nyv;
      WL[2] = 0.0;
      WL[3] = M4(s, s->W, bb, 3, k);
      WR[0] = M4(s, s->W, a, 0, k);
      WR[1] = M4(s, s->W, a, 1, k) * nxv + M4(s, s->W, a, 2, k) * nyv;
      WR[2] = 0.0;
      WR[3] = M4(s, s->W, a, 3, k);
      real SM, ps;
      if (PASSIVE(s, a) || PASSIVE(s, bb)) {
        /* free surface (Sec. 3 Case II): the ambient is not solved; the
           surface pressure is prescribed, and the surface moves with the
           velocity the solved side's wave reaches at that pressure (the
           solved side is the right state when it is a, the left one
           otherwise, along n) */
        ps = fs_pressure(s, s->tstage);
        SM = PASSIVE(s, bb) ? WR[1] + wave_jump(s, a, WR, ps) : WL[1] - wave_jump(s, bb, WL, ps);
      } else {
        real SL, SR;
        wave_speeds(WL, s->c.gamma[bb], s->pinfe[bb], s->tait[bb], WR, s->c.gamma[a],
                    s->pinfe[a], s->tait[a], &SL, &SR);
        SM = contact_speed(WL, WR, SL, SR);
        real pL = WL[3], pR = WR[3], uL = WL[1], uR = WR[1];
        ps = 0.5 * ((pL + WL[0] * (SL - uL) * (SM - uL)) +
                    (pR + WR[0] * (SR - uR) * (SM - uR)));
      }
      M4(s, s->X, a, 0, k) = 0.0;
      M4(s, s->X, a, 1, k) = ps * cxa;
      M4(s, s->X, a, 2, k) = ps * cya;
      M4(s, s->X, a, 3, k) = ps * SM * nrm;
      for (int v = 0; v < 4; v++) M4(s, s->X, bb, v, k) = -M4(s, s->X, a, v, k);
      /* nothing is exchanged with an ambient that is not solved */
      if (PASSIVE(s, a))
        for (int v = 0; v < 4; v++) M4(s, s->X, a, v, k) = 0.0;
      if (PASSIVE(s, bb))
        for (int v = 0; v < 4; v++) M4(s, s->X, bb, v, k) = 0.0;
      if (stage == 0) {
        s->vx[k] = SM * nxv;
        s->vy[k] = SM * nyv;
        s->vok[k] = 1;
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Aperture-weighted face fluxes (Eq. discretized_equ)                       */
/* ------------------------------------------------------------------------ */
/* Flux of material r across a face with A^r > 0: component-wise WENO5 of the
 * primitive variables from the six cells around the face (the right state is
 * the same routine on the mirrored stencil), then HLLC.  Reading (guards): if
 * a reconstructed density or p + p_inf is not positive, or a stencil cell has
 * no state, the first-order states of the two face cells are used. */
/* ------------------------------------------------------------------------ */
/* Roe flux with characteristic-wise WENO5 (the variant of the face flux;    */
/* Sec. 3 uses a 5th-order WENO scheme; the Roe solver and the projection  */
/* onto characteristic fields are the classical ones)                      */
/* ------------------------------------------------------------------------ */
/* Conserved (rho, rho u_n, rho u_t, rho E) of a primitive state (rho, u_n,
 * u_t, p) of material m. */
static void cons_of(const St *s, int m, const real *W, real *U) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = energy(s, m, W[0], W[1], W[2], W[3]);
}

/* Roe average of two states of one stiffened gas (normal direction first):
 * velocity, enthalpy and sound speed, c^2 = (gamma-1)(H - |u|^2/2). */
static void roe_avg(const St *s, int m, const real *WL, const real *WR, real *u,
                    real *v, real *Hr, real *c) {
  real sL = sqrt(WL[0]), sR = sqrt(WR[0]);
  real iw = 1.0 / (sL + sR);
  real HL = (energy(s, m, WL[0], WL[1], WL[2], WL[3]) + WL[3]) / WL[0];
  real HR = (energy(s, m, WR[0], WR[1], WR[2], WR[3]) + WR[3]) / WR[0];
  *u = (sL * WL[1] + sR * WR[1]) * iw;
  *v = (sL * WL[2] + sR * WR[2]) * iw;
  *Hr = (sL * HL + sR * HR) * iw;
  *c = sqrt((s->c.gamma[m] - 1.0) * (*Hr - 0.5 * (*u * *u + *v * *v)));
}

/* Left (L[k][.]) and right (R[.][k]) eigenvectors of the Euler flux
 * Jacobian in the normal direction at (u, v, H, c): eigenvalues u - c, u,
 * u (shear), u + c. */
static void eigvecs(double g, real u, real v, real Hr, real c, real L[4][4], real R[4][4]) {
  real q2 = 0.5 * (u * u + v * v);
  real b1 = (g - 1.0) / (c * c), b2 = q2 * b1;
  R[0][0] = 1.0; R[1][0] = u - c; R[2][0] = v; R[3][0] = Hr - u * c;
  R[0][1] = 1.0; R[1][1] = u;     R[2][1] = v; R[3][1] = q2;
  R[0][2] = 0.0; R[1][2] = 0.0;   R[2][2] = 1.0; R[3][2] = v;
  R[0][3] = 1.0; R[1][3] = u + c; R[2][3] = v; R[3][3] = Hr + u * c;
  L[0][0] = 0.5 * (b2 + u / c); L[0][1] = -0.5 * (b1 * u + 1.0 / c);
  L[0][2] = -0.5 * (b1 * v); L[0][3] = 0.5 * b1;
  L[1][0] = 1.0 - b2; L[1][1] = b1 * u; L[1][2] = b1 * v; L[1][3] = -b1;
  L[2][0] = -v; L[2][1] = 0.0; L[2][2] = 1.0; L[2][3] = 0.0;
  L[3][0] = 0.5 * (b2 - u / c); L[3][1] = -0.5 * (b1 * u - 1.0 / c);
  L[3][2] = -0.5 * (b1 * v); L[3][3] = 0.5 * b1;
}

static void matvec(real A[4][4], const real *x, real *y) {
  for (int k = 0; k < 4; k++) y[k] = ((A[k][0] * x[0] + A[k][1] * x[1]) + A[k][2] * x[2]) + A[k][3] * x[3];
}

/* Physical flux of a conserved state in the normal direction. */
static void euler_flux(const St *s, int m, const real *U, real *F, real *p_out) {
  real rho = U[0], un = U[1] / rho, ut = U[2] / rho;
  real p = (s->c.gamma[m] - 1.0) * (U[3] - 0.5 * rho * (un * un + ut * ut)) - s->c.gamma[m] * s->pinfe[m];
  F[0] = U[1];
  F[1] = U[1] * un + p;
  F[2] = U[1] * ut;
  F[3] = un * (U[3] + p);
  *p_out = p;
}

/* Speed u_n -+ c of a conserved state (sign -1: the left acoustic field,
 * +1 the right one); 0 with ok = 0 if the state is not physical. */
static real acoustic_speed(const St *s, int m, const real *U, int sign, int *ok) {
  real rho = U[0];
  real un = U[1] / rho, ut = U[2] / rho;
  real p = (s->c.gamma[m] - 1.0) * (U[3] - 0.5 * rho * (un * un + ut * ut)) - s->c.gamma[m] * s->pinfe[m];
  *ok = rho > 0.0 && p + s->pinfe[m] > 0.0;
  if (!*ok) return 0.0;
  real c = sqrt(s->c.gamma[m] * (p + s->pinfe[m]) / rho);
  return sign < 0 ? un - c : un + c;
}

/* Roe's flux between the states WL, WR, with the Harten-Hyman entropy fix
 * on the two acoustic fields: with lambda_a, lambda_b the field's speeds in
 * the states on either side of that wave of the linearised solution (U_L
 * and U_L + a_1 r_1 for the left field, U_R - a_4 r_4 and U_R for the right
 * one) and delta = max(0, lambda~ - lambda_a, lambda_b - lambda~), |lambda~|
 * below delta is replaced by (lambda~^2 + delta^2)/(2 delta).  Only a
 * transonic rarefaction has delta > 0; shocks keep Roe's exact resolution. */
static void roe_flux(const St *s, int m, const real *WL, const real *WR, real *G) {
  real UL[4], UR[4], FL[4], FR[4], pL, pR;
  cons_of(s, m, WL, UL);
  cons_of(s, m, WR, UR);
  euler_flux(s, m, UL, FL, &pL);
  euler_flux(s, m, UR, FR, &pR);
  real u, v, Hr, c, L[4][4], R[4][4];
  roe_avg(s, m, WL, WR, &u, &v, &Hr, &c);
  eigvecs(s->c.gamma[m], u, v, Hr, c, L, R);
  real dU[4], a[4];
  for (int k = 0; k < 4; k++) dU[k] = UR[k] - UL[k];
  matvec(L, dU, a);
  real lam[4] = {u - c, u, u, u + c};
  /* states on either side of the two acoustic waves */
  real Ua[4], Ub[4];
  for (int q = 0; q < 4; q++) {
    Ua[q] = UL[q] + a[0] * R[q][0];
    Ub[q] = UR[q] - a[3] * R[q][3];
  }
  for (int k = 0; k < 4; k++) {
    real l = fabs(lam[k]);
    if (k == 0 || k == 3) {
      int oka, okb;
      real la = k == 0 ? acoustic_speed(s, m, UL, -1, &oka) : acoustic_speed(s, m, Ub, 1, &oka);
      real lb = k == 0 ? acoustic_speed(s, m, Ua, -1, &okb) : acoustic_speed(s, m, UR, 1, &okb);
      if (oka && okb) {
        real d1 = lam[k] - la, d2 = lb - lam[k];
        real delta = d1 > d2 ? d1 : d2;
        if (delta > 0.0 && l < delta) l = (lam[k] * lam[k] + delta * delta) / (2.0 * delta);
      }
    }
    a[k] = l * a[k];
  }
  for (int q = 0; q < 4; q++) {
    real d = ((R[q][0] * a[0] + R[q][1] * a[1]) + R[q][2] * a[2]) + R[q][3] * a[3];
    G[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * d;
  }
}

/* Characteristic-wise WENO5 at a face: the six cells' conserved states are
 * projected onto the characteristic fields of the Roe average of the two
 * face cells, reconstructed field by field (left-biased from cells 0..4,
 * right-biased from 5..1) and projected back; returns the primitive states
 * (rho, u_n, u_t, p) on both sides. */
static void char_weno(const St *s, int m, real Wc[6][4], const int *perm, real *WL, real *WR) {
  real Ws[6][4], U[6][4], w[6][4];
  for (int q = 0; q < 6; q++) {
    for (int v = 0; v < 4; v++) Ws[q][v] = Wc[q][perm[v]];
    cons_of(s, m, Ws[q], U[q]);
  }
  real u, v, Hr, c, L[4][4], R[4][4];
  roe_avg(s, m, Ws[2], Ws[3], &u, &v, &Hr, &c);
  eigvecs(s->c.gamma[m], u, v, Hr, c, L, R);
  for (int q = 0; q < 6; q++) matvec(L, U[q], w[q]);
  real cl[4], cr[4], UL[4], UR[4];
  for (int k = 0; k < 4; k++) {
    cl[k] = weno5(w[0][k], w[1][k], w[2][k], w[3][k], w[4][k]);
    cr[k] = weno5(w[5][k], w[4][k], w[3][k], w[2][k], w[1][k]);
  }
  matvec(R, cl, UL);
  matvec(R, cr, UR);
  real pL, pR, FL[4];
  euler_flux(s, m, UL, FL, &pL);
  euler_flux(s, m, UR, FL, &pR);
  WL[0] = UL[0]; WL[1] = UL[1] / UL[0]; WL[2] = UL[2] / UL[0]; WL[3] = pL;
  WR[0] = UR[0]; WR[1] = UR[1] / UR[0]; WR[2] = UR[2] / UR[0]; WR[3] = pR;
}

static int face_flux(St *s, int r, const int *kk /* 6 cells */, int normal,
                     real *F) {
  real WL[4], WR[4], Wc[6][4];
  int ok = 1;
  for (int q = 0; q < 6; q++) {
    if (!M1(s, s->Wv, r, kk[q])) ok = 0;
    for (int v = 0; v < 4; v++) Wc[q][v] = M4(s, s->W, r, v, kk[q]);
  }
  if (!M1(s, s->Wv, r, kk[2]) || !M1(s, s->Wv, r, kk[3])) {
    s->n_fluxskip++;
    for (int v = 0; v < 4; v++) F[v] = 0.0;
    return 0;
  }
  /* component order: rho, normal velocity, tangential velocity, p */
  int perm[4] = {0, normal == 0 ? 1 : 2, normal == 0 ? 2 : 1, 3};
  int roe = s->c.flux == 1;
  if (ok) {
    if (roe) {
      char_weno(s, r, Wc, perm, WL, WR);
    } else {
      for (int v = 0; v < 4; v++) {
        int c = perm[v];
        WL[v] = weno5(Wc[0][c], Wc[1][c], Wc[2][c], Wc[3][c], Wc[4][c]);
        WR[v] = weno5(Wc[5][c], Wc[4][c], Wc[3][c], Wc[2][c], Wc[1][c]);
      }
    }
    double pinf = s->pinfe[r];
    if (!(WL[0] > 0.0) || !(WR[0] > 0.0) || !(WL[3] + pinf > 0.0) ||
        !(WR[3] + pinf > 0.0))
      ok = 0;
  }
  if (!ok) {
    s->n_posfix++;
    for (int v = 0; v < 4; v++) {
      WL[v] = Wc[2][perm[v]];
      WR[v] = Wc[3][perm[v]];
    }
  }
  real G[4];
  if (roe)
    roe_flux(s, r, WL, WR, G);
  else
    hllc_flux(s, r, WL, WR, G);
  F[0] = G[0];
  F[1 + (normal == 0 ? 0 : 1)] = G[1];
  F[1 + (normal == 0 ? 1 : 0)] = G[2];
  F[3] = G[3];
  return 1;
}

static void fluxes(St *s) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int r = 0; r < s->M; r++) {
    if (PASSIVE(s, r)) {
      memset(&M4(s, s->Fx, r, 0, 0), 0, (size_t)4 * s->NC * sizeof(real));
      if (s->c.dim == 2) memset(&M4(s, s->Fy, r, 0, 0), 0, (size_t)4 * s->NC * sizeof(real));
      continue;
    }
    for (int j = 0; j < ny; j++)
      for (int i = -1; i < nx; i++) {
        int k = ID(s, i, j);
        real F[4] = {0.0, 0.0, 0.0, 0.0};
        if (M1(s, s->ax, r, k) > 0.0) {
          int kk[6];
          for (int q = 0; q < 6; q++) kk[q] = ID(s, i - 2 + q, j);
          face_flux(s, r, kk, 0, F);
        }
        for (int v = 0; v < 4; v++) M4(s, s->Fx, r, v, k) = F[v];
      }
    if (s->c.dim < 2) continue;
    for (int j = -1; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, j);
        real F[4] = {0.0, 0.0, 0.0, 0.0};
        if (M1(s, s->ay, r, k) > 0.0) {
          int kk[6];
          for (int q = 0; q < 6; q++) kk[q] = ID(s, i, j - 2 + q);
          face_flux(s, r, kk, 1, F);
        }
        for (int v = 0; v < 4; v++) M4(s, s->Fy, r, v, k) = F[v];
      }
  }
}

/* RK-stage coefficients of the beta-form used for the level set (Eq.
 * local-advection) and the fluid alike.  Reading: third-order SSP
 * Runge-Kutta (Shu-Osher), beta = (0, 3/4, 1/3); rk_order 2 gives the
 * paper's second-order TVD scheme, beta = (0, 1/2). */
static int rk_stages(const St *s, double *b, double *c, double *w) {
  if (s->c.rk_order == 2) {
    b[0] = 0.0; b[1] = 0.5;
    c[0] = 1.0; c[1] = 0.5;
    w[0] = 0.5; w[1] = 0.5;
    return 2;
  }
  b[0] = 0.0; b[1] = 0.75; b[2] = 1.0 / 3.0;
  c[0] = 1.0; c[1] = 0.25; c[2] = 2.0 / 3.0;
  w[0] = 1.0 / 6.0; w[1] = 1.0 / 6.0; w[2] = 2.0 / 3.0;
  return 3;
}

/* Stage update of Eq. discretized_equ in the beta-form:
 * Q* = b Q^n + c [Q^(s) + dt/dx (A F)_{i-1/2} - (A F)_{i+1/2}) + dt/dy (...)
 *                 + dt/(dx dy) X].
 * Reading: the y bracket is scaled by dt/dy (the printed dt/dx is a slip;
 * dx = dy in every workload here).  In 1D the exchange is scaled by dt/dx. */
static void rk_update(St *s, double b, double c, double w) {
  int nx = s->c.nx, ny = s->c.ny;
  /* unit of work: one material-cell with alpha > 0 updated in one stage */
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++)
        if (M1(s, s->al, r, ID(s, i, j)) > 0.0 && !PASSIVE(s, r)) s->n_upd++;
  real lx = s->dt / s->dx, ly = s->dt / s->dy;
  real lv = s->c.dim == 2 ? s->dt / (s->dx * s->dy) : s->dt / s->dx;
  int cyl = s->c.coord == 1;
  for (int r = 0; r < s->M; r++)
    for (int v = 0; v < 4; v++) {
      if (PASSIVE(s, r)) {  /* not solved: the stage leaves it as it is */
        for (int j = 0; j < ny; j++)
          for (int i = 0; i < nx; i++) M4(s, s->Qt, r, v, ID(s, i, j)) = M4(s, s->Q, r, v, ID(s, i, j));
        continue;
      }
      for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
          int k = ID(s, i, j), kl = ID(s, i - 1, j);
          real Al = M1(s, s->ax, r, kl), Ar = M1(s, s->ax, r, k);
          real fl = Al > 0.0 ? Al * M4(s, s->Fx, r, v, kl) : 0.0;
          real fr = Ar > 0.0 ? Ar * M4(s, s->Fx, r, v, k) : 0.0;
          real rhs = lx * (fl - fr);
          if (cyl) {
            /* cylindrical: face areas r_{i-1/2}, r_{i+1/2} per cell volume
               r_i dx, and the geometric source p alpha / r_i of the radial
               momentum (the pressure of the material's state in the cell) */
            double rl = s->c.x0 + i * s->dx, rr = s->c.x0 + (i + 1) * s->dx;
            double ri = s->c.x0 + (i + 0.5) * s->dx;
            rhs = lx * (fl * rl - fr * rr) / ri;
            if (v == 1 && M1(s, s->Wv, r, k))
              rhs = rhs + s->dt * (M1(s, s->al, r, k) * M4(s, s->W, r, 3, k) / ri);
          }
          if (s->c.dim == 2) {
            int kb = ID(s, i, j - 1);
            real Ab = M1(s, s->ay, r, kb), At = M1(s, s->ay, r, k);
            real fb = Ab > 0.0 ? Ab * M4(s, s->Fy, r, v, kb) : 0.0;
            real ft = At > 0.0 ? At * M4(s, s->Fy, r, v, k) : 0.0;
            rhs = rhs + ly * (fb - ft);
          }
          rhs = rhs + lv * M4(s, s->X, r, v, k);
          M4(s, s->Qt, r, v, k) = b * M4(s, s->Qn, r, v, k) + c * (M4(s, s->Q, r, v, k) + rhs);
        }
      /* conservation book-keeping: net inflow through the domain boundary and
         exchange totals, weighted by the stage's share of the full step */
      real in = 0.0;
      for (int j = 0; j < ny; j++) {
        int kl = ID(s, -1, j), kr = ID(s, nx - 1, j);
        real Al = M1(s, s->ax, r, kl), Ar = M1(s, s->ax, r, kr);
        /* cylindrical: r-weighted (the sums are of r_i Q_i) */
        double rlo = cyl ? s->c.x0 : 1.0, rhi = cyl ? s->c.x0 + nx * s->dx : 1.0;
        in += lx * ((Al > 0.0 ? Al * M4(s, s->Fx, r, v, kl) : 0.0) * rlo -
                    (Ar > 0.0 ? Ar * M4(s, s->Fx, r, v, kr) : 0.0) * rhi);
      }
      if (s->c.dim == 2)
        for (int i = 0; i < nx; i++) {
          int kb = ID(s, i, -1), kt = ID(s, i, ny - 1);
          real Ab = M1(s, s->ay, r, kb), At = M1(s, s->ay, r, kt);
          in += ly * ((Ab > 0.0 ? Ab * M4(s, s->Fy, r, v, kb) : 0.0) -
                      (At > 0.0 ? At * M4(s, s->Fy, r, v, kt) : 0.0));
        }
      real xsum = 0.0;
      for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
          int k = ID(s, i, j);
          if (!cyl) {
            xsum += lv * M4(s, s->X, r, v, k);
            continue;
          }
          /* cylindrical: r-weighted exchange plus the geometric source */
          double ri = s->c.x0 + (i + 0.5) * s->dx;
          xsum += lv * M4(s, s->X, r, v, k) * ri;
          if (v == 1 && M1(s, s->Wv, r, k))
            xsum += s->dt * (M1(s, s->al, r, k) * M4(s, s->W, r, 3, k));
        }
      neumaier(&s->bnd[r][v], &s->bnd_c[r][v], w * in);
      neumaier(&s->xsum[r][v], &s->xsum_c[r][v], w * xsum);
    }
}

/* Advection velocity v^n of the level set (Eq. local-advection uses the
 * time-n velocity in every sub-step).  Reading: interface cells carry the
 * interface velocity S_M n of their Riemann problem; it is carried off the
 * interface by 4 Jacobi sweeps over band cells (phi^n below the band width),
 * each taking the upwind neighbours towards smaller phi weighted by the
 * gradient components of phi; every other cell takes the velocity of its own
 * material's state (0 if it has none). */
static void ls_velocity(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2;
  int n = 0;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      if (!s->vok[k] && s->phi[k] < s->bls) s->list[n++] = k;
    }
  for (int it = 0; it < 4; it++) {
    for (int q = 0; q < n; q++) {
      int k = s->list[q];
      int i = k % s->NX - OR_H, j = k / s->NX - s->HY;
      s->lok[q] = 0;
      if (s->vok[k]) continue;
      real gx = s->phi[ID(s, i + 1, j)] - s->phi[ID(s, i - 1, j)];
      real gy = two ? s->phi[ID(s, i, j + 1)] - s->phi[ID(s, i, j - 1)] : 0.0;
      int kx = -1, ky = -1;
      if (gx != 0.0) {
        int ii = i - (gx > 0.0 ? 1 : -1);
        if (ii >= 0 && ii < nx && s->vok[ID(s, ii, j)]) kx = ID(s, ii, j);
      }
      if (gy != 0.0) {
        int jj = j - (gy > 0.0 ? 1 : -1);
        if (jj >= 0 && jj < ny && s->vok[ID(s, i, jj)]) ky = ID(s, i, jj);
      }
      real *o = &s->lv[(size_t)q * 2];
      if (kx >= 0 && ky >= 0) {
        real wx = fabs(gx), wy = fabs(gy);
        o[0] = (wx * s->vx[kx] + wy * s->vx[ky]) / (wx + wy);
        o[1] = (wx * s->vy[kx] + wy * s->vy[ky]) / (wx + wy);
        s->lok[q] = 1;
      } else if (kx >= 0) {
        o[0] = s->vx[kx];
        o[1] = s->vy[kx];
        s->lok[q] = 1;
      } else if (ky >= 0) {
        o[0] = s->vx[ky];
        o[1] = s->vy[ky];
        s->lok[q] = 1;
      }
    }
    for (int q = 0; q < n; q++)
      if (s->lok[q]) {
        int k = s->list[q];
        s->vx[k] = s->lv[(size_t)q * 2];
        s->vy[k] = s->lv[(size_t)q * 2 + 1];
        s->vok[k] = 1;
      }
  }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j), r = s->chi[k];
      if (s->vok[k]) continue;
      if (M1(s, s->Wv, r, k)) {
        s->vx[k] = M4(s, s->W, r, 1, k);
        s->vy[k] = M4(s, s->W, r, 2, k);
      }
    }
}

/* Level-set update region.  Reading: the narrow band is the set of cells
 * with phi below the band width or a mixed local set; a cell is updated when
 * such a cell lies within Chebyshev distance 3 (the reach of the HJ-WENO5
 * stencil), so the band follows a moving interface; all other cells keep
 * phi at the band width. */
static void ls_region(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2;
  unsigned char *f = s->band, *rb = s->band2;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      unsigned b = s->xs[k];
      f[k] = (unsigned char)(s->phi[k] < s->bls || (b & (b - 1)) != 0);
    }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      unsigned char h = 0;
      for (int di = -3; di <= 3; di++)
        if (i + di >= 0 && i + di < nx) h |= f[ID(s, i + di, j)];
      rb[ID(s, i, j)] = h;
    }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      unsigned char h = 0;
      for (int dj = -3 * two; dj <= 3 * two; dj++)
        if (j + dj >= 0 && j + dj < ny) h |= rb[ID(s, i, j + dj)];
      s->reg[ID(s, i, j)] = h;
    }
}

/* ------------------------------------------------------------------------ */
/* Level-set stage (Sec. 2.2, Eq. local-advection and Eq. reconstruction)   */
/* ------------------------------------------------------------------------ */
/* For every cell of the update region and every r in its local set X_s: construct phi^r on the stencil, take the HJ-WENO5 upwind
 * derivative (the WENO5 routine applied to the five one-sided divided
 * differences on the upwind side of v^n), advance with the beta-form, then
 * reconstruct phi = |max_r phi^r|, chi = argmax_r phi^r (ties: smaller
 * index).  Reading: phi is clamped to the band width; cells outside the
 * region keep their values; no reinitialisation is applied. */
static real hj_deriv(St *s, int r, int i, int j, int dir, real vel) {
  real d[7]; /* divided differences d(q) = (phi_q - phi_{q-1})/h, q = i-2 .. i+3 */
  double ih = dir == 0 ? s->idx : s->idy;
  for (int q = 0; q < 6; q++) {
    int o = q - 2;
    int k1 = dir == 0 ? ID(s, i + o, j) : ID(s, i, j + o);
    int k0 = dir == 0 ? ID(s, i + o - 1, j) : ID(s, i, j + o - 1);
    d[q] = (lsv(s->phi, s->chi, r, k1) - lsv(s->phi, s->chi, r, k0)) * ih;
  }
  if (vel > 0.0) return weno5(d[0], d[1], d[2], d[3], d[4]);
  if (vel < 0.0) return weno5(d[5], d[4], d[3], d[2], d[1]);
  return 0.0;
}

static void levelset_stage(St *s, double b, double c) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      if (!s->reg[k]) {
        s->phit[k] = s->phi[k];
        s->chit[k] = s->chi[k];
        continue;
      }
      real best = 0.0;
      int br = -1;
      for (int r = 0; r < s->M; r++) {
        if (!(s->xs[k] >> r & 1)) continue;
        real gx = hj_deriv(s, r, i, j, 0, s->vx[k]);
        real adv = s->vx[k] * gx;
        if (s->c.dim == 2) {
          real gy = hj_deriv(s, r, i, j, 1, s->vy[k]);
          adv = adv + s->vy[k] * gy;
        }
        real val = lsv(s->phi, s->chi, r, k) - s->dt * adv;
        real nv = b * lsv(s->phin, s->chin, r, k) + c * val;
        if (br < 0 || nv > best) {
          best = nv;
          br = r;
        }
      }
      real a = fabs(best);
      s->phit[k] = a < s->bls ? a : s->bls;
      s->chit[k] = br;
    }
}

/* ------------------------------------------------------------------------ */
/* Mixing of small, new and vanishing cut cells (Sec. 2.3.2, after each RK  */
/* sub-step)                                                                */
/* ------------------------------------------------------------------------ */
/* Reading (the weights of hu2006conservative are not reproduced in the
 * paper): for each material r, a source cell has 0 < alpha < alpha_mix, or
 * alpha > 0 with its centre outside r (chi != r: it has no real state of
 * its own), or alpha = 0 with a non-zero state.  Its targets are the
 * neighbours in x, in y and diagonally along the side of increasing phi^r
 * (central differences g); a target needs alpha_t >= alpha_mix and chi = r.  Weights g_x^2 alpha_x,
 * g_y^2 alpha_y and |g_x g_y| alpha_xy, normalised.  Exchange from target t:
 * M_t = beta_t (alpha_s Q_t - alpha_t Q_s)/(alpha_s + alpha_t), added to the
 * source and taken from the target, all from pre-mixing values (a target
 * sums what it receives in mirror-symmetric pairs of neighbours).  For a
 * vanishing source (alpha_s = 0) this is M_t = -beta_t Q_s; the last target
 * in the order x, y, diagonal takes the exact remainder, so the source is
 * left at exactly zero.  Without an
 * eligible target the 8-neighbour (2-neighbour in 1D) of largest alpha >=
 * alpha_mix and chi = r takes the whole exchange (ties: lower linear index); without one
 * the cell is left as it is and counted. */
/* The conserved quantities of material r in cell k join those of material
 * to, book-kept in xfer with the weight xw that a change of the current
 * stage's state carries into the end of the step (the product of the later
 * stages' coefficients of the previous stage in the beta form: 1/6, 2/3, 1
 * for the three stages of RK3; 1 after the step). */
static void move_q(St *s, int k, int r, int to) {
  /* cylindrical: the book-keeping is of r_i Q_i, like the balances */
  double ri = 1.0;
  if (s->c.coord == 1) ri = s->c.x0 + ((k % s->NX) - OR_H + 0.5) * s->dx;
  for (int v = 0; v < 4; v++) {
    real q = M4(s, s->Q, r, v, k);
    M4(s, s->Q, to, v, k) = M4(s, s->Q, to, v, k) + q;
    M4(s, s->Q, r, v, k) = 0.0;
    neumaier(&s->xfer[to][v], &s->xfer_c[to][v], s->xw * q * ri);
    neumaier(&s->xfer[r][v], &s->xfer_c[r][v], -(s->xw * q * ri));
  }
}

static void mixing(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2;
  double amix = s->c.alpha_mix;
  size_t nc = s->NC;
  s->nab = s->nrl = 0;
  int cyl = s->c.coord == 1;
  for (int r = 0; r < s->M; r++) {
    if (PASSIVE(s, r)) continue;  /* not solved */
    int *T = s->mixT;
    real *Mx = s->mixM;
    for (size_t q = 0; q < 3 * nc; q++) T[q] = -1;
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, j);
        real as = M1(s, s->al, r, k);
        /* Reading (empty part): a cell's own material with a volume
           fraction but no conserved quantities at all (left so by a move
           between materials, stranded sources or scale separation) is
           filled from its neighbours like a new cell, whatever its alpha;
           so is a part with 0 < alpha < 1 and no mass (a partial density of
           zero or roundoff of either sign: an interface that crossed a face
           that had no aperture yet for this material) */
        int empty = 1;
        for (int v = 0; v < 4; v++)
          if (M4(s, s->Qt, r, v, k) != 0.0) empty = 0;
        if (!(M4(s, s->Qt, r, 0, k) > 0.0) && as < 1.0) empty = 1;
        if (!(as < amix) && s->chit[k] == r && !(empty && as > 0.0)) continue;
        if (!(as > 0.0)) {
          int nz = 0;
          for (int v = 0; v < 4; v++)
            if (M4(s, s->Qt, r, v, k) != 0.0) nz = 1;
          if (!nz) continue;
        }
        s->n_mixsrc++;
        real gx = lsv(s->phit, s->chit, r, ID(s, i + 1, j)) - lsv(s->phit, s->chit, r, ID(s, i - 1, j));
        real gy = two ? lsv(s->phit, s->chit, r, ID(s, i, j + 1)) - lsv(s->phit, s->chit, r, ID(s, i, j - 1)) : 0.0;
        int sx = gx > 0.0 ? 1 : (gx < 0.0 ? -1 : 0);
        int sy = gy > 0.0 ? 1 : (gy < 0.0 ? -1 : 0);
        int tk[3] = {-1, -1, -1};
        real w[3] = {0.0, 0.0, 0.0};
        if (sx != 0 && i + sx >= 0 && i + sx < nx) {
          int t = ID(s, i + sx, j);
          real at = M1(s, s->al, r, t);
          if (at >= amix && s->chit[t] == r) { tk[0] = t; w[0] = gx * gx * at; }
        }
        if (sy != 0 && j + sy >= 0 && j + sy < ny) {
          int t = ID(s, i, j + sy);
          real at = M1(s, s->al, r, t);
          if (at >= amix && s->chit[t] == r) { tk[1] = t; w[1] = gy * gy * at; }
        }
        if (sx != 0 && sy != 0 && i + sx >= 0 && i + sx < nx && j + sy >= 0 && j + sy < ny) {
          int t = ID(s, i + sx, j + sy);
          real at = M1(s, s->al, r, t);
          if (at >= amix && s->chit[t] == r) { tk[2] = t; w[2] = fabs(gx * gy) * at; }
        }
        real wsum = (w[0] + w[1]) + w[2];
        real beta[3] = {0.0, 0.0, 0.0};
        if (wsum > 0.0) {
          for (int q = 0; q < 3; q++)
            if (w[q] > 0.0) beta[q] = w[q] / wsum;
            else tk[q] = -1;
        } else {
          tk[0] = tk[1] = tk[2] = -1;
          real bestA = -1.0;
          int bt = -1;
          for (int dj = -two; dj <= two; dj++)
            for (int di = -1; di <= 1; di++) {
              if (di == 0 && dj == 0) continue;
              int ii = i + di, jj = j + dj;
              if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
              int t = ID(s, ii, jj);
              real at = M1(s, s->al, r, t);
              if (at >= amix && s->chit[t] == r && at > bestA) { bestA = at; bt = t; }
            }
          if (bt < 0) {
            /* Reading (stranded source): no neighbour of material r can
               take the exchange.  If r is the cell's own material (a
               fragment of r too small to be resolved, with no resolved part
               of r next to it), the cell is given to the other material of
               largest volume fraction in it (ties: lower index), the
               indicator swap of the scale-separation model (Sec. 2.3.3).
               After the exchanges, the conserved quantities of every
               stranded source join those of the cell's material as it is
               after these swaps (a source of that material itself stays).
               Total mass, momentum and energy stay conserved; the masses
               of the single materials do not. */
            if (s->chit[k] == r) {
              real ba = 0.0;
              int to = -1;
              for (int m = 0; m < s->M; m++)
                if (m != r && M1(s, s->al, m, k) > ba) {
                  ba = M1(s, s->al, m, k);
                  to = m;
                }
              if (to >= 0) {
                s->rlk[s->nrl] = k;
                s->rlto[s->nrl] = to;
                s->nrl++;
              }
            }
            s->abk[s->nab] = k;
            s->abr[s->nab] = r;
            s->nab++;
            continue;
          }
          tk[0] = bt;
          beta[0] = 1.0;
        }
        int last = -1;
        for (int q = 0; q < 3; q++) {
          T[(size_t)q * nc + k] = tk[q];
          if (tk[q] >= 0) last = q;
        }
        /* cylindrical: volumes and contents carry the cells' radii (the
           exchange is of content, alpha r and Q r in place of alpha and Q) */
        double rs = cyl ? s->c.x0 + (i + 0.5) * s->dx : 1.0;
        if (as > 0.0) {
          for (int q = 0; q < 3; q++) {
            if (tk[q] < 0) continue;
            real at = M1(s, s->al, r, tk[q]);
            double rt = cyl ? s->c.x0 + (i + (tk[q] - k) + 0.5) * s->dx : 1.0;
            for (int v = 0; v < 4; v++) {
              real Qs = M4(s, s->Qt, r, v, k), Qtg = M4(s, s->Qt, r, v, tk[q]);
              if (cyl) {
                real aS = as * rs, aT = at * rt, qS = Qs * rs, qT = Qtg * rt;
                Mx[((size_t)q * 4 + v) * nc + k] = beta[q] * ((aS * qT - aT * qS) / (aS + aT));
              } else {
                Mx[((size_t)q * 4 + v) * nc + k] = beta[q] * ((as * Qtg - at * Qs) / (as + at));
              }
            }
          }
        } else {
          /* vanishing cell: with alpha_s = 0 the exchange is M_t = -beta_t Q_s;
             the last target takes the exact remainder so the source ends at 0 */
          for (int v = 0; v < 4; v++) {
            real Qs = M4(s, s->Qt, r, v, k);
            if (cyl) Qs = Qs * rs;
            real acc = Qs;
            for (int q = 0; q < 3; q++) {
              if (tk[q] < 0) continue;
              real m = q == last ? -acc : -(beta[q] * Qs);
              Mx[((size_t)q * 4 + v) * nc + k] = m;
              acc = acc + m;
            }
          }
        }
      }
    /* apply as a gather: sources add their exchanges in target order, targets
       subtract what their 8 neighbours sent them, in row-major order */
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, j);
        for (int v = 0; v < 4; v++) {
          real q0 = M4(s, s->Qt, r, v, k);
          double rc = cyl ? s->c.x0 + (i + 0.5) * s->dx : 1.0;
          int src = 0;
          for (int q = 0; q < 3; q++)
            if (T[(size_t)q * nc + k] >= 0) {
              q0 = cyl ? q0 + Mx[((size_t)q * 4 + v) * nc + k] / rc
                       : q0 + Mx[((size_t)q * 4 + v) * nc + k];
              src = 1;
            }
          if (!src) {
            /* received exchanges, summed in mirror-symmetric pairs */
            real row[3];
            for (int dj = -1; dj <= 1; dj++) {
              real a[3] = {0.0, 0.0, 0.0};
              for (int di = -1; di <= 1; di++) {
                int ii = i + di, jj = j + dj;
                if ((di == 0 && dj == 0) || (!two && dj != 0) || ii < 0 || ii >= nx ||
                    jj < 0 || jj >= ny) continue;
                int n = ID(s, ii, jj);
                for (int q = 0; q < 3; q++)
                  if (T[(size_t)q * nc + n] == k) a[di + 1] = Mx[((size_t)q * 4 + v) * nc + n];
              }
              row[dj + 1] = (a[0] + a[2]) + a[1];
            }
            q0 = cyl ? q0 - ((row[0] + row[2]) + row[1]) / rc : q0 - ((row[0] + row[2]) + row[1]);
          }
          M4(s, s->Q, r, v, k) = q0;
        }
      }
  }
  /* stranded sources join the material of their cell after the swaps, in
     the order found (material, then row-major cell) */
  for (long a = 0; a < s->nab; a++) {
    int k = s->abk[a], r = s->abr[a], to = s->chit[k];
    for (long b = 0; b < s->nrl; b++)
      if (s->rlk[b] == k) to = s->rlto[b];
    if (to == r) {
      s->n_stranded++;
      continue;
    }
    move_q(s, k, r, to);
    s->n_absorb++;
  }
  s->n_relabel += s->nrl;
}

/* ------------------------------------------------------------------------ */
/* Interface scale separation (Sec. 2.3.3)                                  */
/* ------------------------------------------------------------------------ */
/* Does cell k hold part of the contour phi^r = off?  Reading: the contour
 * crosses the cell when the local level set of r at its centre and its four
 * corners (each the mean of the four cells around it) is <= off somewhere
 * and > off somewhere else. */
static int crosses(const St *s, const real *phi, const int *chi, int r, int k, double off) {
  int NX = s->NX, two = s->c.dim == 2;
  real c = lsv(phi, chi, r, k) - off;
  real mn = c, mx = c;
  for (int cj = 0; cj < 1 + two; cj++)
    for (int ci = 0; ci < 2; ci++) {
      int k0 = k + (ci ? 0 : -1) + (two ? (cj ? 0 : -NX) : 0);
      real v;
      if (two)
        v = (lsv(phi, chi, r, k0) + lsv(phi, chi, r, k0 + 1) + lsv(phi, chi, r, k0 + NX) +
             lsv(phi, chi, r, k0 + NX + 1)) * 0.25 - off;
      else
        v = (lsv(phi, chi, r, k0) + lsv(phi, chi, r, k0 + 1)) * 0.5 - off;
      if (v < mn) mn = v;
      if (v > mx) mx = v;
    }
  return mn <= 0.0 && mx > 0.0;
}

/* After a time step: with eps = 0.75 h, S_-^r (S_+^r) are the cells crossed
 * by the contour phi^r = eps (= -eps), the boundary of material r shrunk
 * (grown) by eps.  An oddball cell is a cut cell whose own material chi_1
 * has no cell of S_-^chi_1 in its 3 x 3 block: the material is thinner than
 * 2 eps there.  It is given to the other material chi_1* of largest volume
 * fraction, and its distance becomes |d_min - eps|, d_min the distance from
 * its centre to the eps-grown boundary of chi_1*, found from the cells of
 * S_+^chi_1* within 3 cells (the point of the contour along the normal at
 * their centres); without such a cell the distance is kept.
 * Readings: (1) the new topology must be resolved: chi_1* itself needs a
 * cell of S_-^chi_1* in the 3 x 3 block, else the cell is left as it is (in
 * mixing layers where both materials are thinner than 2 eps the criterion
 * otherwise flags the cells of both in turn and swaps them back and forth,
 * step after step); (2) the conserved quantities of chi_1 in the cell join
 * those of chi_1* (the paper does not say how they move; totals are
 * conserved); (3) the distance is capped at the band width.
 * Every decision reads the fields before any swap.  The geometry and the
 * volume-fraction correction are then evaluated again. */
static void scale_separation(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2, M = s->M;
  double eps = 0.75 * s->h;
  size_t nc = s->NC;
  unsigned char *sm = s->xs, *sp = s->band2;
  int *newchi = s->co;
  real *newphi = s->cv;
  memcpy(newchi, s->chi, nc * sizeof(int));
  memcpy(newphi, s->phi, nc * sizeof(real));
  memset(sm, 0, nc);
  memset(sp, 0, nc);
  for (int j = -two; j < ny + two; j++)
    for (int i = -1; i <= nx; i++) {
      int k = ID(s, i, j);
      for (int r = 0; r < M; r++) {
        if (crosses(s, s->phi, s->chi, r, k, eps)) sm[k] |= (unsigned char)(1u << r);
        if (crosses(s, s->phi, s->chi, r, k, -eps)) sp[k] |= (unsigned char)(1u << r);
      }
    }
  int any = 0;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j), c1 = s->chi[k];
      if (!(M1(s, s->al, c1, k) < 1.0)) continue;
      unsigned near = 0;
      for (int dj = -two; dj <= two; dj++)
        for (int di = -1; di <= 1; di++) near |= sm[ID(s, i + di, j + dj)];
      if (near >> c1 & 1) continue;
      int c2 = -1;
      real ba = 0.0;
      for (int r = 0; r < M; r++)
        if (r != c1 && M1(s, s->al, r, k) > ba) {
          ba = M1(s, s->al, r, k);
          c2 = r;
        }
      if (c2 < 0 || !(near >> c2 & 1)) continue;
      s->n_oddball++;
      any = 1;
      real dmin = -1.0;
      for (int dj = -3 * two; dj <= 3 * two; dj++)
        for (int di = -3; di <= 3; di++) {
          int ii = i + di, jj = j + dj;
          if (ii < -1 || ii > nx || (two && (jj < -1 || jj > ny))) continue;
          int k0 = ID(s, ii, jj);
          if (!(sp[k0] >> c2 & 1)) continue;
          real gx = lsv(s->phi, s->chi, c2, k0 + 1) - lsv(s->phi, s->chi, c2, k0 - 1);
          real gy = two ? lsv(s->phi, s->chi, c2, k0 + s->NX) - lsv(s->phi, s->chi, c2, k0 - s->NX)
                        : 0.0;
          real gn = sqrt(gx * gx + gy * gy);
          if (!(gn > 0.0)) continue;
          real f = lsv(s->phi, s->chi, c2, k0) + eps;
          real ex = di * s->dx - f * (gx / gn), ey = dj * s->dy - f * (gy / gn);
          real d = sqrt(ex * ex + ey * ey);
          if (dmin < 0.0 || d < dmin) dmin = d;
        }
      newchi[k] = c2;
      if (dmin >= 0.0) {
        real a = fabs(dmin - eps);
        newphi[k] = a < s->bls ? a : (real)s->bls;
      }
      move_q(s, k, c1, c2);
    }
  if (!any) return;
  memcpy(s->chi, newchi, nc * sizeof(int));
  memcpy(s->phi, newphi, nc * sizeof(real));
  fill_ls(s, s->phi, s->chi);
  geometry(s, s->phi, s->chi);
  for (int r = 0; r < M; r++)
    for (size_t k = 0; k < nc; k++) M1(s, s->mass, r, k) = M4(s, s->Q, r, 0, k);
  vf_correction(s, s->chi, s->mass);
}

/* Redistancing of the regional level set after every time step.  Reading:
 * the paper describes no reinitialisation (its reference for the
 * multi-region level set is not at hand); without one the distance field
 * degenerates in stretched layers (values near 0 over whole regions, every
 * cell cut), which stops the triple point's run.  Band cells (phi below the
 * band width) take new distances, the others keep the band width; the
 * material indicator does not change.
 * (1) A band cell with an interior 4-neighbour of another material: per
 * axis, the distance to the crossing of the local level set between the
 * two centres, h phi_c / (phi_c + phi_n) (h/2 where both are 0), the
 * smaller of the two sides; with crossings on both axes the distance to the
 * straight line through them, d_x d_y / sqrt(d_x^2 + d_y^2) (0 when one is
 * 0), else the one crossing; capped at the band width.  Other cells: the
 * band width.
 * (2) band_ls + 1 Jacobi sweeps over the band cells: the smallest of the
 * cell's value and, over its interior 8 neighbours of the same material,
 * the neighbour's value plus the distance of the centres; capped at the
 * band width.
 * Then the frame, the geometry and the correction (masses of the state). */
static void reinit(St *s) {
  int nx = s->c.nx, ny = s->c.ny, two = s->c.dim == 2;
  double bls = s->bls;
  real *a = s->cv, *b = s->phit;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      real pc = s->phi[k], best = bls;
      if (pc < bls) {
        real dxm = -1.0, dym = -1.0;
        for (int q = 0; q < 4; q++) {
          int di = q == 0 ? -1 : (q == 1 ? 1 : 0), dj = q == 2 ? -1 : (q == 3 ? 1 : 0);
          if (!two && dj != 0) continue;
          int ii = i + di, jj = j + dj;
          if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
          int kn = ID(s, ii, jj);
          if (s->chi[kn] == s->chi[k]) continue;
          real pn = s->phi[kn], sum = pc + pn;
          double hh = q < 2 ? s->dx : s->dy;
          real d = sum > 0.0 ? hh * (pc / sum) : 0.5 * hh;
          if (q < 2) {
            if (dxm < 0.0 || d < dxm) dxm = d;
          } else if (dym < 0.0 || d < dym) {
            dym = d;
          }
        }
        if (dxm >= 0.0 && dym >= 0.0)
          best = dxm > 0.0 && dym > 0.0 ? (dxm * dym) / sqrt(dxm * dxm + dym * dym) : 0.0;
        else if (dxm >= 0.0)
          best = dxm;
        else if (dym >= 0.0)
          best = dym;
        if (best > bls) best = bls;
      }
      a[k] = best;
    }
  for (int sw = 0; sw <= s->c.band_ls; sw++) {
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        int k = ID(s, i, j);
        real v = a[k];
        if (s->phi[k] < bls)
          for (int dj = -two; dj <= two; dj++)
            for (int di = -1; di <= 1; di++) {
              if (di == 0 && dj == 0) continue;
              int ii = i + di, jj = j + dj;
              if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
              int kn = ID(s, ii, jj);
              if (s->chi[kn] != s->chi[k]) continue;
              double ex = di * s->dx, ey = dj * s->dy;
              real cand = a[kn] + sqrt(ex * ex + ey * ey);
              if (cand < v) v = cand;
            }
        b[k] = v < bls ? v : bls;
      }
    real *t = a;
    a = b;
    b = t;
  }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int k = ID(s, i, j);
      if (s->phi[k] < bls) s->phi[k] = a[k];
    }
  fill_ls(s, s->phi, s->chi);
  geometry(s, s->phi, s->chi);
  for (int r = 0; r < s->M; r++)
    for (size_t k = 0; k < (size_t)s->NC; k++) M1(s, s->mass, r, k) = M4(s, s->Q, r, 0, k);
  vf_correction(s, s->chi, s->mass);
}

/* ------------------------------------------------------------------------ */
/* Public C API used by the tests through ctypes                            */
/* ------------------------------------------------------------------------ */
#ifdef __cplusplus
extern "C" {
#endif
static void *zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void or_destroy(St *s) {
  if (!s) return;
  void *p[] = {s->phi, s->phin, s->phit, s->chi, s->chin, s->chit, s->Q,
               s->Qn, s->Qt, s->al, s->ax, s->ay, s->cx, s->cy, s->W, s->lw,
               s->Wv, s->lok, s->band, s->band2, s->list, s->vok, s->reg, s->lv, s->X, s->vx, s->vy, s->Fx, s->Fy,
               s->mass, s->cv, s->co, s->xs, s->mixM, s->mixT, s->abk, s->abr,
               s->rlk, s->rlto};
  for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); i++) free(p[i]);
  free(s);
}

St *or_create(const or_config *c) {
  if (!c || (c->dim != 1 && c->dim != 2) || c->nx < 1 || c->ny < 1 ||
      (c->dim == 1 && c->ny != 1) || c->n_mat < 1 || c->n_mat > OR_MAXM)
    return NULL;
  if ((c->coord != 0 && c->coord != 1) || (c->coord == 1 && (c->dim != 1 || c->x0 < 0.0)))
    return NULL;
  if (c->fs_on != 0 && c->fs_on != 1) return NULL;
  if (c->reinit != 0 && c->reinit != 1) return NULL;
  if (c->fs_on) {
    if (c->fs_mat < 0 || c->fs_mat >= c->n_mat || !(c->fs_p[4] > 0.0) ||
        !(c->fs_p[3] > c->fs_p[2]) || c->flux != 0)
      return NULL;
    for (int m = 0; m < c->n_mat; m++)
      if (c->eos[m] != 0) return NULL;
  }
  for (int m = 0; m < c->n_mat; m++)
    if (c->eos[m] < 0 || c->eos[m] > 1 ||
        (c->eos[m] == 1 && !(c->rho0[m] > 0.0 && c->tait_B[m] > 0.0)))
      return NULL;
  if (c->flux < 0 || c->flux > 1) return NULL;
  for (int m = 0; m < c->n_mat; m++)
    if (c->flux == 1 && c->eos[m] == 1) return NULL; /* Roe variant: stiffened gases */
  St *s = (St *)zalloc(sizeof(St));
  s->c = *c;
  s->M = c->n_mat;
  s->NX = c->nx + 2 * OR_H;
  s->HY = c->dim == 2 ? OR_H : 0;
  s->NY = c->ny + 2 * s->HY;
  s->NC = s->NX * s->NY;
  s->dx = (c->x1 - c->x0) / c->nx;
  s->dy = c->dim == 2 ? (c->y1 - c->y0) / c->ny : 1.0;
  s->h = c->dim == 2 ? (s->dx < s->dy ? s->dx : s->dy) : s->dx;
  s->bls = c->band_ls * s->h;
  s->idx = 1.0 / s->dx;
  s->idy = 1.0 / s->dy;
  for (int m = 0; m < s->M; m++) {
    s->igm1[m] = 1.0 / (c->gamma[m] - 1.0);
    s->tait[m] = c->eos[m] == 1;
    s->pinfe[m] = s->tait[m] ? c->tait_B[m] - c->p0[m] : c->pinf[m];
  }
  size_t nc = s->NC, M = s->M, R = sizeof(real);
  s->phi = (real *)zalloc(nc * R); s->phin = (real *)zalloc(nc * R);
  s->phit = (real *)zalloc(nc * R);
  s->chi = (int *)zalloc(nc * 4); s->chin = (int *)zalloc(nc * 4); s->chit = (int *)zalloc(nc * 4);
  s->Q = (real *)zalloc(M * 4 * nc * R); s->Qn = (real *)zalloc(M * 4 * nc * R);
  s->Qt = (real *)zalloc(M * 4 * nc * R);
  s->al = (real *)zalloc(M * nc * R); s->ax = (real *)zalloc(M * nc * R);
  s->ay = (real *)zalloc(M * nc * R);
  s->cx = (real *)zalloc(M * nc * R); s->cy = (real *)zalloc(M * nc * R);
  s->W = (real *)zalloc(M * 4 * nc * R); s->lw = (real *)zalloc(4 * nc * R);
  s->Wv = (unsigned char *)zalloc(M * nc); s->lok = (unsigned char *)zalloc(nc);
  s->band = (unsigned char *)zalloc(nc);
  s->band2 = (unsigned char *)zalloc(nc); s->list = (int *)zalloc(nc * 4);
  s->X = (real *)zalloc(M * 4 * nc * R);
  s->vx = (real *)zalloc(nc * R); s->vy = (real *)zalloc(nc * R);
  s->vok = (unsigned char *)zalloc(nc); s->reg = (unsigned char *)zalloc(nc);
  s->lv = (real *)zalloc(2 * nc * R);
  s->Fx = (real *)zalloc(M * 4 * nc * R); s->Fy = (real *)zalloc(M * 4 * nc * R);
  s->mass = (real *)zalloc(M * nc * R);
  s->cv = (real *)zalloc(nc * R); s->co = (int *)zalloc(nc * 4);
  s->xs = (unsigned char *)zalloc(nc);
  s->mixM = (real *)zalloc(3 * 4 * nc * R); s->mixT = (int *)zalloc(3 * nc * 4);
  s->abk = (int *)zalloc(M * nc * 4); s->abr = (int *)zalloc(M * nc * 4);
  s->rlk = (int *)zalloc(nc * 4); s->rlto = (int *)zalloc(nc * 4);
  for (int v = 0; v < 4; v++) s->inflow[v] = c->inflow_W[v];
  if (!s->mixT || !s->mixM || !s->Q) {
    or_destroy(s);
    return NULL;
  }
  return s;
}

/* Initial state: phi, chi [ny][nx]; W [n_mat][dim+2][ny][nx] primitive
 * (rho, u, [v], p) of each material, used wherever that material has a
 * volume fraction.  Q^0 = alpha^0 U(W), with alpha^0 corrected by the
 * masses alpha * rho. */
/* Input field W (and, in the tangent build, its derivative dW, nullable). */
static real w_in(const double *W, const double *dW, size_t at) {
#ifdef OR_TANGENT
  return or_dual(W[at], dW ? dW[at] : 0.0);
#else
  (void)dW;
  return W[at];
#endif
}

static int init_impl(St *s, const double *phi, const int32_t *chi, const double *W,
                     const double *dW) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      if (chi[q] < 0 || chi[q] >= s->M || !(phi[q] >= 0.0)) return OR_EINVAL;
      s->phi[ID(s, i, j)] = phi[q];
      s->chi[ID(s, i, j)] = chi[q];
    }
  fill_ls(s, s->phi, s->chi);
  geometry(s, s->phi, s->chi);
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        size_t q = (size_t)j * nx + i;
        M1(s, s->mass, r, ID(s, i, j)) =
            M1(s, s->al, r, ID(s, i, j)) * w_in(W, dW, ((size_t)r * nv + 0) * plane + q);
      }
  vf_correction(s, s->chi, s->mass);
  s->err_code = OR_OK;
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        size_t q = (size_t)j * nx + i;
        int k = ID(s, i, j);
        real a = M1(s, s->al, r, k);
        real w[4];
        w[0] = w_in(W, dW, ((size_t)r * nv + 0) * plane + q);
        w[1] = w_in(W, dW, ((size_t)r * nv + 1) * plane + q);
        w[2] = nv == 4 ? w_in(W, dW, ((size_t)r * nv + 2) * plane + q) : (real)0.0;
        w[3] = w_in(W, dW, ((size_t)r * nv + nv - 1) * plane + q);
        if (a > 0.0 && (!(w[0] > 0.0) || !(w[3] + s->pinfe[r] > 0.0) ||
                        !isfinite(w[1]) || !isfinite(w[2])))
          record_err(s, OR_ENONPHYS, i, j);
        real U[4];
        U[0] = w[0];
        U[1] = w[0] * w[1];
        U[2] = w[0] * w[2];
        U[3] = energy(s, r, w[0], w[1], w[2], w[3]);
        for (int v = 0; v < 4; v++) M4(s, s->Q, r, v, k) = a > 0.0 ? a * U[v] : 0.0;
      }
  s->t = 0.0;
  s->nstep = 0;
  memset(s->bnd, 0, sizeof(s->bnd));
  memset(s->bnd_c, 0, sizeof(s->bnd_c));
  memset(s->xsum, 0, sizeof(s->xsum));
  memset(s->xsum_c, 0, sizeof(s->xsum_c));
  memset(s->xfer, 0, sizeof(s->xfer));
  memset(s->xfer_c, 0, sizeof(s->xfer_c));
  return s->err_code;
}

int or_init(St *s, const double *phi, const int32_t *chi, const double *W) {
  return init_impl(s, phi, chi, W, NULL);
}

/* Geometry and correction of the current level set, as after a step
 * (masses: the partial densities of the current state). */
static void state_geometry(St *s) {
  fill_ls(s, s->phi, s->chi);
  geometry(s, s->phi, s->chi);
  for (int r = 0; r < s->M; r++)
    for (size_t k = 0; k < (size_t)s->NC; k++) M1(s, s->mass, r, k) = M4(s, s->Q, r, 0, k);
  vf_correction(s, s->chi, s->mass);
}

/* Replace the state: Q [n_mat][dim+2][ny][nx] (alpha U), phi >= 0 and chi
 * [ny][nx]; the geometry is rebuilt.  Derivative parts (tangent build) are
 * cleared. */
int or_set_state(St *s, const double *Q, const double *phi, const int32_t *chi) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  for (size_t q = 0; q < plane; q++)
    if (chi[q] < 0 || chi[q] >= s->M || !(phi[q] >= 0.0)) return OR_EINVAL;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      int k = ID(s, i, j);
      for (int r = 0; r < s->M; r++) {
        M4(s, s->Q, r, 0, k) = Q[((size_t)r * nv + 0) * plane + q];
        M4(s, s->Q, r, 1, k) = Q[((size_t)r * nv + 1) * plane + q];
        M4(s, s->Q, r, 2, k) = nv == 4 ? Q[((size_t)r * nv + 2) * plane + q] : 0.0;
        M4(s, s->Q, r, 3, k) = Q[((size_t)r * nv + nv - 1) * plane + q];
      }
      s->phi[k] = phi[q];
      s->chi[k] = chi[q];
    }
  state_geometry(s);
  return OR_OK;
}

/* Replay a fixed step size instead of the CFL one (0 = CFL). */
void or_set_dt(St *s, double dt) { s->dt_fixed = dt; }

/* One full time step in the fixed stage order: primitive and ghost states,
 * (dt at stage 0), interface exchange, fluxes and RK update, level-set
 * stage, frame of the level set, geometry + correction of the new stage,
 * mixing. */
int or_step(St *s, int nsteps) {
  double b[3], c[3], w[3];
  int ns = rk_stages(s, b, c, w);
  size_t qb = (size_t)s->M * 4 * s->NC * sizeof(real);
  for (int n = 0; n < nsteps; n++) {
    memcpy(s->Qn, s->Q, qb);
    memcpy(s->phin, s->phi, s->NC * sizeof(real));
    memcpy(s->chin, s->chi, s->NC * sizeof(int));
    for (int st = 0; st < ns; st++) {
      s->err_code = OR_OK;
      /* time of the stage's input state: t_n, then t_n + dt (and for RK3
         t_n + dt/2) */
      s->tstage = st == 0 ? s->t : s->t + (st == 1 ? 1.0 : 0.5) * (double)RV(s->dt);
      local_sets(s, s->chi, s->xs);
      real_states(s);
      if (s->err_code) return s->err_code;
      /* the step size is a function of the state, but it is held fixed
         under differentiation (the derivative is taken at frozen dt) */
      if (st == 0) s->dt = s->dt_fixed > 0.0 ? (real)s->dt_fixed : CONST_R(cfl_dt(s));
      extension(s);
      fill_W(s);
      interface_exchange(s, st);
      if (st == 0) ls_velocity(s);
      fluxes(s);
      rk_update(s, b[st], c[st], w[st]);
      ls_region(s);
      levelset_stage(s, b[st], c[st]);
      fill_ls(s, s->phit, s->chit);
      geometry(s, s->phit, s->chit);
      for (int r = 0; r < s->M; r++)
        for (size_t k = 0; k < (size_t)s->NC; k++)
          M1(s, s->mass, r, k) = M4(s, s->Qt, r, 0, k);
      vf_correction(s, s->chit, s->mass);
      s->xw = 1.0;
      for (int later = st + 1; later < ns; later++) s->xw *= c[later];
      mixing(s);
      if (s->nrl) {
        /* relabelled cells: geometry and correction of the new indicator
           field, the correction ordered by the masses after mixing */
        for (long a = 0; a < s->nrl; a++) s->chit[s->rlk[a]] = s->rlto[a];
        fill_ls(s, s->phit, s->chit);
        geometry(s, s->phit, s->chit);
        for (int r = 0; r < s->M; r++)
          for (size_t k = 0; k < (size_t)s->NC; k++)
            M1(s, s->mass, r, k) = M4(s, s->Q, r, 0, k);
        vf_correction(s, s->chit, s->mass);
      }
      real *tp = s->phi; s->phi = s->phit; s->phit = tp;
      int *tc = s->chi; s->chi = s->chit; s->chit = tc;
    }
    s->t += RV(s->dt);
    s->nstep++;
    s->xw = 1.0;
    if (s->c.scale_sep) scale_separation(s);
    if (s->c.reinit) reinit(s);
  }
  return OR_OK;
}

/* Copy out Q [n_mat][dim+2][ny][nx], alpha [n_mat][ny][nx] (nullable),
 * phi, chi [ny][nx] (nullable). */
int or_get(const St *s, double *Q, double *alpha, double *phi, int32_t *chi) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      int k = ID(s, i, j);
      for (int r = 0; r < s->M; r++) {
        if (Q) {
          Q[((size_t)r * nv + 0) * plane + q] = RV(M4(s, s->Q, r, 0, k));
          Q[((size_t)r * nv + 1) * plane + q] = RV(M4(s, s->Q, r, 1, k));
          if (nv == 4) Q[((size_t)r * nv + 2) * plane + q] = RV(M4(s, s->Q, r, 2, k));
          Q[((size_t)r * nv + nv - 1) * plane + q] = RV(M4(s, s->Q, r, 3, k));
        }
        if (alpha) alpha[(size_t)r * plane + q] = RV(M1(s, s->al, r, k));
      }
      if (phi) phi[q] = RV(s->phi[k]);
      if (chi) chi[q] = s->chi[k];
    }
  return OR_OK;
}

/* Face apertures of the current geometry: Ax [n_mat][ny][nx+1] (x-face i-1/2
 * at column i), Ay [n_mat][ny+1][nx] (y-face j-1/2 at row j). */
int or_get_apertures(const St *s, double *Ax, double *Ay) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int r = 0; r < s->M; r++) {
    for (int j = 0; j < ny; j++)
      for (int i = 0; i <= nx; i++)
        Ax[((size_t)r * ny + j) * (nx + 1) + i] = RV(M1(s, s->ax, r, ID(s, i - 1, j)));
    if (Ay && s->c.dim == 2)
      for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++)
          Ay[((size_t)r * (ny + 1) + j) * nx + i] = RV(M1(s, s->ay, r, ID(s, i, j - 1)));
  }
  return OR_OK;
}

/* Diagnostics: out[0..8] = t, dt, steps, positivity fallbacks, skipped
 * fluxes, skipped interfaces, stranded mixing sources, mixing sources,
 * material-cell updates; then bnd[n_mat][4] (net boundary inflow) and
 * xsum[n_mat][4] (exchange totals), both as increments of sum(Q). */
int or_diag(const St *s, double *out) {
  out[0] = s->t;
  out[1] = RV(s->dt);
  out[2] = (double)s->nstep;
  out[3] = (double)s->n_posfix;
  out[4] = (double)s->n_fluxskip;
  out[5] = (double)s->n_ifskip;
  out[6] = (double)s->n_stranded;
  out[7] = (double)s->n_mixsrc;
  out[8] = (double)s->n_upd;
  for (int r = 0; r < s->M; r++)
    for (int v = 0; v < 4; v++) {
      out[9 + r * 4 + v] = RV(s->bnd[r][v] + s->bnd_c[r][v]);
      out[9 + s->M * 4 + r * 4 + v] = RV(s->xsum[r][v] + s->xsum_c[r][v]);
    }
  for (int r = 0; r < s->M; r++)
    for (int v = 0; v < 4; v++) out[12 + 8 * s->M + r * 4 + v] = RV(s->xfer[r][v] + s->xfer_c[r][v]);
  out[9 + 8 * s->M] = (double)s->n_absorb;
  out[10 + 8 * s->M] = (double)s->n_relabel;
  out[11 + 8 * s->M] = (double)s->n_oddball;
  return OR_OK;
}

long or_err_cell(const St *s) { return s->err_cell; }

/* ------------------------------------------------------------------------ */
/* Unit entry points for the oracle's own pins                              */
/* ------------------------------------------------------------------------ */
double or_t_weno5(double v1, double v2, double v3, double v4, double v5) {
  return RV(weno5(v1, v2, v3, v4, v5));
}

/* HLLC face flux of material m between primitive states (rho, un, ut, p). */
void or_t_hllc(const St *s, int m, const double *WL, const double *WR, double *F) {
  real L[4], R[4], G[4];
  for (int v = 0; v < 4; v++) {
    L[v] = WL[v];
    R[v] = WR[v];
  }
  hllc_flux(s, m, L, R, G);
  for (int v = 0; v < 4; v++) F[v] = RV(G[v]);
}

/* Roe face flux of material m between primitive states (rho, un, ut, p). */
void or_t_roe(St *s, int m, const double *WL, const double *WR, double *F) {
  real L[4], R[4], G[4];
  for (int v = 0; v < 4; v++) {
    L[v] = WL[v];
    R[v] = WR[v];
  }
  roe_flux(s, m, L, R, G);
  for (int v = 0; v < 4; v++) F[v] = RV(G[v]);
}

/* Characteristic-wise WENO5 states at a face from six stencil states
 * Wc[q] = (rho, u_n, u_t, p), q = 0..5 (cells i-2 .. i+3 of face i+1/2). */
/* the redistancing alone, on the current state (its level set is replaced) */
void or_t_reinit(St *s) { reinit(s); }

void or_t_char_weno(St *s, int m, const double *Wc, double *WL, double *WR) {
  real W6[6][4], L[4], R[4];
  int perm[4] = {0, 1, 2, 3};
  for (int q = 0; q < 6; q++)
    for (int v = 0; v < 4; v++) W6[q][v] = Wc[q * 4 + v];
  char_weno(s, m, W6, perm, L, R);
  for (int v = 0; v < 4; v++) {
    WL[v] = RV(L[v]);
    WR[v] = RV(R[v]);
  }
}

/* Interface Riemann problem between material mL (left state) and mR (right
 * state), states (rho, un, ut, p); out = (S_L, S_R, S_M, p*). */
void or_t_iface(const St *s, int mL, const double *WLd, int mR, const double *WRd,
                double *out) {
  real WL[4], WR[4];
  for (int v = 0; v < 4; v++) {
    WL[v] = WLd[v];
    WR[v] = WRd[v];
  }
  real SL, SR;
  wave_speeds(WL, s->c.gamma[mL], s->pinfe[mL], s->tait[mL], WR, s->c.gamma[mR], s->pinfe[mR],
              s->tait[mR], &SL, &SR);
  real SM = contact_speed(WL, WR, SL, SR);
  real pL = WL[3], pR = WR[3], uL = WL[1], uR = WR[1];
  out[0] = RV(SL);
  out[1] = RV(SR);
  out[2] = RV(SM);
  out[3] = RV(0.5 * ((pL + WL[0] * (SL - uL) * (SM - uL)) + (pR + WR[0] * (SR - uR) * (SM - uR))));
}

/* Interface closure vectors of the current geometry, [n_mat][ny][nx] each. */
int or_get_closure(const St *s, double *cx, double *cy) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        size_t q = ((size_t)r * ny + j) * nx + i;
        cx[q] = RV(M1(s, s->cx, r, ID(s, i, j)));
        cy[q] = RV(M1(s, s->cy, r, ID(s, i, j)));
      }
  return OR_OK;
}

/* Interior cells of a [ny][nx] input into a padded field (frame left zero). */
static void load_plane_d(St *s, real *f, const double *in) {
  int nx = s->c.nx, ny = s->c.ny;
  memset(f, 0, (size_t)s->NC * sizeof(real));
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) f[ID(s, i, j)] = in[(size_t)j * nx + i];
}

/* The level set (phi, chi) [ny][nx] into the given padded fields, with its
 * boundary frame. */
static int load_ls(St *s, real *phi, int *chi, const double *ph, const int32_t *ch) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      if (ch[q] < 0 || ch[q] >= s->M || !(ph[q] >= 0.0)) return OR_EINVAL;
      phi[ID(s, i, j)] = ph[q];
      chi[ID(s, i, j)] = ch[q];
    }
  fill_ls(s, phi, chi);
  return OR_OK;
}

/* Mixing alone (Sec. 2.3.2, the step after each Runge-Kutta sub-step).
 * Qt [n_mat][dim+2][ny][nx] is the state after the stage update, alpha
 * [n_mat][ny][nx] the volume fractions and (phi, chi) [ny][nx] the level set
 * of the new stage (alpha need not be the geometry of phi: the unit pins
 * choose both); Q [n_mat][dim+2][ny][nx] receives the mixed state.  The
 * source and stranded-source counters of or_diag are advanced. */
int or_t_mixing(St *s, const double *Qt, const double *alpha, const double *phi,
                const int32_t *chi, double *Q) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  if (load_ls(s, s->phit, s->chit, phi, chi)) return OR_EINVAL;
  memset(s->Qt, 0, (size_t)s->M * 4 * s->NC * sizeof(real));
  for (int r = 0; r < s->M; r++) {
    load_plane_d(s, &M1(s, s->al, r, 0), alpha + (size_t)r * plane);
    int src[4] = {0, 1, nv == 4 ? 2 : -1, nv - 1};
    for (int v = 0; v < 4; v++)
      if (src[v] >= 0)
        load_plane_d(s, &M4(s, s->Qt, r, v, 0), Qt + ((size_t)r * nv + src[v]) * plane);
  }
  mixing(s);
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        size_t q = (size_t)j * nx + i;
        int k = ID(s, i, j);
        Q[((size_t)r * nv + 0) * plane + q] = RV(M4(s, s->Q, r, 0, k));
        Q[((size_t)r * nv + 1) * plane + q] = RV(M4(s, s->Q, r, 1, k));
        if (nv == 4) Q[((size_t)r * nv + 2) * plane + q] = RV(M4(s, s->Q, r, 2, k));
        Q[((size_t)r * nv + nv - 1) * plane + q] = RV(M4(s, s->Q, r, 3, k));
      }
  return OR_OK;
}

/* Ghost-state extension alone (Sec. 2.3.2, the ghost state of a material
 * outside its region).  (phi, chi) [ny][nx] is the level set; W
 * [n_mat][4][ny][nx] (rho, u, v, p) and valid [n_mat][ny][nx] the states
 * present before the extension (real cells); Wout and vout receive the
 * states and validity after it. */
int or_t_extension(St *s, const double *phi, const int32_t *chi, const double *W,
                   const unsigned char *valid, double *Wout, unsigned char *vout) {
  int nx = s->c.nx, ny = s->c.ny;
  size_t plane = (size_t)nx * ny;
  if (load_ls(s, s->phi, s->chi, phi, chi)) return OR_EINVAL;
  memset(s->Wv, 0, (size_t)s->M * s->NC);
  for (int r = 0; r < s->M; r++) {
    for (int v = 0; v < 4; v++)
      load_plane_d(s, &M4(s, s->W, r, v, 0), W + ((size_t)r * 4 + v) * plane);
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++)
        M1(s, s->Wv, r, ID(s, i, j)) = valid[(size_t)r * plane + (size_t)j * nx + i] ? 1 : 0;
  }
  extension(s);
  for (int r = 0; r < s->M; r++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        size_t q = (size_t)j * nx + i;
        int k = ID(s, i, j);
        for (int v = 0; v < 4; v++) Wout[((size_t)r * 4 + v) * plane + q] = RV(M4(s, s->W, r, v, k));
        vout[(size_t)r * plane + q] = M1(s, s->Wv, r, k);
      }
  return OR_OK;
}

/* Level-set advection velocity alone (Eq. local-advection's v^n).  (phi,
 * chi) [ny][nx] is the level set; v [2][ny][nx] and vok [ny][nx] the
 * velocities already set (the interface cells' S_M n); W [n_mat][4][ny][nx]
 * and valid [n_mat][ny][nx] the material states.  vout [2][ny][nx] receives
 * the velocity field. */
int or_t_ls_velocity(St *s, const double *phi, const int32_t *chi, const double *v,
                     const unsigned char *vok, const double *W, const unsigned char *valid,
                     double *vout) {
  int nx = s->c.nx, ny = s->c.ny;
  size_t plane = (size_t)nx * ny;
  if (load_ls(s, s->phi, s->chi, phi, chi)) return OR_EINVAL;
  load_plane_d(s, s->vx, v);
  load_plane_d(s, s->vy, v + plane);
  memset(s->vok, 0, (size_t)s->NC);
  memset(s->Wv, 0, (size_t)s->M * s->NC);
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) s->vok[ID(s, i, j)] = vok[(size_t)j * nx + i] ? 1 : 0;
  for (int r = 0; r < s->M; r++) {
    for (int c = 0; c < 4; c++)
      load_plane_d(s, &M4(s, s->W, r, c, 0), W + ((size_t)r * 4 + c) * plane);
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++)
        M1(s, s->Wv, r, ID(s, i, j)) = valid[(size_t)r * plane + (size_t)j * nx + i] ? 1 : 0;
  }
  ls_velocity(s);
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      vout[(size_t)j * nx + i] = RV(s->vx[ID(s, i, j)]);
      vout[plane + (size_t)j * nx + i] = RV(s->vy[ID(s, i, j)]);
    }
  return OR_OK;
}

#ifdef OR_TANGENT
/* ------------------------------------------------------------------------ */
/* Tangent build only: directional derivatives of the discrete step         */
/* ------------------------------------------------------------------------ */
/* Initial state with the derivative dW of the input field W (same layout);
 * the level set carries no derivative. */
int or_init_tangent(St *s, const double *phi, const int32_t *chi, const double *W,
                    const double *dW) {
  return init_impl(s, phi, chi, W, dW);
}

/* Derivative of the primitive state on inflow sides (held for every step). */
void or_set_inflow_tangent(St *s, const double *d) {
  for (int v = 0; v < 4; v++) s->inflow[v] = or_dual(RV(s->inflow[v]), d[v]);
}

/* Replace the derivative part of the current state: dQ [n_mat][dim+2][ny][nx]
 * and dphi [ny][nx]; the geometry is rebuilt as by or_set_state. */
void or_seed_state(St *s, const double *dQ, const double *dphi) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      int k = ID(s, i, j);
      for (int r = 0; r < s->M; r++) {
        int src[4] = {0, 1, nv == 4 ? 2 : -1, nv - 1};
        for (int v = 0; v < 4; v++) {
          real *x = &M4(s, s->Q, r, v, k);
          *x = or_dual(RV(*x), src[v] < 0 ? 0.0 : dQ[((size_t)r * nv + src[v]) * plane + q]);
        }
      }
      s->phi[k] = or_dual(RV(s->phi[k]), dphi[q]);
    }
  /* the geometry of the current level set is an input of the next step */
  state_geometry(s);
}

/* Derivative parts of the state: dQ, dalpha (nullable), dphi (nullable). */
int or_get_tangent(const St *s, double *dQ, double *dalpha, double *dphi) {
  int nx = s->c.nx, ny = s->c.ny, nv = s->c.dim + 2;
  size_t plane = (size_t)nx * ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t q = (size_t)j * nx + i;
      int k = ID(s, i, j);
      for (int r = 0; r < s->M; r++) {
        if (dQ) {
          dQ[((size_t)r * nv + 0) * plane + q] = M4(s, s->Q, r, 0, k).d;
          dQ[((size_t)r * nv + 1) * plane + q] = M4(s, s->Q, r, 1, k).d;
          if (nv == 4) dQ[((size_t)r * nv + 2) * plane + q] = M4(s, s->Q, r, 2, k).d;
          dQ[((size_t)r * nv + nv - 1) * plane + q] = M4(s, s->Q, r, 3, k).d;
        }
        if (dalpha) dalpha[(size_t)r * plane + q] = M1(s, s->al, r, k).d;
      }
      if (dphi) dphi[q] = s->phi[k].d;
    }
  return OR_OK;
}
#endif

#ifdef __cplusplus
}
#endif
