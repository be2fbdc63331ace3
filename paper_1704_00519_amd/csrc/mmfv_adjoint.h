// Adjoint of the time step: the transpose of the step linearised about the
// forward trajectory, with the step size dt held fixed and every branch
// (upwind choices, HLLC wave pattern, ghost-cell sources, interface pairs,
// mixing sources and targets, level-set argmax, volume-fraction correction)
// taken as the forward step took it.  Stages are reversed in the opposite
// order; within a stage each operator of the step is transposed in turn:
//
//   mixing (Sec. 2.3.2)  ->  geometry of the new level set (Sec. 2.3)
//   -> level-set stage (Eq. local-advection, Eq. reconstruction)
//   -> RK stage update (Eq. discretized_equ)  -> aperture-weighted fluxes
//   -> level-set velocity (stage 0)  -> interface exchange (Sec. 2.3.2)
//   -> primitive-state frames  -> ghost extension  -> real states
//   -> geometry of the stage's level set.
//
// Point-wise local Jacobians (WENO5, HLLC, interface Riemann problem,
// primitive variables, cut-cell fractions) come from forward-mode
// evaluation of the very templates the step uses (mmfv_dual.h); the
// transposition of the stencils, of the sweeps and of the RK combination is
// written out here.  Scatters into shared adjoint entries use FP64 atomics,
// so adjoint values are reproducible to rounding, not bit for bit.
#pragma once
#include "mmfv_dual.h"
#include "mmfv_kernels.h"

namespace mmfv {

struct Adj {
  double* lQ;      // [M][4][NC] adjoint of the stage input Q^(s) (1D: comp 2 unused)
  double* lQs;     // [M][4][NC] adjoint of Q* (after the update, before mixing)
  double* lQn;     // [M][4][NC] adjoint of Q^n collected from later stages
  double* lphi;    // [NC] adjoint of phi^(s)
  double* lphis;   // [NC] adjoint of the stage's new level set phi*
  double* lphin;   // [NC] adjoint of phi^n collected from later stages
  double* lW;      // [M][4][NC] adjoint of the primitive states
  double *lal, *lax, *lay, *lcx, *lcy;  // [M][NC] adjoint of the geometry
  double *lvx, *lvy;                     // [NC] adjoint of v^n
  double* linflow;   // [4] adjoint of the inflow state, accumulated
  double* Qstar;     // [M][D+2][NC] copy of Q* (before mixing)
  uint8_t* occstar;  // its occupancy
  double* lalpha;    // [M][NC] adjoint of the step's output volume fractions
  double* lW2;       // [M][4][NC] output buffer of the tile-wise ghost-state adjoint
};

MMD double& A4(const Params& P, double* a, int r, int v, int k) {
  return a[((size_t)r * 4 + v) * P.NC + k];
}
MMD double& A1(const Params& P, double* a, int r, int k) { return a[(size_t)r * P.NC + k]; }
// sign of the construction operator: phi^r = s phi with s = +1 inside r
MMD double lsgn(const uint8_t* chi, int r, int k) { return chi[k] == r ? 1.0 : -1.0; }
MMD void aadd(double* p, double x) {
  if (x != 0.0) atomicAdd(p, x);
}

#define ADJ_CELL_LOOP                                        \
  int i = blockIdx.x * blockDim.x + threadIdx.x;             \
  int j = blockIdx.y * blockDim.y + threadIdx.y;             \
  if (i >= P.nx || j >= P.ny) return;                        \
  int k = cid(P, i, j);

// ---------------------------------------------------------------------------
// Mixing (Sec. 2.3.2).  Q^(s+1) = Q* + sum of exchanges; sources, targets
// and exchanges are recomputed from Q* (A.Qstar) and the new level set and
// geometry (in B).  In: A.lQ (the adjoint of Q^(s+1), already copied into
// A.lQs); out: A.lQs, A.lal (new geometry), A.lphis (through the normal
// directions).
// ---------------------------------------------------------------------------
// Grid slice z = M (the step's first reversed stage only): one thread sets
// the step size of the step from the recorded one (no kernel of this phase
// reads it).
template <int D>
__global__ void __launch_bounds__(256) k_a_mix(Params P, Bufs B, Adj A) {
  if ((int)blockIdx.z == P.M) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
      double smax = __longlong_as_double((long long)B.ctr[C_SMAX]);
      B.ctr[C_SMAX] = 0;
      dt_finish<D>(P, B, smax);
    }
    return;
  }
  ADJ_CELL_LOOP
  double amix = P.amix;
  // the sources of the forward mixing, from Q* and the new geometry; one
  // material per grid slice z
  if (!B.cut[k] && A.occstar[k] == (uint8_t)(1u << B.chi[k])) return;
  for (int r = blockIdx.z; r == (int)blockIdx.z; r++) {
    double as = alpha_at<D>(P, B, r, k);
    // own-material parts with nothing in them, or with 0 < alpha < 1 and no
    // mass, are sources like new cells
    if (!(as < amix) && B.chi[k] == r) {
      bool nz = false;
      for (int v = 0; v < 4; v++)
        if (loadQ<D>(P, A.Qstar, A.occstar, r, v, k) != 0.0) nz = true;
      bool nomass = !nz || (!(loadQ<D>(P, A.Qstar, A.occstar, r, 0, k) > 0.0) && as < 1.0);
      if (!(nomass && as > 0.0)) continue;
    }
    if (!(as > 0.0)) {
      bool nz = false;
      for (int v = 0; v < 4; v++)
        if (loadQ<D>(P, A.Qstar, A.occstar, r, v, k) != 0.0) nz = true;
      if (!nz) continue;
    }
    int kxp = cid(P, i + 1, j), kxm = cid(P, i - 1, j);
    double gx = lsv(B.phi, B.chi, r, kxp) - lsv(B.phi, B.chi, r, kxm);
    double gy = 0.0;
    int kyp = k, kym = k;
    if (D == 2) {
      kyp = cid(P, i, j + 1);
      kym = cid(P, i, j - 1);
      gy = lsv(B.phi, B.chi, r, kyp) - lsv(B.phi, B.chi, r, kym);
    }
    int sx = gx > 0.0 ? 1 : (gx < 0.0 ? -1 : 0);
    int sy = gy > 0.0 ? 1 : (gy < 0.0 ? -1 : 0);
    int tk[3] = {-1, -1, -1};
    double w[3] = {0.0, 0.0, 0.0}, at[3] = {0.0, 0.0, 0.0};
    auto eligible = [&](int ii, int jj, double& a) -> bool {
      if (!interior(P, ii, jj)) return false;
      int t = cid(P, ii, jj);
      a = alpha_at<D>(P, B, r, t);
      return a >= amix && B.chi[t] == r;
    };
    double a;
    if (sx != 0 && eligible(i + sx, j, a)) {
      tk[0] = cid(P, i + sx, j);
      at[0] = a;
      w[0] = gx * gx * a;
    }
    if (sy != 0 && eligible(i, j + sy, a)) {
      tk[1] = cid(P, i, j + sy);
      at[1] = a;
      w[1] = gy * gy * a;
    }
    if (sx != 0 && sy != 0 && eligible(i + sx, j + sy, a)) {
      tk[2] = cid(P, i + sx, j + sy);
      at[2] = a;
      w[2] = fabs(gx * gy) * a;
    }
    double wsum = (w[0] + w[1]) + w[2];
    double beta[3] = {0.0, 0.0, 0.0};
    bool fallback = !(wsum > 0.0);
    if (!fallback) {
      for (int q = 0; q < 3; q++)
        if (w[q] > 0.0)
          beta[q] = w[q] / wsum;
        else
          tk[q] = -1;
    } else {
      tk[0] = tk[1] = tk[2] = -1;
      double bestA = -1.0;
      int bt = -1;
      for (int dj = -(D == 2); dj <= (D == 2); dj++)
        for (int di = -1; di <= 1; di++) {
          if (di == 0 && dj == 0) continue;
          if (eligible(i + di, j + dj, a) && a > bestA) {
            bestA = a;
            bt = cid(P, i + di, j + dj);
          }
        }
      if (bt < 0) continue;  // stranded: nothing was exchanged
      tk[0] = bt;
      at[0] = bestA;
      beta[0] = 1.0;
    }
    int last = -1;
    for (int q = 0; q < 3; q++)
      if (tk[q] >= 0) last = q;
    double lbeta[3] = {0.0, 0.0, 0.0}, lat[3] = {0.0, 0.0, 0.0}, las = 0.0;
    for (int v = 0; v < 4; v++) {
      if (D == 1 && v == 2) continue;
      double Qs = loadQ<D>(P, A.Qstar, A.occstar, r, v, k);
      double ls = A4(P, A.lQ, r, v, k);
      double lQsrc = 0.0;
      if (as > 0.0) {
        for (int q = 0; q < 3; q++) {
          if (tk[q] < 0) continue;
          double Qt = loadQ<D>(P, A.Qstar, A.occstar, r, v, tk[q]);
          double lM = ls - A4(P, A.lQ, r, v, tk[q]);
          double den = as + at[q];
          double b = beta[q];
          aadd(&A4(P, A.lQs, r, v, tk[q]), lM * b * as / den);
          lQsrc += -lM * b * at[q] / den;
          las += lM * b * at[q] * (Qt + Qs) / (den * den);
          lat[q] += -lM * b * as * (Qs + Qt) / (den * den);
          lbeta[q] += lM * (as * Qt - at[q] * Qs) / den;
        }
      } else {
        // vanishing source: M_q = -beta_q Qs, the last target takes the
        // remainder M_last = -Qs + sum_{q<last} beta_q Qs
        double lMlast = ls - A4(P, A.lQ, r, v, tk[last]);
        double sb = 0.0;
        for (int q = 0; q < last; q++) {
          if (tk[q] < 0) continue;
          double lM = ls - A4(P, A.lQ, r, v, tk[q]);
          lQsrc += -lM * beta[q];
          lbeta[q] += Qs * (lMlast - lM);
          sb += beta[q];
        }
        lQsrc += lMlast * (-1.0 + sb);
      }
      aadd(&A4(P, A.lQs, r, v, k), lQsrc);
    }
    aadd(&A1(P, A.lal, r, k), las);
    for (int q = 0; q < 3; q++)
      if (tk[q] >= 0) aadd(&A1(P, A.lal, r, tk[q]), lat[q]);
    if (fallback) continue;
    // beta_q = w_q / sum(w)
    double sbl = 0.0;
    for (int q = 0; q < 3; q++)
      if (tk[q] >= 0) sbl += beta[q] * lbeta[q];
    double lgx = 0.0, lgy = 0.0;
    for (int q = 0; q < 3; q++) {
      if (tk[q] < 0) continue;
      double lw = (lbeta[q] - sbl) / wsum;
      if (q == 0) {
        lgx += lw * 2.0 * gx * at[0];
        aadd(&A1(P, A.lal, r, tk[0]), lw * gx * gx);
      } else if (q == 1) {
        lgy += lw * 2.0 * gy * at[1];
        aadd(&A1(P, A.lal, r, tk[1]), lw * gy * gy);
      } else {
        double sg = gx * gy < 0.0 ? -1.0 : 1.0;  // d|x|/dx = +1 at 0, as fabs of the dual types
        lgx += lw * sg * gy * at[2];
        lgy += lw * sg * gx * at[2];
        aadd(&A1(P, A.lal, r, tk[2]), lw * fabs(gx * gy));
      }
    }
    aadd(&A.lphis[kxp], lgx * lsgn(B.chi, r, kxp));
    aadd(&A.lphis[kxm], -lgx * lsgn(B.chi, r, kxm));
    if (D == 2) {
      aadd(&A.lphis[kyp], lgy * lsgn(B.chi, r, kyp));
      aadd(&A.lphis[kym], -lgy * lsgn(B.chi, r, kym));
    }
  }
}

// adjoint of the step's output volume fractions (interior layout in lalpha)
__global__ void __launch_bounds__(256) k_a_add_alpha(Params P, Bufs B, Adj A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  int k = cid(P, i, j);
  for (int r = 0; r < P.M; r++) A1(P, A.lal, r, k) += A1(P, A.lalpha, r, k);
}

// ---------------------------------------------------------------------------
// Geometry (Sec. 2.3) of the level set in B.phi/B.chi, cut cells only (all
// other cells have constant fractions): the adjoints of the corrected volume
// fractions, of the stored apertures and of the closure vectors go to the
// level set through the corner and centre values.  Out: lphi_out (atomics).
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_a_geom(Params P, Bufs B, Adj A, double* lphi_out) {
  ADJ_CELL_LOOP
  if (!B.cut[k]) return;
  const double* phi = B.phi;
  const uint8_t* chi = B.chi;
  // volume-fraction correction: alpha'_f = 1 - sum of the other unclamped
  // fractions; clamped ones are constant zero
  double lam[MAXM];
  for (int r = 0; r < P.M; r++) lam[r] = A1(P, A.lal, r, k);
  unsigned code = B.vfc[k], f = code & 0xff, z = code >> 8;
  if (f != 0xff) {
    double lf = lam[f];
    lam[f] = 0.0;
    for (int r = 0; r < P.M; r++)
      if (r != (int)f && !((z >> r) & 1)) lam[r] -= lf;
  }
  for (int r = 0; r < P.M; r++)
    if ((z >> r) & 1) lam[r] = 0.0;
  for (int r = blockIdx.z; r == (int)blockIdx.z; r++) {  // one material per grid slice z
    if (D == 1) {
      int kl = cid(P, i - 1, j), kr = cid(P, i + 1, j);
      if (lam[r] == 0.0) continue;
      Dn<3> l = dn_seed<3>(lsv(phi, chi, r, kl), 0);
      Dn<3> c = dn_seed<3>(lsv(phi, chi, r, k), 1);
      Dn<3> rr = dn_seed<3>(lsv(phi, chi, r, kr), 2);
      Dn<3> fl = (l + c) * 0.5;
      Dn<3> fr = (c + rr) * 0.5;
      int ol = chi[kl] < chi[k] ? chi[kl] : chi[k];
      int orr = chi[k] < chi[kr] ? chi[k] : chi[kr];
      bool il = inside(fl, ol, r), ir = inside(fr, orr, r), ic = inside(c, chi[k], r);
      Dn<3> al = (seg_frac(fl, il, c, ic) + seg_frac(c, ic, fr, ir)) * 0.5;
      aadd(&lphi_out[kl], lam[r] * al.d[0] * lsgn(chi, r, kl));
      aadd(&lphi_out[k], lam[r] * al.d[1] * lsgn(chi, r, k));
      aadd(&lphi_out[kr], lam[r] * al.d[2] * lsgn(chi, r, kr));
      continue;
    }
    double lAr = A1(P, A.lcx, r, k) * P.dy + A1(P, A.lax, r, k);
    double lAl = -A1(P, A.lcx, r, k) * P.dy + (i == 0 ? A1(P, A.lax, r, cid(P, -1, j)) : 0.0);
    double lAt = A1(P, A.lcy, r, k) * P.dx + A1(P, A.lay, r, k);
    double lAb = -A1(P, A.lcy, r, k) * P.dx + (j == 0 ? A1(P, A.lay, r, cid(P, i, -1)) : 0.0);
    if (lam[r] == 0.0 && lAr == 0.0 && lAl == 0.0 && lAt == 0.0 && lAb == 0.0) continue;
    Dn<5> cv[2][2];
    int co[2][2];
    for (int b = 0; b < 2; b++)
      for (int a = 0; a < 2; a++) {
        int ci = i + a - 1, cj = j + b - 1;
        int k00 = cid(P, ci, cj), k10 = cid(P, ci + 1, cj), k01 = cid(P, ci, cj + 1),
            k11 = cid(P, ci + 1, cj + 1);
        double v = ((lsv(phi, chi, r, k00) + lsv(phi, chi, r, k11)) +
                    (lsv(phi, chi, r, k10) + lsv(phi, chi, r, k01))) * 0.25;
        cv[b][a] = dn_seed<5>(v, b * 2 + a);
        int o = chi[k00];
        if (chi[k10] < o) o = chi[k10];
        if (chi[k01] < o) o = chi[k01];
        if (chi[k11] < o) o = chi[k11];
        co[b][a] = o;
      }
    Dn<5> vsw = cv[0][0], vse = cv[0][1], vnw = cv[1][0], vne = cv[1][1];
    bool isw = inside(vsw, co[0][0], r), ise = inside(vse, co[0][1], r),
         inw = inside(vnw, co[1][0], r), ine = inside(vne, co[1][1], r);
    Dn<5> c = dn_seed<5>(lsv(phi, chi, r, k), 4);
    bool ic = inside(c, chi[k], r);
    Dn<5> Ar = seg_frac(vse, ise, vne, ine);
    Dn<5> Al = seg_frac(vsw, isw, vnw, inw);
    Dn<5> At = seg_frac(vnw, inw, vne, ine);
    Dn<5> Ab = seg_frac(vsw, isw, vse, ise);
    Dn<5> tl = tri_frac(vsw, isw, vnw, inw, c, ic);
    Dn<5> tr = tri_frac(vse, ise, vne, ine, c, ic);
    Dn<5> tb = tri_frac(vsw, isw, vse, ise, c, ic);
    Dn<5> tt = tri_frac(vnw, inw, vne, ine, c, ic);
    Dn<5> al = ((tl + tr) + (tb + tt)) * 0.25;
    double g[5];
    for (int q = 0; q < 5; q++)
      g[q] = lam[r] * al.d[q] + lAr * Ar.d[q] + lAl * Al.d[q] + lAt * At.d[q] + lAb * Ab.d[q];
    for (int b = 0; b < 2; b++)
      for (int a = 0; a < 2; a++) {
        double gc = 0.25 * g[b * 2 + a];
        if (gc == 0.0) continue;
        int ci = i + a - 1, cj = j + b - 1;
        int ks[4] = {cid(P, ci, cj), cid(P, ci + 1, cj), cid(P, ci, cj + 1), cid(P, ci + 1, cj + 1)};
        for (int q = 0; q < 4; q++) aadd(&lphi_out[ks[q]], gc * lsgn(chi, r, ks[q]));
      }
    aadd(&lphi_out[k], g[4] * lsgn(chi, r, k));
  }
}

// ---------------------------------------------------------------------------
// Frames of the level set: every frame cell is a copy of an inside cell, so
// its adjoint is added to that cell.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_a_bc_ls_x(Params P, double* l) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.ny * 2 * H) return;
  int j = t / (2 * H), q = t % (2 * H);
  int ii, si;
  if (q < H) {
    ii = -1 - q;
    si = src_lo(ii, P.bc[0]);
  } else {
    ii = P.nx + (q - H);
    si = src_hi(ii, P.nx, P.bc[1]);
  }
  int k = cid(P, ii, j), ks = cid(P, si, j);
  double x = l[k];
  l[k] = 0.0;
  aadd(&l[ks], x);
}
// both sides in one launch (2D): every frame cell passes its adjoint to the
// interior source of the two maps composed (a corner to the source of the
// x side of its source row), the sum the two passes in sequence deliver
MMD void a_bc_ls2_cell(const Params& P, double* l, int t) {
  int nxs = P.ny * 2 * H, nys = (P.nx + 2 * H) * 2 * H;
  if (t >= nxs + nys) return;
  int i, j, si, sj;
  if (t < nxs) {
    int q = t % (2 * H);
    j = sj = t / (2 * H);
    i = q < H ? -1 - q : P.nx + (q - H);
  } else {
    t -= nxs;
    int q = t % (2 * H);
    i = si = t / (2 * H) - H;
    j = q < H ? -1 - q : P.ny + (q - H);
    sj = q < H ? src_lo(j, P.bc[2]) : src_hi(j, P.ny, P.bc[3]);
  }
  if (i < 0) si = src_lo(i, P.bc[0]);
  if (i >= P.nx) si = src_hi(i, P.nx, P.bc[1]);
  int k = cid(P, i, j), ks = cid(P, si, sj);
  double x = l[k];
  l[k] = 0.0;
  aadd(&l[ks], x);
}
__global__ void __launch_bounds__(256) k_a_bc_ls2(Params P, double* l) {
  a_bc_ls2_cell(P, l, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// RK stage update Q* = b Q^n + c (Q^(s) + rhs): lQn += b lQs, lQ = c lQs.
// ---------------------------------------------------------------------------
MMD void a_update_cell(const Params& P, const Adj& A, int k, double bcoef, double ccoef) {
  for (int r = 0; r < P.M; r++)
    for (int v = 0; v < 4; v++) {
      double l = A4(P, A.lQs, r, v, k);
      if (bcoef != 0.0) A4(P, A.lQn, r, v, k) += bcoef * l;
      A4(P, A.lQ, r, v, k) = ccoef * l;
    }
}

// ---------------------------------------------------------------------------
// Level-set stage (Eq. local-advection, Eq. reconstruction) in the update
// region (dls <= 3); outside it phi is carried over.  In: A.lphis; out:
// A.lphi (stencil, atomics), A.lphin, A.lvx, A.lvy.
// ---------------------------------------------------------------------------
// weno5 of doubles and its gradient g[q] = d weno5 / d v_{q+1}, in one
// forward and one reverse pass over its formula (the derivative of
// each of its steps, taken in reverse order)
MMD double weno5_grad(double v1, double v2, double v3, double v4, double v5, double g[5]) {
  const double c13 = 13.0 / 12.0;
  double t0 = v1 - 2.0 * v2 + v3, u0 = v1 - 4.0 * v2 + 3.0 * v3;
  double t1 = v2 - 2.0 * v3 + v4, u1 = v2 - v4;
  double t2 = v3 - 2.0 * v4 + v5, u2 = 3.0 * v3 - 4.0 * v4 + v5;
  double s0 = 1e-6 + (c13 * (t0 * t0) + 0.25 * (u0 * u0));
  double s1 = 1e-6 + (c13 * (t1 * t1) + 0.25 * (u1 * u1));
  double s2 = 1e-6 + (c13 * (t2 * t2) + 0.25 * (u2 * u2));
  double e0 = s0 * s0, e1 = s1 * s1, e2 = s2 * s2;
  double a0 = 0.1 * (e1 * e2), a1 = 0.6 * (e0 * e2), a2 = 0.3 * (e0 * e1);
  double q0 = 2.0 * v1 - 7.0 * v2 + 11.0 * v3;
  double q1 = -v2 + 5.0 * v3 + 2.0 * v4;
  double q2 = 2.0 * v3 + 5.0 * v4 - v5;
  double S = a0 + a1 + a2;
  double y = (a0 * q0 + a1 * q1 + a2 * q2) / (6.0 * S);
  // y = N / (6 S): dN = 1 / (6 S), dS = -y / S
  double dN = 1.0 / (6.0 * S), dS = -y / S;
  double da0 = q0 * dN + dS, da1 = q1 * dN + dS, da2 = q2 * dN + dS;
  double dq0 = a0 * dN, dq1 = a1 * dN, dq2 = a2 * dN;
  double de0 = 0.6 * e2 * da1 + 0.3 * e1 * da2;
  double de1 = 0.1 * e2 * da0 + 0.3 * e0 * da2;
  double de2 = 0.1 * e1 * da0 + 0.6 * e0 * da1;
  // e_k = s_k^2, s_k = eps + c13 t_k^2 + u_k^2 / 4
  double ds0 = 2.0 * s0 * de0, ds1 = 2.0 * s1 * de1, ds2 = 2.0 * s2 * de2;
  double dt0 = 2.0 * c13 * t0 * ds0, du0 = 0.5 * u0 * ds0;
  double dt1 = 2.0 * c13 * t1 * ds1, du1 = 0.5 * u1 * ds1;
  double dt2 = 2.0 * c13 * t2 * ds2, du2 = 0.5 * u2 * ds2;
  g[0] = 2.0 * dq0 + dt0 + du0;
  g[1] = -7.0 * dq0 - dq1 - 2.0 * dt0 - 4.0 * du0 + dt1 + du1;
  g[2] = 11.0 * dq0 + 5.0 * dq1 + 2.0 * dq2 + dt0 + 3.0 * du0 - 2.0 * dt1 + dt2 + 3.0 * du2;
  g[3] = 2.0 * dq1 + 5.0 * dq2 + dt1 - du1 - 2.0 * dt2 - 4.0 * du2;
  g[4] = -dq2 + dt2 + du2;
  return y;
}

template <int D>
MMD void a_hj(const Params& P, const Bufs& B, const Adj& A, int r, int i, int j, int dir,
              double vel, double lg) {
  if (lg == 0.0 || vel == 0.0) return;
  double ih = dir == 0 ? P.idx : P.idy;
  int kk[7];
  for (int q = 0; q < 7; q++) {
    int o = q - 3;
    kk[q] = dir == 0 ? cid(P, i + o, j) : cid(P, i, j + o);
  }
  // d[q] = (phi^r_{q-2} - phi^r_{q-3}) / h, q = 0..5 (cells kk[q+1], kk[q])
  double d[6];
  for (int q = 0; q < 6; q++)
    d[q] = (lsv(B.phi, B.chi, r, kk[q + 1]) - lsv(B.phi, B.chi, r, kk[q])) * ih;
  int map[5];
  if (vel > 0.0) {
    for (int q = 0; q < 5; q++) map[q] = q;
  } else {
    for (int q = 0; q < 5; q++) map[q] = 5 - q;
  }
  double gq[5];
  weno5_grad(d[map[0]], d[map[1]], d[map[2]], d[map[3]], d[map[4]], gq);
  for (int q = 0; q < 5; q++) {
    double ld = lg * gq[q] * ih;
    if (ld == 0.0) continue;
    int m = map[q];
    aadd(&A.lphi[kk[m + 1]], ld * lsgn(B.chi, r, kk[m + 1]));
    aadd(&A.lphi[kk[m]], -ld * lsgn(B.chi, r, kk[m]));
  }
}

// grid z = 0: the level-set stage; z = 1: the RK update of Q (independent:
// they share no adjoint); z = 2 (with tiles): the tile list of the stage's
// own level set for the ghost-extension adjoint (its counter was cleared
// before), over all workgroups of the slice
template <int D>
__global__ void __launch_bounds__(256) k_a_ls(Params P, Bufs B, Adj A, double bcoef, double ccoef,
                                              int sidx) {
  if (blockIdx.z == 2) {
    int nb = gridDim.x * gridDim.y, tid = threadIdx.y * blockDim.x + threadIdx.x;
    int nt = tiles_x(P) * ((P.ny + tile_h(P) - 1) / tile_h(P));
    for (int t = blockIdx.y * gridDim.x + blockIdx.x; t < nt; t += nb)
      tile_flag(P, B, sidx, sidx, t, tid, blockDim.x * blockDim.y);
    return;
  }
  ADJ_CELL_LOOP
  if (blockIdx.z == 1) {
    a_update_cell(P, A, k, bcoef, ccoef);
    return;
  }
  double lp = A.lphis[k];
  if (B.dls[k] > 3) {
    aadd(&A.lphi[k], lp);
    return;
  }
  if (lp == 0.0) return;
  double dt = B.scal[S_DT];
  double best = 0.0, bgx = 0.0, bgy = 0.0;
  int br = -1;
  unsigned xs = B.xs[k];
  for (int r = 0; r < P.M; r++) {
    if (!((xs >> r) & 1)) continue;
    double gx = hj_deriv<D>(P, B, r, i, j, 0, B.vx[k]);
    double adv = B.vx[k] * gx;
    double gy = 0.0;
    if (D == 2) {
      gy = hj_deriv<D>(P, B, r, i, j, 1, B.vy[k]);
      adv = adv + B.vy[k] * gy;
    }
    double val = lsv(B.phi, B.chi, r, k) - dt * adv;
    double nv = bcoef * lsv(B.phin, B.chin, r, k) + ccoef * val;
    if (br < 0 || nv > best) {
      best = nv;
      br = r;
      bgx = gx;
      bgy = gy;
    }
  }
  if (br < 0) return;
  double a = fabs(best);
  if (!(a < P.bls)) return;  // clamped to the band width
  double lb = best < 0.0 ? -lp : lp;
  aadd(&A.lphin[k], bcoef * lb * lsgn(B.chin, br, k));
  double lval = ccoef * lb;
  aadd(&A.lphi[k], lval * lsgn(B.chi, br, k));
  double ladv = -dt * lval;
  A.lvx[k] += ladv * bgx;
  a_hj<D>(P, B, A, br, i, j, 0, B.vx[k], ladv * B.vx[k]);
  if (D == 2) {
    A.lvy[k] += ladv * bgy;
    a_hj<D>(P, B, A, br, i, j, 1, B.vy[k], ladv * B.vy[k]);
  }
}


// ---------------------------------------------------------------------------
// Aperture-weighted face fluxes (Eq. discretized_equ).  One thread per face
// of direction dir: x-faces i+1/2 (i in [-1, nx)), y-faces j+1/2 (j in
// [-1, ny)).  In: ccoef * lQs of the two cells; out: A.lW (stencil, atomics),
// A.lax / A.lay (the face's stored aperture).
// ---------------------------------------------------------------------------
template <int D>
MMD void a_face(const Params& P, const Bufs& B, const Adj& A, const double* Q,
                const uint8_t* occ, int r, int i, int j, int dir, const double lF[4],
                double& lAF) {
  Prim Wc[6];
  bool vc[6];
  int kc[6];
  bool ok = true;
  for (int q = 0; q < 6; q++) {
    int ii = dir == 0 ? i - 2 + q : i, jj = dir == 0 ? j : j - 2 + q;
    kc[q] = cid(P, ii, jj);
    Wc[q] = Wget<D>(P, B, Q, occ, r, ii, jj, vc[q]);
    if (!vc[q]) ok = false;
  }
  lAF = 0.0;
  if (!vc[2] || !vc[3]) return;  // no flux was taken
  double pinf = P.pinf[r];
  // component c of a state in face coordinates: rho, normal, tangential, p
  auto comp = [&](const Prim& w, int c) -> double {
    return c == 0 ? w.r : (c == 1 ? (dir == 0 ? w.u : w.v) : (c == 2 ? (dir == 0 ? w.v : w.u) : w.p));
  };
  double L[4], R[4];
  if (ok) {
    for (int c = 0; c < 4; c++) {
      if (D == 1 && c == 2) {
        L[c] = R[c] = 0.0;
        continue;
      }
      L[c] = weno5(comp(Wc[0], c), comp(Wc[1], c), comp(Wc[2], c), comp(Wc[3], c), comp(Wc[4], c));
      R[c] = weno5(comp(Wc[5], c), comp(Wc[4], c), comp(Wc[3], c), comp(Wc[2], c), comp(Wc[1], c));
    }
    if (!(L[0] > 0.0) || !(R[0] > 0.0) || !(L[3] + pinf > 0.0) || !(R[3] + pinf > 0.0)) ok = false;
  }
  if (!ok) {
    for (int c = 0; c < 4; c++) {
      L[c] = comp(Wc[2], c);
      R[c] = comp(Wc[3], c);
    }
  }
  // HLLC Jacobian over (L, R)
  PrimT<Dn<8>> DL, DR;
  DL.r = dn_seed<8>(L[0], 0);
  DL.u = dn_seed<8>(L[1], 1);
  DL.v = dn_seed<8>(L[2], 2);
  DL.p = dn_seed<8>(L[3], 3);
  DR.r = dn_seed<8>(R[0], 4);
  DR.u = dn_seed<8>(R[1], 5);
  DR.v = dn_seed<8>(R[2], 6);
  DR.p = dn_seed<8>(R[3], 7);
  Dn<8> G[4];
  hllc_flux(DL, DR, eos_of(P, r), P.igm1[r], G);
  // face flux F in grid order from G in face order
  double Fv[4] = {G[0].v, dir == 0 ? G[1].v : G[2].v, dir == 0 ? G[2].v : G[1].v, G[3].v};
  for (int v = 0; v < 4; v++) lAF += Fv[v] * lF[v];  // (times A applied by the caller)
  double lG[4] = {lF[0], dir == 0 ? lF[1] : lF[2], dir == 0 ? lF[2] : lF[1], lF[3]};
  double lLR[8];
  for (int q = 0; q < 8; q++) {
    double s = 0.0;
    for (int m = 0; m < 4; m++) s += lG[m] * G[m].d[q];
    lLR[q] = s;
  }
  // back to the stencil states
  double lWc[6][4];
  for (int q = 0; q < 6; q++)
    for (int c = 0; c < 4; c++) lWc[q][c] = 0.0;
  for (int c = 0; c < 4; c++) {
    if (D == 1 && c == 2) continue;
    double lL = lLR[c], lR = lLR[4 + c];
    if (ok) {
      double gq[5];
      weno5_grad(comp(Wc[0], c), comp(Wc[1], c), comp(Wc[2], c), comp(Wc[3], c), comp(Wc[4], c),
                 gq);
      for (int q = 0; q < 5; q++) lWc[q][c] += lL * gq[q];
      weno5_grad(comp(Wc[5], c), comp(Wc[4], c), comp(Wc[3], c), comp(Wc[2], c), comp(Wc[1], c),
                 gq);
      for (int q = 0; q < 5; q++) lWc[5 - q][c] += lR * gq[q];
    } else {
      lWc[2][c] += lL;
      lWc[3][c] += lR;
    }
  }
  for (int q = 0; q < 6; q++) {
    // face components back to (rho, u, v, p)
    double lw[4] = {lWc[q][0], dir == 0 ? lWc[q][1] : lWc[q][2],
                    dir == 0 ? lWc[q][2] : lWc[q][1], lWc[q][3]};
    for (int c = 0; c < 4; c++) aadd(&A4(P, A.lW, r, c, kc[q]), lw[c]);
  }
}

// own-material velocity of the remaining band cells (stage 0), reversed
template <int D>
MMD void a_vfill_cell(const Params& P, const Bufs& B, const Adj& A, int sidx, int i, int j) {
  int k = cid(P, i, j);
  if (B.dls[k] > RV || B.vit[k] != 0) return;
  double lx = A.lvx[k], ly = A.lvy[k];
  A.lvx[k] = 0.0;
  A.lvy[k] = 0.0;
  if (lx == 0.0 && ly == 0.0) return;
  bool valid;
  int r = B.chi[k];
  Wget<D>(P, B, B.Q[sidx], B.occ[sidx], r, i, j, valid);
  if (!valid) return;
  aadd(&A4(P, A.lW, r, 1, k), lx);
  if (D == 2) aadd(&A4(P, A.lW, r, 2, k), ly);
}

template <int D>
// x-faces (threads t < nx0 faces) and, in 2D, the y-faces after them, in one
// launch: twice the faces in flight; workgroups from nfb on (stage 0) reverse
// the velocity fill, one thread per cell (it shares no adjoint with the
// fluxes but the state adjoints, which both add to with atomics)
__global__ void __launch_bounds__(256) k_a_flux(Params P, Bufs B, Adj A, int sidx, double ccoef,
                                                int nfb) {
  if ((int)blockIdx.x >= nfb) {
    int q = ((int)blockIdx.x - nfb) * blockDim.x + threadIdx.x;
    if (q < P.nx * P.ny) a_vfill_cell<D>(P, B, A, sidx, q % P.nx, q / P.nx);
    return;
  }
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int n0 = (P.nx + 1) * P.ny;
  int dir = t < n0 ? 0 : 1;
  if (D == 1 && dir == 1) return;
  if (dir == 1) t -= n0;
  int nfx = dir == 0 ? P.nx + 1 : P.nx, nfy = dir == 0 ? P.ny : P.ny + 1;
  if (t >= nfx * nfy) return;
  int i = t % nfx, j = t / nfx;
  if (dir == 0) i -= 1;
  else j -= 1;
  int kL = cid(P, i, j), kR = dir == 0 ? cid(P, i + 1, j) : cid(P, i, j + 1);
  bool inL = interior(P, i, j), inR = dir == 0 ? interior(P, i + 1, j) : interior(P, i, j + 1);
  double l = dir == 0 ? B.scal[S_LX] : B.scal[S_LY];
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  for (int r = 0; r < P.M; r++) {
    double Af = dir == 0 ? apx<D>(P, B, r, i, j) : apy(P, B, r, i, j);
    if (!(Af > 0.0)) continue;
    double lAFv[4], lF[4];
    bool any = false;
    for (int v = 0; v < 4; v++) {
      double lr = inR ? ccoef * A4(P, A.lQs, r, v, kR) : 0.0;
      double ll = inL ? ccoef * A4(P, A.lQs, r, v, kL) : 0.0;
      lAFv[v] = l * (lr - ll);
      lF[v] = Af * lAFv[v];
      if (lAFv[v] != 0.0) any = true;
    }
    if (!any) continue;
    double lA;
    a_face<D>(P, B, A, Q, occ, r, i, j, dir, lF, lA);
    // lA = sum F lF = A * sum F lAF: the aperture adjoint is sum F lAF
    double lAp = lA / Af;
    // the stored aperture is used only where apx/apy read it
    bool stored;
    if (dir == 0) {
      if (i < 0) stored = B.cut[kR];
      else if (i >= P.nx - 1) stored = B.cut[kL];
      else stored = B.cut[kL] && B.cut[kR];
      if (stored) A1(P, A.lax, r, kL) += lAp;
    } else {
      if (j < 0) stored = B.cut[kR];
      else if (j >= P.ny - 1) stored = B.cut[kL];
      else stored = B.cut[kL] && B.cut[kR];
      if (stored) A1(P, A.lay, r, kL) += lAp;
    }
  }
}

// ---------------------------------------------------------------------------
// Level-set velocity v^n (stage 0): own-material velocity in the remaining
// band cells, then the extension sweeps in reverse.
// ---------------------------------------------------------------------------

template <int D>
__global__ void __launch_bounds__(256) k_a_vext(Params P, Bufs B, Adj A, int sweep) {
  ADJ_CELL_LOOP
  if (B.vit[k] != sweep + 2) return;
  double lox = A.lvx[k], loy = A.lvy[k];
  A.lvx[k] = 0.0;
  A.lvy[k] = 0.0;
  if (lox == 0.0 && loy == 0.0) return;
  auto valid_prev = [&](int ii, int jj) -> bool {
    if (!interior(P, ii, jj)) return false;
    uint8_t it = B.vit[cid(P, ii, jj)];
    return it != 0 && it <= sweep + 1;
  };
  int kxp = cid(P, i + 1, j), kxm = cid(P, i - 1, j);
  double gx = B.phi[kxp] - B.phi[kxm];
  double gy = 0.0;
  int kyp = k, kym = k;
  if (D == 2) {
    kyp = cid(P, i, j + 1);
    kym = cid(P, i, j - 1);
    gy = B.phi[kyp] - B.phi[kym];
  }
  int kx = -1, ky = -1;
  if (gx != 0.0) {
    int ii = i - (gx > 0.0 ? 1 : -1);
    if (valid_prev(ii, j)) kx = cid(P, ii, j);
  }
  if (gy != 0.0) {
    int jj = j - (gy > 0.0 ? 1 : -1);
    if (valid_prev(i, jj)) ky = cid(P, i, jj);
  }
  if (kx >= 0 && ky >= 0) {
    double wx = fabs(gx), wy = fabs(gy), ws = wx + wy;
    double ox = (wx * B.vx[kx] + wy * B.vx[ky]) / ws;
    double oy = (wx * B.vy[kx] + wy * B.vy[ky]) / ws;
    aadd(&A.lvx[kx], lox * wx / ws);
    aadd(&A.lvx[ky], lox * wy / ws);
    aadd(&A.lvy[kx], loy * wx / ws);
    aadd(&A.lvy[ky], loy * wy / ws);
    double lwx = (lox * (B.vx[kx] - ox) + loy * (B.vy[kx] - oy)) / ws;
    double lwy = (lox * (B.vx[ky] - ox) + loy * (B.vy[ky] - oy)) / ws;
    double lgx = gx < 0.0 ? -lwx : lwx, lgy = gy < 0.0 ? -lwy : lwy;
    aadd(&A.lphi[kxp], lgx);
    aadd(&A.lphi[kxm], -lgx);
    aadd(&A.lphi[kyp], lgy);
    aadd(&A.lphi[kym], -lgy);
  } else if (kx >= 0 || ky >= 0) {
    int ks = kx >= 0 ? kx : ky;
    aadd(&A.lvx[ks], lox);
    aadd(&A.lvy[ks], loy);
  }
}

// ---------------------------------------------------------------------------
// Reduced interface exchange (Sec. 2.3.2) in cut cells; at stage 0 also the
// interface velocity S_M n.  Out: A.lW of the pair, A.lcx / A.lcy of a.
// ---------------------------------------------------------------------------
// both sides at once (2D), frame cell t: x-side frame cells of rows [0, ny) as in
// the x pass; a y-side frame cell takes its side's map (inflow, or the
// source row with the normal velocity negated at a reflective side), and
// where that source is an x-side frame cell (a corner), the x side's map on
// top: the sum the two passes in sequence deliver
MMD void a_bc_W_to(const Params& P, const Adj& A, int r, int side_type, int ks, int flip,
                   double sgn, const double l[4]) {
  if (side_type == 2 && r == P.inflow_mat) {
    for (int v = 0; v < 4; v++) aadd(&A.linflow[v], l[v]);
    return;
  }
  for (int v = 0; v < 4; v++) aadd(&A4(P, A.lW, r, v, ks), v == flip ? l[v] * sgn : l[v]);
}
MMD void a_bc_W2_cell(const Params& P, const Adj& A, int t) {
  int nxs = P.ny * 2 * H, nys = (P.nx + 2 * H) * 2 * H;
  if (t >= (nxs + nys) * P.M) return;
  int r, i, j, ytype = -1, sj = 0;
  if (t < nxs * P.M) {
    r = t / nxs;
    int rem = t % nxs, q = rem % (2 * H);
    j = rem / (2 * H);
    i = q < H ? -1 - q : P.nx + (q - H);
  } else {
    t -= nxs * P.M;
    r = t / nys;
    int rem = t % nys, q = rem % (2 * H);
    i = rem / (2 * H) - H;
    j = q < H ? -1 - q : P.ny + (q - H);
    ytype = q < H ? P.bc[2] : P.bc[3];
    sj = q < H ? src_lo(j, ytype) : src_hi(j, P.ny, ytype);
  }
  int k = cid(P, i, j);
  double l[4];
  for (int v = 0; v < 4; v++) {
    l[v] = A4(P, A.lW, r, v, k);
    A4(P, A.lW, r, v, k) = 0.0;
  }
  if (ytype >= 0) {
    if (ytype == 2 && r == P.inflow_mat) {
      for (int v = 0; v < 4; v++) aadd(&A.linflow[v], l[v]);
      return;
    }
    l[2] = l[2] * (ytype == 1 ? -1.0 : 1.0);
    if (i >= 0 && i < P.nx) {
      a_bc_W_to(P, A, r, -1, cid(P, i, sj), -1, 1.0, l);
      return;
    }
    j = sj;  // corner: on to the x side's source of row sj
  }
  int xtype = i < 0 ? P.bc[0] : P.bc[1];
  int si = i < 0 ? src_lo(i, xtype) : src_hi(i, P.nx, xtype);
  a_bc_W_to(P, A, r, xtype, cid(P, si, j), 1, xtype == 1 ? -1.0 : 1.0, l);
}

// grid z = 1 (2D): the frames of the primitive states, one thread per frame
// cell and material over all workgroups of the slice; the exchange adds to
// the state adjoints of cut cells with atomics, as the frames do to the cells
// next to the boundary
template <int D>
__global__ void __launch_bounds__(256) k_a_iface(Params P, Bufs B, Adj A, int sidx, double ccoef, int stage0) {
  if (blockIdx.z == 1) {
    int nb = gridDim.x * gridDim.y, nt = blockDim.x * blockDim.y;
    int nfr = (P.ny + P.nx + 2 * H) * 2 * H * P.M;
    for (int t = (blockIdx.y * gridDim.x + blockIdx.x) * nt + threadIdx.y * blockDim.x + threadIdx.x;
         t < nfr; t += nb * nt)
      a_bc_W2_cell(P, A, t);
    return;
  }
  ADJ_CELL_LOOP
  if (!B.cut[k]) return;
  unsigned b = B.xs[k];
  if ((b & (b - 1)) == 0) return;
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  int a = -1, bb = -1;
  for (int r = 0; r < P.M; r++) {
    if (!((b >> r) & 1)) continue;
    if (a < 0 || loadQ<D>(P, Q, occ, r, 0, k) > loadQ<D>(P, Q, occ, a, 0, k)) a = r;
  }
  for (int r = 0; r < P.M; r++) {
    if (!((b >> r) & 1) || r == a) continue;
    if (bb < 0 || loadQ<D>(P, Q, occ, r, 0, k) > loadQ<D>(P, Q, occ, bb, 0, k)) bb = r;
  }
  double cxa = B.cx[(size_t)a * P.NC + k], cya = B.cy[(size_t)a * P.NC + k];
  if (cxa == 0.0 && cya == 0.0) return;
  bool va, vb;
  Prim Wa = Wget<D>(P, B, Q, occ, a, i, j, va);
  Prim Wb = Wget<D>(P, B, Q, occ, bb, i, j, vb);
  if (!va || !vb) return;
  double lv = B.scal[S_LV];
  double lX[4];
  for (int v = 1; v < 4; v++)
    lX[v] = lv * ccoef * (A4(P, A.lQs, a, v, k) - A4(P, A.lQs, bb, v, k));
  double lvx = 0.0, lvy = 0.0;
  if (stage0 && B.vit[k] == 1) {
    lvx = A.lvx[k];
    lvy = A.lvy[k];
    A.lvx[k] = 0.0;
    A.lvy[k] = 0.0;
  }
  if (lX[1] == 0.0 && lX[2] == 0.0 && lX[3] == 0.0 && lvx == 0.0 && lvy == 0.0) return;
  typedef Dn<10> T;
  PrimT<T> Db, Da;
  Db.r = dn_seed<10>(Wb.r, 0);
  Db.u = dn_seed<10>(Wb.u, 1);
  Db.v = dn_seed<10>(Wb.v, 2);
  Db.p = dn_seed<10>(Wb.p, 3);
  Da.r = dn_seed<10>(Wa.r, 4);
  Da.u = dn_seed<10>(Wa.u, 5);
  Da.v = dn_seed<10>(Wa.v, 6);
  Da.p = dn_seed<10>(Wa.p, 7);
  T cx = dn_seed<10>(cxa, 8), cy = dn_seed<10>(cya, 9);
  T nrm = sqrt(cx * cx + cy * cy);
  T nxv = cx / nrm, nyv = cy / nrm;
  PrimT<T> L, R;
  L.r = Db.r;
  L.u = Db.u * nxv + Db.v * nyv;
  L.v = T(0.0);
  L.p = Db.p;
  R.r = Da.r;
  R.u = Da.u * nxv + Da.v * nyv;
  R.v = T(0.0);
  R.p = Da.p;
  T SL, SR;
  wave_speeds(L, eos_of(P, bb), R, eos_of(P, a), SL, SR);
  T SM = contact_speed(L, R, SL, SR);
  T ps = 0.5 * ((L.p + L.r * (SL - L.u) * (SM - L.u)) + (R.p + R.r * (SR - R.u) * (SM - R.u)));
  T X1 = ps * cx, X2 = ps * cy, X3 = ps * SM * nrm;
  T ovx = SM * nxv, ovy = SM * nyv;
  double g[10];
  for (int q = 0; q < 10; q++)
    g[q] = lX[1] * X1.d[q] + lX[2] * X2.d[q] + lX[3] * X3.d[q] + lvx * ovx.d[q] + lvy * ovy.d[q];
  for (int c = 0; c < 4; c++) {
    if (D == 1 && c == 2) continue;
    aadd(&A4(P, A.lW, bb, c, k), g[c]);
    aadd(&A4(P, A.lW, a, c, k), g[4 + c]);
  }
  A1(P, A.lcx, a, k) += g[8];
  if (D == 2) A1(P, A.lcy, a, k) += g[9];
}

// ---------------------------------------------------------------------------
// Frames of the primitive states: a frame state is a copy (normal velocity
// negated at a reflective side) of a state next to the boundary, or the
// fixed inflow state.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_a_bc_W_x(Params P, Bufs B, Adj A) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.ny * 2 * H * P.M) return;
  int r = t / (P.ny * 2 * H);
  int rem = t % (P.ny * 2 * H);
  int j = rem / (2 * H), q = rem % (2 * H);
  int ii, si, type;
  if (q < H) {
    ii = -1 - q;
    type = P.bc[0];
    si = src_lo(ii, type);
  } else {
    ii = P.nx + (q - H);
    type = P.bc[1];
    si = src_hi(ii, P.nx, type);
  }
  int k = cid(P, ii, j), ks = cid(P, si, j);
  double l[4];
  for (int v = 0; v < 4; v++) {
    l[v] = A4(P, A.lW, r, v, k);
    A4(P, A.lW, r, v, k) = 0.0;
  }
  if (type == 2 && r == P.inflow_mat) {
    for (int v = 0; v < 4; v++) aadd(&A.linflow[v], l[v]);
    return;
  }
  double sx = type == 1 ? -1.0 : 1.0;
  aadd(&A4(P, A.lW, r, 0, ks), l[0]);
  aadd(&A4(P, A.lW, r, 1, ks), l[1] * sx);
  aadd(&A4(P, A.lW, r, 2, ks), l[2]);
  aadd(&A4(P, A.lW, r, 3, ks), l[3]);
}


// ---------------------------------------------------------------------------
// Ghost extension: the (cell, material) pairs filled in sweep `sweep` pass
// their adjoint to the states they were built from (and, for the upwind
// sweeps, to the level set through the weights).  Pairs come from the ghost
// queue of the recomputed stage.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_a_ext(Params P, Bufs B, Adj A, int sidx, int sweep) {
  unsigned long long n = B.ctr[C_NGHOST];
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  for (unsigned long long e = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (unsigned long long)gridDim.x * blockDim.x) {
    int code = B.glist[e];
    int k = code >> 3, r = code & 7;
    if (B.Wit[(size_t)r * P.NC + k] != sweep + 2) continue;
    double lo[4];
    bool any = false;
    for (int c = 0; c < 4; c++) {
      lo[c] = A4(P, A.lW, r, c, k);
      A4(P, A.lW, r, c, k) = 0.0;
      if (lo[c] != 0.0) any = true;
    }
    if (!any) continue;
    int i = k % P.NX - H, j = k / P.NX - P.HY;
    auto valid_prev = [&](int ii, int jj) -> bool {
      if (!interior(P, ii, jj)) return false;
      int kk = cid(P, ii, jj);
      if (B.dcut[kk] > 7) return B.chi[kk] == r;
      uint8_t it = B.Wit[(size_t)r * P.NC + kk];
      return it != 0 && it <= sweep + 1;
    };
    if (sweep < P.kext) {
      int kxp = cid(P, i + 1, j), kxm = cid(P, i - 1, j);
      double gx = lsv(B.phi, B.chi, r, kxp) - lsv(B.phi, B.chi, r, kxm);
      double gy = 0.0;
      int kyp = k, kym = k;
      if (D == 2) {
        kyp = cid(P, i, j + 1);
        kym = cid(P, i, j - 1);
        gy = lsv(B.phi, B.chi, r, kyp) - lsv(B.phi, B.chi, r, kym);
      }
      int xi = -1, yj = -1;
      bool hx = false, hy = false;
      if (gx != 0.0) {
        xi = i + (gx > 0.0 ? 1 : -1);
        hx = valid_prev(xi, j);
      }
      if (gy != 0.0) {
        yj = j + (gy > 0.0 ? 1 : -1);
        hy = valid_prev(i, yj);
      }
      bool vd;
      if (hx && hy) {
        int ka = cid(P, xi, j), kb = cid(P, i, yj);
        Prim a = Wget<D>(P, B, Q, occ, r, xi, j, vd);
        Prim b = Wget<D>(P, B, Q, occ, r, i, yj, vd);
        double wx = fabs(gx), wy = fabs(gy), ws = wx + wy;
        double av[4] = {a.r, a.u, a.v, a.p}, bv[4] = {b.r, b.u, b.v, b.p};
        double lwx = 0.0, lwy = 0.0;
        for (int c = 0; c < 4; c++) {
          double out = (wx * av[c] + wy * bv[c]) / ws;
          aadd(&A4(P, A.lW, r, c, ka), lo[c] * wx / ws);
          aadd(&A4(P, A.lW, r, c, kb), lo[c] * wy / ws);
          lwx += lo[c] * (av[c] - out) / ws;
          lwy += lo[c] * (bv[c] - out) / ws;
        }
        double lgx = gx < 0.0 ? -lwx : lwx, lgy = gy < 0.0 ? -lwy : lwy;
        aadd(&A.lphi[kxp], lgx * lsgn(B.chi, r, kxp));
        aadd(&A.lphi[kxm], -lgx * lsgn(B.chi, r, kxm));
        aadd(&A.lphi[kyp], lgy * lsgn(B.chi, r, kyp));
        aadd(&A.lphi[kym], -lgy * lsgn(B.chi, r, kym));
      } else if (hx || hy) {
        int ks = hx ? cid(P, xi, j) : cid(P, i, yj);
        for (int c = 0; c < 4; c++) aadd(&A4(P, A.lW, r, c, ks), lo[c]);
      }
    } else {
      int cnt = 0;
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++)
          if ((di != 0 || dj != 0) && (D == 2 || dj == 0) && valid_prev(i + di, j + dj)) cnt++;
      if (cnt == 0) continue;
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++)
          if ((di != 0 || dj != 0) && (D == 2 || dj == 0) && valid_prev(i + di, j + dj)) {
            int ks = cid(P, i + di, j + dj);
            for (int c = 0; c < 4; c++) aadd(&A4(P, A.lW, r, c, ks), lo[c] / (double)cnt);
          }
    }
  }
}

// The ghost-state sweeps in reverse, tile-wise (2D): one workgroup per
// active tile and material loads the forward states, stamps and adjoints of
// the tile and its 12-cell frame, runs the reverse sweeps in LDS (a pair's
// adjoint goes to the neighbours it was computed from, as in k_a_ext) and
// writes the tile's own adjoints to lW2; the level-set adjoint of the tile's
// own pairs goes to lphi.  Adjoints reach a tile cell from at most 12 cells
// away, so the tile's values are complete.  lW is only read (other
// workgroups read it for their frames).
struct AExtSmem {
  double W[4][EXW * EXW];
  double L[4][EXW * EXW];  // adjoints of the states
  double lphi[EXG * EXG];
  uint8_t st[EXW * EXW];
  uint16_t list[EXW * EXW];
  int nlist;
};
__global__ void __launch_bounds__(256) k_a_ext_tiles(Params P, Bufs B, Adj A, int sidx) {
  __shared__ AExtSmem S;
  const int r = blockIdx.y, tid = threadIdx.x, ntx = tiles_x(P);
  const int ntile = (int)B.ctr[C_NTILES], nsw = P.kext + 4;
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  constexpr int NQ = (EXW * EXW + 255) / 256, NG = (EXG * EXG + 255) / 256;
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    int tile = B.tiles[t];
    int ti0 = (tile % ntx) * EXT, tj0 = (tile / ntx) * EXT;
    int x0 = ti0 - EXR, y0 = tj0 - EXR;
    if (tid == 0) S.nlist = 0;
    __syncthreads();
    int kq[NQ];
    uint8_t dcq[NQ], chq[NQ], itq[NQ], ocq[NQ];
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int q = tid + n * 256;
      int ci = x0 + q % EXW, cj = y0 + q / EXW;
      bool in = q < EXW * EXW && interior(P, ci, cj);
      int k = in ? cid(P, ci, cj) : -1, ks = in ? k : cid(P, 0, 0);
      kq[n] = k;
      uint8_t a0 = B.dcut[ks], a1 = B.chi[ks], a2 = B.Wit[(size_t)r * P.NC + ks], a5 = occ[ks];
      dcq[n] = in ? a0 : 0;
      chq[n] = in ? a1 : 0;
      itq[n] = in ? a2 : 0;
      ocq[n] = in ? a5 : 0;
    }
    double U[NQ][4], Lq[NQ][4];
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int k = kq[n];
      bool far = dcq[n] > 7 && chq[n] == r;
      bool need = k >= 0 && (far || (dcq[n] <= 7 && itq[n] != 0));
      const double* base = far ? Q : B.W;
      size_t o = (size_t)r * 4 * P.NC + (k >= 0 ? k : cid(P, 0, 0));
      for (int c = 0; c < 4; c++) {
        double u = base[o + (size_t)c * P.NC], l = A.lW[o + (size_t)c * P.NC];
        U[n][c] = need ? u : 0.0;
        Lq[n][c] = k >= 0 ? l : 0.0;
      }
    }
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int q = tid + n * 256;
      if (q >= EXW * EXW) continue;
      int k = kq[n];
      uint8_t st = 0;
      double w[4] = {0.0, 0.0, 0.0, 0.0};
      if (k >= 0) {
        if (dcq[n] > 7) {
          if (chq[n] == r) {
            st = 1;
            bool has = (ocq[n] >> r) & 1;
            double U0 = has ? U[n][0] / 1.0 : 0.0, U1 = has ? U[n][1] / 1.0 : 0.0,
                   U2 = has ? U[n][2] / 1.0 : 0.0, U3 = has ? U[n][3] / 1.0 : 0.0;
            Prim pw = prim_from_U(U0, U1, U2, U3, eos_of(P, r));
            w[0] = pw.r; w[1] = pw.u; w[2] = pw.v; w[3] = pw.p;
          }
        } else {
          st = itq[n];
          if (st)
            for (int c = 0; c < 4; c++) w[c] = U[n][c];
          // a pair that got its state in a sweep (stamps 0/1 are no state / real)
          if (dcq[n] <= 4 && st >= 2) S.list[atomicAdd(&S.nlist, 1)] = (uint16_t)q;
        }
      }
      S.st[q] = st;
      for (int c = 0; c < 4; c++) {
        S.W[c][q] = w[c];
        S.L[c][q] = Lq[n][c];
      }
    }
    double ph[NG];
    uint8_t pc[NG];
#pragma unroll
    for (int n = 0; n < NG; n++) {
      int q = tid + n * 256;
      int ci = x0 - 1 + q % EXG, cj = y0 - 1 + q / EXG;
      bool in = q < EXG * EXG && ci >= -H && ci < P.nx + H && cj >= -H && cj < P.ny + H;
      int k = in ? cid(P, ci, cj) : cid(P, 0, 0);
      double a = B.phi[k];
      uint8_t b = B.chi[k];
      ph[n] = in ? a : 0.0;
      pc[n] = in ? b : (uint8_t)r;
    }
#pragma unroll
    for (int n = 0; n < NG; n++) {
      int q = tid + n * 256;
      if (q < EXG * EXG) S.lphi[q] = pc[n] == r ? ph[n] : -ph[n];
    }
    __syncthreads();
    const int nl = S.nlist;
    if (nl > 0) {
      auto valid = [&](int lx, int ly, int ci, int cj, int s) -> bool {
        if (lx < 0 || lx >= EXW || ly < 0 || ly >= EXW || !interior(P, ci, cj)) return false;
        int it = S.st[ly * EXW + lx];
        return it != 0 && it <= s + 1;
      };
      for (int s = nsw - 1; s >= 0; s--) {
        for (int e = tid; e < nl; e += 256) {
          int q = S.list[e];
          if (S.st[q] != s + 2) continue;
          double lo[4];
          bool any = false;
          for (int c = 0; c < 4; c++) {
            lo[c] = S.L[c][q];
            S.L[c][q] = 0.0;
            if (lo[c] != 0.0) any = true;
          }
          if (!any) continue;
          int lx = q % EXW, ly = q / EXW, ci = x0 + lx, cj = y0 + ly;
          bool own = lx >= EXR && lx < EXR + EXT && ly >= EXR && ly < EXR + EXT;
          if (s < P.kext) {
            int g = (ly + 1) * EXG + lx + 1;
            double gx = S.lphi[g + 1] - S.lphi[g - 1];
            double gy = S.lphi[g + EXG] - S.lphi[g - EXG];
            int sx = 0, sy = 0;
            bool hx = false, hy = false;
            if (gx != 0.0) {
              sx = gx > 0.0 ? 1 : -1;
              hx = valid(lx + sx, ly, ci + sx, cj, s);
            }
            if (gy != 0.0) {
              sy = gy > 0.0 ? 1 : -1;
              hy = valid(lx, ly + sy, ci, cj + sy, s);
            }
            if (hx && hy) {
              int a = ly * EXW + lx + sx, b = (ly + sy) * EXW + lx;
              double wx = fabs(gx), wy = fabs(gy), ws = wx + wy;
              double lwx = 0.0, lwy = 0.0;
              for (int c = 0; c < 4; c++) {
                double av = S.W[c][a], bv = S.W[c][b];
                double out = (wx * av + wy * bv) / ws;
                atomicAdd(&S.L[c][a], lo[c] * wx / ws);
                atomicAdd(&S.L[c][b], lo[c] * wy / ws);
                lwx += lo[c] * (av - out) / ws;
                lwy += lo[c] * (bv - out) / ws;
              }
              if (own) {
                int kc = cid(P, ci, cj);
                int kxp = kc + 1, kxm = kc - 1, kyp = kc + P.NX, kym = kc - P.NX;
                double lgx = gx < 0.0 ? -lwx : lwx, lgy = gy < 0.0 ? -lwy : lwy;
                aadd(&A.lphi[kxp], lgx * lsgn(B.chi, r, kxp));
                aadd(&A.lphi[kxm], -lgx * lsgn(B.chi, r, kxm));
                aadd(&A.lphi[kyp], lgy * lsgn(B.chi, r, kyp));
                aadd(&A.lphi[kym], -lgy * lsgn(B.chi, r, kym));
              }
            } else if (hx || hy) {
              int a = hx ? ly * EXW + lx + sx : (ly + sy) * EXW + lx;
              for (int c = 0; c < 4; c++) atomicAdd(&S.L[c][a], lo[c]);
            }
          } else {
            int cnt = 0;
            for (int dj = -1; dj <= 1; dj++)
              for (int di = -1; di <= 1; di++)
                if ((di != 0 || dj != 0) && valid(lx + di, ly + dj, ci + di, cj + dj, s)) cnt++;
            if (cnt == 0) continue;
            for (int dj = -1; dj <= 1; dj++)
              for (int di = -1; di <= 1; di++)
                if ((di != 0 || dj != 0) && valid(lx + di, ly + dj, ci + di, cj + dj, s)) {
                  int a = (ly + dj) * EXW + lx + di;
                  for (int c = 0; c < 4; c++) atomicAdd(&S.L[c][a], lo[c] / (double)cnt);
                }
          }
        }
        __syncthreads();
      }
    }
    // the tile's own adjoints (unchanged ones included) to the output buffer
    {
      int lx = EXR + tid % EXT, ly = EXR + tid / EXT, i = x0 + lx, j = y0 + ly;
      int q = ly * EXW + lx;
      if (i < P.nx && j < P.ny) {
        size_t o = (size_t)r * 4 * P.NC + cid(P, i, j);
        for (int c = 0; c < 4; c++) A.lW2[o + (size_t)c * P.NC] = S.L[c][q];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Real states W = prim(Q / alpha): to Q^(s) and, in cut cells, to alpha.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_a_real(Params P, Bufs B, Adj A, int sidx) {
  ADJ_CELL_LOOP
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  for (int r = blockIdx.z; r == (int)blockIdx.z; r++) {  // one material per grid slice z
    bool real = (B.dcut[k] > 7 && B.chi[k] == r) || B.Wit[(size_t)r * P.NC + k] == 1;
    if (!real) continue;
    double lw[4];
    bool any = false;
    for (int c = 0; c < 4; c++) {
      lw[c] = A4(P, A.lW, r, c, k);
      if (lw[c] != 0.0) any = true;
    }
    if (!any) continue;
    double a = B.cut[k] ? B.al[(size_t)r * P.NC + k] : 1.0;
    double Qv[4], U[4];
    for (int v = 0; v < 4; v++) {
      Qv[v] = loadQ<D>(P, Q, occ, r, v, k);
      U[v] = Qv[v] / a;
    }
    Dn<4> u0 = dn_seed<4>(U[0], 0), u1 = dn_seed<4>(U[1], 1), u2 = dn_seed<4>(U[2], 2),
          u3 = dn_seed<4>(U[3], 3);
    PrimT<Dn<4>> w = prim_from_U(u0, u1, u2, u3, eos_of(P, r));
    double lU[4];
    for (int q = 0; q < 4; q++)
      lU[q] = lw[0] * w.r.d[q] + lw[1] * w.u.d[q] + (D == 2 ? lw[2] * w.v.d[q] : 0.0) +
              lw[3] * w.p.d[q];
    double la = 0.0;
    for (int v = 0; v < 4; v++) {
      if (D == 1 && v == 2) continue;
      A4(P, A.lQ, r, v, k) += lU[v] / a;
      la += -lU[v] * U[v] / a;
    }
    if (B.cut[k]) A1(P, A.lal, r, k) += la;
  }
}

// ---------------------------------------------------------------------------
// Packing between the interior layout of the C ABI ([M][D+2][ny][nx],
// [ny][nx]) and the padded adjoint buffers.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_a_unpack(Params P, Adj A, const double* lQ, const double* lphi,
                           const double* lalpha) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  int k = cid(P, i, j);
  size_t plane = (size_t)P.nx * P.ny, q = (size_t)j * P.nx + i;
  // a NULL input keeps the adjoint carried from the previous reverse step
  for (int r = 0; r < P.M; r++) {
    if (lQ)
      for (int v = 0; v < 4; v++) {
        double x = 0.0;
        if (D == 2) x = lQ[((size_t)r * 4 + v) * plane + q];
        else if (v != 2) x = lQ[((size_t)r * 3 + (v == 3 ? 2 : v)) * plane + q];
        A4(P, A.lQ, r, v, k) = x;
      }
    A1(P, A.lalpha, r, k) = lalpha ? lalpha[(size_t)r * plane + q] : 0.0;
  }
  if (lphi) A.lphi[k] = lphi[q];
}
template <int D>
__global__ void __launch_bounds__(256) k_a_pack(Params P, Adj A, double* lQ, double* lphi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  int k = cid(P, i, j);
  size_t plane = (size_t)P.nx * P.ny, q = (size_t)j * P.nx + i;
  for (int r = 0; r < P.M; r++)
    for (int v = 0; v < 4; v++) {
      if (D == 2) lQ[((size_t)r * 4 + v) * plane + q] = A4(P, A.lQ, r, v, k);
      else if (v != 2) lQ[((size_t)r * 3 + (v == 3 ? 2 : v)) * plane + q] = A4(P, A.lQ, r, v, k);
    }
  if (lphi) lphi[q] = A.lphi[k];
}
// end of a step: the time-n adjoints collected from later stages join those
// of the stage-0 input
__global__ void __launch_bounds__(256) k_a_finish(Params P, Adj A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  int k = cid(P, i, j);
  for (int r = 0; r < P.M; r++)
    for (int v = 0; v < 4; v++) A4(P, A.lQ, r, v, k) += A4(P, A.lQn, r, v, k);
  A.lphi[k] += A.lphin[k];
}
// 2D: the level-set frame pass of the step's first stage (workgroups below
// nfrb) beside the finish (the others, one thread per cell; its level-set
// add is atomic, as the frame's adds to the cells next to the boundary)
__global__ void __launch_bounds__(256) k_a_bc_ls2_finish(Params P, Adj A, int nfrb) {
  if ((int)blockIdx.x < nfrb) {
    a_bc_ls2_cell(P, A.lphi, blockIdx.x * blockDim.x + threadIdx.x);
    return;
  }
  int q = ((int)blockIdx.x - nfrb) * blockDim.x + threadIdx.x;
  if (q >= P.nx * P.ny) return;
  int k = cid(P, q % P.nx, q / P.nx);
  for (int r = 0; r < P.M; r++)
    for (int v = 0; v < 4; v++) A4(P, A.lQ, r, v, k) += A4(P, A.lQn, r, v, k);
  aadd(&A.lphi[k], A.lphin[k]);
}

}  // namespace mmfv
