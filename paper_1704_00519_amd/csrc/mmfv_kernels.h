// HIP kernels of the cut-cell multi-material step for gfx950.
//
// Layout (HBM): every field is a padded Cartesian array of NC = NX*NY cells
// with a frame of H = 4 halo cells (none in y for 1D).  Conserved state is
// SoA [material][component][cell] with NV = dim+2 components; geometry is
// [material][cell]; primitive ghost/real states are [material][4][cell].
// A per-cell occupancy byte (bit r set = material r's slot may be non-zero)
// travels with each state buffer, so a cell away from interfaces only ever
// touches its own material's slot.
#pragma once
#include "mmfv_math.h"

namespace mmfv {

struct Bufs {
  double* Q[3];
  uint8_t* occ[3];
  double *phi, *ptmp, *phin;
  uint8_t *chi, *ctmp, *chin;
  double *al, *ax, *ay, *cx, *cy;
  double* W;
  uint8_t* Wit;
  uint8_t *cut, *xs, *dcut, *dls, *rowc, *rowl, *tdc, *tdl, *nrow, *near4, *bulk;
  double* X;
  double *vx, *vy;
  uint8_t* vit;
  double* mixM;
  int32_t* mixT;
  uint32_t *srcStamp, *tgtStamp;
  int32_t* tiles;          // active tiles of the current stage
  int32_t* blist;          // cells updated by the general (band) path
  int32_t* glist;          // (cell, material) pairs waiting for a ghost state
  uint16_t* vfc;           // per cut cell: volume-fraction correction taken
                           // (low byte: absorbing material or 0xff, high
                           // byte: materials set to zero)
  double* cons;            // conservation book-keeping, CONS_N doubles
  double* cpart;           // per-workgroup partial sums of the book-keeping
  double* scal;            // dt, dt/dx, dt/dy, dt/(dx dy) or dt/dx, dt_fixed, t,
                           // replay position and length of the step-size schedule
  unsigned long long* ctr; // smax bits, error cell, counters
  const double* dts;       // step-size schedule (replayed while position < length)
  double* dtpart;          // per-workgroup maxima of the wave speeds (step size)
  // stranded mixing sources of the stage (stamp per material and cell), the
  // cells holding one (list and listing stamp), relabelled cells (stamp and
  // new material); scale separation: oddball cells and their new material
  // and distance
  // 2D classification blocks that held no cut or band cell, one map per
  // stage parity (1: quiet; 0: not, or not known)
  uint8_t* cquiet[2];
  uint32_t *strStamp, *abMark, *rlStamp;
  uint8_t *rlTo, *ssTo;
  int32_t *abList, *ssList;
  double* ssPhi;
};

enum { S_DT = 0, S_LX, S_LY, S_LV, S_DTFIX, S_T, S_SPOS, S_SN };

// Device-to-device copies (and fills with zeros: no source), every buffer
// 8-byte aligned: for a launch of their own, or for extra workgroups of a
// kernel whose work touches none of them
constexpr int MAXCOPY = 32;
struct CopyList {
  const char* src[MAXCOPY];
  char* dst[MAXCOPY];
  size_t bytes[MAXCOPY];
  int n;
};
// workgroup b of nb: its share of every entry (strided over the words)
MMD void copy_list_part(const CopyList& L, int b, int nb) {
  for (int e = 0; e < L.n; e++) {
    size_t words = L.bytes[e] / 8, tail = L.bytes[e] % 8;
    const double* s8 = (const double*)L.src[e];
    double* d8 = (double*)L.dst[e];
    bool fill = s8 == nullptr;
    for (size_t w = (size_t)b * blockDim.x + threadIdx.x; w < words; w += (size_t)nb * blockDim.x)
      d8[w] = fill ? 0.0 : s8[w];
    if (b == 0 && threadIdx.x < tail)
      L.dst[e][words * 8 + threadIdx.x] = fill ? 0 : L.src[e][words * 8 + threadIdx.x];
  }
}
enum { C_SMAX = 0, C_ERR, C_POSFIX, C_FLUXSKIP, C_IFSKIP, C_STRANDED, C_MIXSRC,
       C_UPD, C_UPDB0, C_UPDB1, C_STAMP, C_NTILES, C_NBAND, C_NGHOST,
       // workgroups of the current launch that have finished (the last one
       // finishes the launch's work and sets the counter back to zero)
       C_DTDONE,
       // time steps completed since the initial state, and the lowest value
       // of that count at which a non-physical state was flagged
       C_STEPNO, C_ERRSTEP,
       // cells of an initial state given in device memory with chi outside
       // [0, n_mat) or phi negative or not a number
       C_BADIN,
       // conserved quantities moved between the materials of a cell (stranded
       // mixing sources), cells relabelled, oddball cells of the scale
       // separation; list lengths of the current stage / step; stamps of the
       // last stage with a relabelled cell and of the last step with an
       // oddball cell (the geometry is evaluated again when they match)
       C_ABSORB, C_RELABEL, C_ODDBALL, C_NAB, C_NSS, C_RLSTAMP, C_SSSTAMP, C_N };
constexpr unsigned long long NO_ERR = ~0ull;
// book-keeping regions of MAXM x 4 doubles each: accumulated net boundary
// inflow and its compensation, accumulated exchange and its compensation,
// and the last computed sums of Q
enum { CONS_BND = 0, CONS_BNDC = 1, CONS_X = 2, CONS_XC = 3, CONS_Q = 4, CONS_N = 5 * MAXM * 4 };
// cells (or boundary rows and columns) per workgroup of the partial sums
constexpr int CONS_CH = 2048;
static_assert(CONS_CH % 256 == 0, "cells of a book-keeping workgroup");

MMD int cid(const Params& P, int i, int j) { return (j + P.HY) * P.NX + i + H; }
MMD bool interior(const Params& P, int i, int j) {
  return i >= 0 && i < P.nx && j >= 0 && j < P.ny;
}
MMD double lsv(const double* phi, const uint8_t* chi, int r, int k) {
  return chi[k] == r ? phi[k] : -phi[k];
}
MMD bool errored(const Bufs& B) { return B.ctr[C_ERR] != NO_ERR; }
MMD void flag_error(const Params& P, const Bufs& B, int i, int j) {
  atomicMin(&B.ctr[C_ERR], (unsigned long long)j * P.nx + i);
  atomicMin(&B.ctr[C_ERRSTEP], B.ctr[C_STEPNO]);
}
// Counters bumped by many lanes at once go through one atomic per wavefront:
// the values of the lanes active at the call are summed with ballots (v < 16)
// and the lowest active lane adds the sum.
MMD void wave_count(unsigned long long* c, unsigned v) {
  unsigned long long act = __ballot(1);
  unsigned long long sum = 0;
  for (int b = 0; b < 4; b++) sum += (unsigned long long)__popcll(__ballot((v >> b) & 1)) << b;
  if (sum && __lane_id() == __ffsll(act) - 1) atomicAdd(c, sum);
}
// slot in a device queue for each active lane with take set: one atomic per
// wavefront reserves the wave's slots; returns the lane's slot (or -1)
MMD long long wave_slot(unsigned long long* c, bool take) {
  unsigned long long act = __ballot(1), m = __ballot(take);
  int leader = __ffsll(act) - 1, lane = __lane_id();
  unsigned long long base = 0;
  if (m && lane == leader) base = atomicAdd(c, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (!take) return -1;
  unsigned long long below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
  return (long long)(base + __popcll(below));
}
MMD bool nonphys(const Prim& w, double pinf) {
  return !(w.r > 0.0) || !(w.p + pinf > 0.0) || !isfinite(w.u) ||
         !isfinite(w.v) || !isfinite(w.r) || !isfinite(w.p);
}

// conserved component v (0..3 = rho, rho u, rho v, rho E) of material r;
// zero unless the occupancy bit is set; in 1D rho v is identically zero
template <int D>
MMD double loadQ(const Params& P, const double* Q, const uint8_t* occ, int r,
                 int v, int k) {
  if (!((occ[k] >> r) & 1)) return 0.0;
  if (D == 1) {
    if (v == 2) return 0.0;
    if (v == 3) v = 2;
  }
  return Q[((size_t)r * (D + 2) + v) * P.NC + k];
}
template <int D>
MMD void storeQ(const Params& P, double* Q, int r, int v, int k, double x) {
  if (D == 1) {
    if (v == 2) return;
    if (v == 3) v = 2;
  }
  Q[((size_t)r * (D + 2) + v) * P.NC + k] = x;
}
MMD double& M1(const Params& P, double* a, int r, int k) {
  return a[(size_t)r * P.NC + k];
}
MMD double& M4(const Params& P, double* a, int r, int v, int k) {
  return a[((size_t)r * 4 + v) * P.NC + k];
}

// geometry readers: cut cells carry stored values, all others are pure
template <int D>
MMD double alpha_at(const Params& P, const Bufs& B, int r, int k) {
  return B.cut[k] ? B.al[(size_t)r * P.NC + k] : (B.chi[k] == r ? 1.0 : 0.0);
}
// aperture of the x-face i+1/2 of row j (i in [-1, nx-1])
template <int D>
MMD double apx(const Params& P, const Bufs& B, int r, int i, int j) {
  int kl = cid(P, i, j), kr = cid(P, i + 1, j);
  // every word read in any case (all in range), then chosen: the loads of a
  // caller overlap; outside the domain the flags are not looked at
  uint8_t cl = B.cut[kl], cr = B.cut[kr], hl = B.chi[kl], hr = B.chi[kr];
  double a = B.ax[(size_t)r * P.NC + kl];
  bool use;
  int h;
  if (i < 0) {
    use = cr;
    h = hr;
  } else if (i >= P.nx - 1) {
    use = cl;
    h = hl;
  } else {
    use = cl && cr;
    h = cl ? hr : hl;
  }
  return use ? a : (h == r ? 1.0 : 0.0);
}
// aperture of the face between (i, j) and its +1 neighbour in direction dir
// (0: x, as apx; 1: y, as apy) with the direction a value, so that lanes of
// different directions run the same instructions
MMD double apd(const Params& P, const Bufs& B, int r, int i, int j, int dir) {
  int kl = cid(P, i, j), kr = dir == 0 ? cid(P, i + 1, j) : cid(P, i, j + 1);
  int q = dir == 0 ? i : j, n = dir == 0 ? P.nx : P.ny;
  uint8_t cl = B.cut[kl], cr = B.cut[kr], hl = B.chi[kl], hr = B.chi[kr];
  double a = (dir == 0 ? B.ax : B.ay)[(size_t)r * P.NC + kl];
  bool use;
  int h;
  if (q < 0) {
    use = cr;
    h = hr;
  } else if (q >= n - 1) {
    use = cl;
    h = hl;
  } else {
    use = cl && cr;
    h = cl ? hr : hl;
  }
  return use ? a : (h == r ? 1.0 : 0.0);
}
// aperture of the y-face j+1/2 of column i (j in [-1, ny-1])
MMD double apy(const Params& P, const Bufs& B, int r, int i, int j) {
  int kb = cid(P, i, j), kt = cid(P, i, j + 1);
  uint8_t cb = B.cut[kb], ct = B.cut[kt], hb = B.chi[kb], ht = B.chi[kt];
  double a = B.ay[(size_t)r * P.NC + kb];
  bool use;
  int h;
  if (j < 0) {
    use = ct;
    h = ht;
  } else if (j >= P.ny - 1) {
    use = cb;
    h = hb;
  } else {
    use = cb && ct;
    h = cb ? ht : hb;
  }
  return use ? a : (h == r ? 1.0 : 0.0);
}

// primitive state of material r at a cell: read from the real/ghost buffer
// within seven cells of a cut cell (where it is refreshed every stage),
// computed on the fly in the pure cells farther away (alpha = 1)
template <int D>
MMD Prim Wget(const Params& P, const Bufs& B, const double* Qs,
              const uint8_t* occs, int r, int i, int j, bool& valid) {
  int k = cid(P, i, j);
  bool in = interior(P, i, j);
  if (D == 2) {
    // branch-free form (the loads of several calls can be in flight
    // together): Q and the state buffer share the [material][4][cell]
    // layout in 2D, so one base pointer is chosen and the same words read
    uint8_t dc = B.dcut[k], ch = B.chi[k], it = B.Wit[(size_t)r * P.NC + k], oc = occs[k];
    bool far = in && dc > 7 && ch == r;
    bool has = (oc >> r) & 1;
    const double* base = far ? Qs : B.W;
    size_t o = (size_t)r * 4 * P.NC + k;
    double a0 = base[o], a1 = base[o + P.NC], a2 = base[o + 2 * (size_t)P.NC],
           a3 = base[o + 3 * (size_t)P.NC];
    valid = far || (it != 0 && (!in || dc <= 7));
    if (far) {
      double U0 = has ? a0 / 1.0 : 0.0, U1 = has ? a1 / 1.0 : 0.0, U2 = has ? a2 / 1.0 : 0.0,
             U3 = has ? a3 / 1.0 : 0.0;
      return prim_from_U(U0, U1, U2, U3, eos_of(P, r));
    }
    Prim w;
    w.r = a0;
    w.u = a1;
    w.v = a2;
    w.p = a3;
    return w;
  }
  if (in && B.dcut[k] > 7 && B.chi[k] == r) {
    valid = true;
    double U0 = loadQ<D>(P, Qs, occs, r, 0, k) / 1.0;
    double U1 = loadQ<D>(P, Qs, occs, r, 1, k) / 1.0;
    double U2 = loadQ<D>(P, Qs, occs, r, 2, k) / 1.0;
    double U3 = loadQ<D>(P, Qs, occs, r, 3, k) / 1.0;
    return prim_from_U(U0, U1, U2, U3, eos_of(P, r));
  }
  // buffer states are refreshed each stage within seven cells of a cut cell
  // (and in the frame); anything older is stale
  valid = B.Wit[(size_t)r * P.NC + k] != 0 && (!in || B.dcut[k] <= 7);
  Prim w;
  w.r = B.W[((size_t)r * 4 + 0) * P.NC + k];
  w.u = B.W[((size_t)r * 4 + 1) * P.NC + k];
  w.v = B.W[((size_t)r * 4 + 2) * P.NC + k];
  w.p = B.W[((size_t)r * 4 + 3) * P.NC + k];
  return w;
}

// ---------------------------------------------------------------------------
// Cylindrical geometry and free surfaces (Sec. 3, Case II)
// ---------------------------------------------------------------------------
// x0 + i dx: the radius of face i - 1/2 for an integer i, of the centre of
// cell i for i + 0.5
MMD double rad(const Params& P, double i) { return P.x0 + i * P.dx; }
// the ambient of a free surface: not solved
MMD bool passive(const Params& P, int r) { return P.fs_on && r == P.fs_mat; }
// time of the input state of stage s: t_n, then t_n + dt (and t_n + dt/2
// for the third stage of RK3)
MMD double stage_time(const Bufs& B, int s) {
  double t = B.scal[S_T];
  return s == 0 ? t : t + (s == 1 ? 1.0 : 0.5) * B.scal[S_DT];
}
// surface pressure p(t): p_hi up to t0, linear to p_lo at t1, p_lo after
MMD double fs_pressure(const Params& P, double t) {
  const double* f = P.fs_p;
  if (t <= f[2]) return f[0];
  if (t >= f[3]) return f[1];
  return f[0] - (f[0] - f[1]) * (t - f[2]) / (f[3] - f[2]);
}
// velocity jump across the wave that brings a stiffened-gas state of
// material m (density rho, pressure p) to the pressure ps: Toro's pressure
// function with pressures shifted by p_inf (shock for ps > p, else
// rarefaction)
MMD double wave_jump(const Params& P, int m, double rho, double p, double ps) {
  double g = P.gamma[m], pinf = P.pinf[m];
  double pb = p + pinf, psb = ps + pinf;
  if (ps > p) {
    double A = 2.0 / ((g + 1.0) * rho);
    double Bs = (g - 1.0) / (g + 1.0) * pb;
    return (ps - p) * sqrt(A / (psb + Bs));
  }
  double c = sqrt(g * pb / rho);
  return 2.0 * c / (g - 1.0) * (::pow(psb / pb, (g - 1.0) / (2.0 * g)) - 1.0);
}
// wave speed bound of a free surface in a cell whose material m has the
// state w: max(|u|, |v|) + |du| + the wave's front speed relative to the
// material (c for a rarefaction, the stiffened-gas shock speed
// c sqrt(1 + (g + 1)/(2 g) (ps - p)/(p + p_inf)) for a shock)
MMD double fs_speed(const Params& P, int m, const Prim& w, double ps) {
  double g = P.gamma[m];
  double pb = w.p + P.pinf[m];
  double c = sqrt(g * pb / w.r);
  if (ps > w.p) c = c * sqrt(1.0 + (g + 1.0) / (2.0 * g) * ((ps - w.p) / pb));
  double u = fabs(w.u), v = fabs(w.v);
  return (u > v ? u : v) + fabs(wave_jump(P, m, w.r, w.p, ps)) + c;
}
// The ambient at stage s, cell k (any cell of the padded array): its state is
// the prescribed one (density fs_p[4], at rest, under p of the stage's time)
// and valid; in interior cells its conserved quantities in buffer sidx are
// alpha U of that state, the occupancy following
template <int D>
MMD void b_ambient(const Params& P, const Bufs& B, int k, int sidx, int s) {
  int r = P.fs_mat;
  double p = fs_pressure(P, stage_time(B, s)), rho = P.fs_p[4];
  size_t o = (size_t)r * 4 * P.NC + k;
  B.W[o] = rho;
  B.W[o + (size_t)P.NC] = 0.0;
  B.W[o + (size_t)2 * P.NC] = 0.0;
  B.W[o + (size_t)3 * P.NC] = p;
  B.Wit[(size_t)r * P.NC + k] = 1;
  int i = k % P.NX - H, j = k / P.NX - P.HY;
  if (!interior(P, i, j)) return;
  double a = alpha_at<D>(P, B, r, k);
  double U[4] = {rho, 0.0, 0.0, total_energy(rho, 0.0, 0.0, p, P.gamma[r], P.pinf[r], P.igm1[r])};
  bool nz = false;
  for (int v = 0; v < 4; v++) {
    double x = a > 0.0 ? a * U[v] : 0.0;
    storeQ<D>(P, B.Q[sidx], r, v, k, x);
    if (x != 0.0 && !(D == 1 && v == 2)) nz = true;
  }
  unsigned occ = B.occ[sidx][k];
  B.occ[sidx][k] = (uint8_t)(nz ? occ | (1u << r) : occ & ~(1u << r));
}
template <int D>
__global__ void __launch_bounds__(256) k_ambient(Params P, Bufs B, int sidx, int s) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < P.NC) b_ambient<D>(P, B, k, sidx, s);
}

// ---------------------------------------------------------------------------
// Boundary frames
// ---------------------------------------------------------------------------
MMD int src_lo(int i, int type) { return type == 1 ? -1 - i : 0; }
MMD int src_hi(int i, int n, int type) { return type == 1 ? 2 * n - 1 - i : n - 1; }

// level set, x sides: rows j in [0, ny), 2*H halo cells per row
MMD void b_bc_ls_x(const Params& P, int t, double* phi, uint8_t* chi) {
  int j = t / (2 * H), q = t % (2 * H);
  int i, si;
  if (q < H) {
    i = -1 - q;
    si = src_lo(i, P.bc[0]);
  } else {
    i = P.nx + (q - H);
    si = src_hi(i, P.nx, P.bc[1]);
  }
  int k = cid(P, i, j), ks = cid(P, si, j);
  phi[k] = phi[ks];
  chi[k] = chi[ks];
}
__global__ void k_bc_ls_x(Params P, Bufs B, double* phi, uint8_t* chi) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.ny * 2 * H) return;
  b_bc_ls_x(P, t, phi, chi);
}
// level set, y sides: columns i in [-H, nx+H)
__global__ void k_bc_ls_y(Params P, Bufs B, double* phi, uint8_t* chi) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int ncol = P.nx + 2 * H;
  if (t >= ncol * 2 * H) return;
  int i = t / (2 * H) - H, q = t % (2 * H);
  int j, sj;
  if (q < H) {
    j = -1 - q;
    sj = src_lo(j, P.bc[2]);
  } else {
    j = P.ny + (q - H);
    sj = src_hi(j, P.ny, P.bc[3]);
  }
  int k = cid(P, i, j), ks = cid(P, i, sj);
  phi[k] = phi[ks];
  chi[k] = chi[ks];
}

// primitive states of every material, x sides (inflow: fixed state of the
// inflow material)
template <int D>
MMD void b_bc_W_x(const Params& P, const Bufs& B, int t, int sidx) {
  int r = t / (P.ny * 2 * H);
  int rem = t % (P.ny * 2 * H);
  int j = rem / (2 * H), q = rem % (2 * H);
  int i, si, type;
  if (q < H) {
    i = -1 - q;
    type = P.bc[0];
    si = src_lo(i, type);
  } else {
    i = P.nx + (q - H);
    type = P.bc[1];
    si = src_hi(i, P.nx, type);
  }
  int k = cid(P, i, j);
  size_t o = (size_t)r * 4 * P.NC;
  if (type == 2 && r == P.inflow_mat) {
    for (int v = 0; v < 4; v++) B.W[o + (size_t)v * P.NC + k] = P.inflow_W[v];
    B.Wit[(size_t)r * P.NC + k] = 1;
    return;
  }
  bool valid;
  Prim w = Wget<D>(P, B, B.Q[sidx], B.occ[sidx], r, si, j, valid);
  double sx = type == 1 ? -1.0 : 1.0;
  B.W[o + k] = w.r;
  B.W[o + (size_t)P.NC + k] = w.u * sx;
  B.W[o + (size_t)2 * P.NC + k] = w.v;
  B.W[o + (size_t)3 * P.NC + k] = w.p;
  B.Wit[(size_t)r * P.NC + k] = valid ? 1 : 0;
}
// state that the x-side frame gets at ghost cell (i, j) of material r, for
// i outside [0, nx) and j inside [0, ny)
MMD Prim bc_x_state(const Params& P, const Bufs& B, int sidx, int r, int i, int j,
                    bool& valid) {
  int type = i < 0 ? P.bc[0] : P.bc[1];
  int si = i < 0 ? src_lo(i, type) : src_hi(i, P.nx, type);
  Prim w;
  if (type == 2 && r == P.inflow_mat) {
    w.r = P.inflow_W[0];
    w.u = P.inflow_W[1];
    w.v = P.inflow_W[2];
    w.p = P.inflow_W[3];
    valid = true;
    return w;
  }
  w = Wget<2>(P, B, B.Q[sidx], B.occ[sidx], r, si, j, valid);
  w.u = w.u * (type == 1 ? -1.0 : 1.0);
  return w;
}
// both frames of the state buffer (2D), frame cell t: t below ny * 2H * M
// takes the x sides of rows [0, ny), the others the y sides of columns
// [-H, nx + H).  A corner cell gets the y-side map applied to the
// x-side state of its source row, the value an x pass followed by a y pass
// leaves there; every source is an interior cell, so no thread reads what
// another writes.
MMD void bc_W2_cell(const Params& P, const Bufs& B, int sidx, int t) {
  int nxs = P.ny * 2 * H, nys = (P.nx + 2 * H) * 2 * H;
  if (t >= (nxs + nys) * P.M) return;
  int r, i, j;
  bool valid;
  Prim w;
  if (t < nxs * P.M) {
    r = t / nxs;
    int rem = t % nxs, q = rem % (2 * H);
    j = rem / (2 * H);
    i = q < H ? -1 - q : P.nx + (q - H);
    w = bc_x_state(P, B, sidx, r, i, j, valid);
  } else {
    t -= nxs * P.M;
    r = t / nys;
    int rem = t % nys, q = rem % (2 * H);
    i = rem / (2 * H) - H;
    j = q < H ? -1 - q : P.ny + (q - H);
    int type = q < H ? P.bc[2] : P.bc[3];
    int sj = q < H ? src_lo(j, type) : src_hi(j, P.ny, type);
    if (type == 2 && r == P.inflow_mat) {
      w.r = P.inflow_W[0];
      w.u = P.inflow_W[1];
      w.v = P.inflow_W[2];
      w.p = P.inflow_W[3];
      valid = true;
    } else {
      w = i < 0 || i >= P.nx ? bc_x_state(P, B, sidx, r, i, sj, valid)
                             : Wget<2>(P, B, B.Q[sidx], B.occ[sidx], r, i, sj, valid);
      w.v = w.v * (type == 1 ? -1.0 : 1.0);
    }
  }
  int k = cid(P, i, j);
  size_t o = (size_t)r * 4 * P.NC;
  B.W[o + k] = w.r;
  B.W[o + (size_t)P.NC + k] = w.u;
  B.W[o + (size_t)2 * P.NC + k] = w.v;
  B.W[o + (size_t)3 * P.NC + k] = w.p;
  B.Wit[(size_t)r * P.NC + k] = valid ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Classification of the current level set: local material sets (3x3 block),
// cut cells, and Chebyshev distances to the nearest cut cell and to the
// nearest narrow-band cell (phi below the band width, or cut), capped at 15.
// ---------------------------------------------------------------------------
#define CELL_LOOP_2D                                         \
  int i = blockIdx.x * blockDim.x + threadIdx.x;             \
  int j = blockIdx.y * blockDim.y + threadIdx.y;             \
  if (i >= P.nx || j >= P.ny) return;                        \
  int k = cid(P, i, j);

template <int D>
MMD void b_classify(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  unsigned b = 0;
  for (int dj = -(D == 2); dj <= (D == 2); dj++)
    for (int di = -1; di <= 1; di++) b |= 1u << B.chi[cid(P, i + di, j + dj)];
  B.xs[k] = (uint8_t)b;
  bool c = (b & (b - 1)) != 0;
  B.cut[k] = c;
  B.rowc[k] = (uint8_t)(c ? 1 : 0);
  B.rowl[k] = (uint8_t)((c || B.phi[k] < P.bls) ? 1 : 0);
}
// gate >= 0: run only if counter gate holds the current stage's stamp (the
// classification and geometry evaluated again after cells changed material)
MMD bool gated_off(const Bufs& B, int gate) {
  return gate >= 0 && B.ctr[gate] != B.ctr[C_STAMP];
}
template <int D>
__global__ void k_classify(Params P, Bufs B, int gate) {
  if (gated_off(B, gate)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i == 0 && j == 0) B.ctr[C_NTILES] = 0;  // the tile list is rebuilt next
  if (i >= P.nx || j >= P.ny) return;
  b_classify<D>(P, B, i, j);
}

constexpr int RD = 13;  // distance cap (consumers test <= 8 and <= 12)
template <int D>
MMD void b_dist_row(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  // rowc/rowl hold 0/1 flags on entry of the cells; distances go to dcut/dls
  int dc = RD, dl = RD;
  for (int di = -RD + 1; di <= RD - 1; di++) {
    int ii = i + di;
    if (ii < 0 || ii >= P.nx) continue;
    int kk = cid(P, ii, j);
    int a = di < 0 ? -di : di;
    if (B.rowc[kk] && a < dc) dc = a;
    if (B.rowl[kk] && a < dl) dl = a;
  }
  // 1D: final distances; 2D: row distances for the column pass
  (D == 1 ? B.dcut : B.tdc)[k] = (uint8_t)dc;
  (D == 1 ? B.dls : B.tdl)[k] = (uint8_t)dl;
}
template <int D>
__global__ void k_dist_row(Params P, Bufs B, int gate) {
  if (gated_off(B, gate)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  b_dist_row<D>(P, B, i, j);
}
// column pass: d = min over dj of max(|dj|, row distance)
// 2D classification and distances in one launch: a CX x CY block of cells
// with a frame of RD - 1 cells (the reach of the distances) classified in LDS
// from the material indicators (one more cell around) and the level set; the
// capped Chebyshev distances of the row and column scans come from bit
// masks of the frame's rows.  Same results, one pass over global memory.
constexpr int CX = 40, CY = 24, CF = RD - 1;
struct ClassDistSmem {
  uint8_t chi[CY + 2 * CF + 2][CX + 2 * CF + 2];
  uint8_t fl[CY + 2 * CF][CX + 2 * CF];  // bit 0: cut, bit 1: level-set band
  unsigned long long mrow[2][CY + 2 * CF];  // the flags of a frame row as bits
};
static_assert(CX + 2 * CF <= 64, "a frame row fits one 64-bit mask");
//
// A block whose 3 x 3 neighbourhood of blocks held no cut or band cell at
// the previous stage is skipped: the level set and the indicators move less
// than a cell per stage, so such a block is still at least CY - 1 > RD cells
// from any flagged cell, and its outputs (single-material local sets, no cut
// cell, capped distances) are those it already holds.  The maps alternate
// with the parity of the stage stamp (read the previous stage's, write the
// current one); a restored state clears them, which makes every block run.
__global__ void __launch_bounds__(256) k_classify_dist2(Params P, Bufs B, int gate) {
  if (gated_off(B, gate)) return;
  __shared__ ClassDistSmem S;
  constexpr int HX = CX + 2 * CF + 2, HY = CY + 2 * CF + 2;
  constexpr int FX = CX + 2 * CF, FY = CY + 2 * CF;
  static_assert(CY - 1 > RD && CX - 1 > RD, "a quiet block neighbourhood spans more than RD");
  int tid = threadIdx.x, i0 = blockIdx.x * CX, j0 = blockIdx.y * CY;
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) B.ctr[C_NTILES] = 0;
  int par = (int)(B.ctr[C_STAMP] & 1);
  const uint8_t* prevq = B.cquiet[par ^ 1];
  uint8_t* curq = B.cquiet[par];
  int me = blockIdx.y * gridDim.x + blockIdx.x;
  {
    bool quiet = true;
    for (int dj = -1; dj <= 1; dj++)
      for (int di = -1; di <= 1; di++) {
        int bx = (int)blockIdx.x + di, by = (int)blockIdx.y + dj;
        if (bx >= 0 && by >= 0 && bx < (int)gridDim.x && by < (int)gridDim.y)
          quiet = quiet && prevq[by * gridDim.x + bx] != 0;
      }
    if (quiet) {
      if (tid == 0) curq[me] = 1;
      return;
    }
  }
  // indicators of the frame cells that border a domain cell (-1..nx, -1..ny)
  // and the level-set test of the frame's domain cells: every load of the
  // thread is issued before the first is used
  constexpr int N1 = (HX * HY + 255) / 256, N2 = (FX * FY + 255) / 256;
  uint8_t cv[N1], lf[N2];
#pragma unroll
  for (int n = 0; n < N1; n++) {
    int q = tid + n * 256;
    int ci = i0 - CF - 1 + q % HX, cj = j0 - CF - 1 + q / HX;
    bool in = q < HX * HY && ci >= -1 && ci <= P.nx && cj >= -1 && cj <= P.ny;
    uint8_t v = B.chi[in ? cid(P, ci, cj) : cid(P, 0, 0)];  // unconditional: no wait per load
    cv[n] = in ? v : 0;
  }
#pragma unroll
  for (int n = 0; n < N2; n++) {
    int q = tid + n * 256;
    int ci = i0 - CF + q % FX, cj = j0 - CF + q / FX;
    bool in = q < FX * FY && ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny;
    double ph = B.phi[in ? cid(P, ci, cj) : cid(P, 0, 0)];
    lf[n] = in && ph < P.bls ? 1 : 0;
  }
#pragma unroll
  for (int n = 0; n < N1; n++) {
    int q = tid + n * 256;
    if (q < HX * HY) S.chi[q / HX][q % HX] = cv[n];
  }
  __syncthreads();
  // flags of the domain cells of the frame (zero outside the domain)
  bool own_flag = false;
#pragma unroll
  for (int n = 0; n < N2; n++) {
    int q = tid + n * 256;
    if (q >= FX * FY) continue;
    int fx = q % FX, fy = q / FX;
    int ci = i0 - CF + fx, cj = j0 - CF + fy;
    uint8_t f = 0;
    if (ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny) {
      unsigned b = 0;
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) b |= 1u << S.chi[fy + 1 + dj][fx + 1 + di];
      bool c = (b & (b - 1)) != 0;
      int k = cid(P, ci, cj);
      f = (uint8_t)((c ? 1 : 0) | ((c || lf[n]) ? 2 : 0));
      if (fx >= CF && fx < CF + CX && fy >= CF && fy < CF + CY) {
        B.xs[k] = (uint8_t)b;
        B.cut[k] = c;
        if (f) own_flag = true;
      }
    }
    S.fl[fy][fx] = f;
  }
  int flagged = __syncthreads_or(own_flag);  // also the barrier after the flags
  if (tid == 0) curq[me] = flagged ? 0 : 1;
  // the frame's rows as bit masks (four 16-cell pieces per row)
  if (tid < 2 * FY) S.mrow[tid / FY][tid % FY] = 0;
  __syncthreads();
  for (int q = tid; q < 4 * FY; q += 256) {
    int y = q >> 2, x0 = (q & 3) * 16;
    unsigned long long m0 = 0, m1 = 0;
    for (int x = x0; x < x0 + 16 && x < FX; x++) {
      m0 |= (unsigned long long)(S.fl[y][x] & 1) << x;
      m1 |= (unsigned long long)((S.fl[y][x] >> 1) & 1) << x;
    }
    atomicOr(&S.mrow[0][y], m0);
    atomicOr(&S.mrow[1][y], m1);
  }
  __syncthreads();
  // Chebyshev distance to the nearest flag (RD when none within RD - 1):
  // the smallest t whose (2t+1) x (2t+1) window holds a flag, the rows of
  // the window OR-ed into one mask
  for (int q = tid; q < CX * CY; q += 256) {
    int x = q % CX, y = q / CX;
    int i = i0 + x, j = j0 + y;
    if (i >= P.nx || j >= P.ny) continue;
    int p = x + CF, yy = y + CF;
    int d[2] = {RD, RD};
    for (int b = 0; b < 2; b++) {
      unsigned long long m = S.mrow[b][yy];
#pragma unroll
      for (int t = 0; t < RD; t++) {  // no early exit: the row reads go out together
        if (t > 0) m |= S.mrow[b][yy - t] | S.mrow[b][yy + t];
        bool hit = ((m >> (p - t)) & ((2ull << (2 * t)) - 1)) != 0;
        if (hit && d[b] == RD) d[b] = t;
      }
    }
    int k = cid(P, i, j);
    B.dcut[k] = (uint8_t)d[0];
    B.dls[k] = (uint8_t)d[1];
  }
}
// next mixing stamp (device-resident so a captured step can be replayed)

// ghost-band membership: OR of the real-material bits within Chebyshev 4
template <int D>
MMD void b_near_row(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  if (B.dcut[k] > 8) {
    B.nrow[k] = 0;
    return;
  }
  unsigned b = 0;
  for (int di = -4; di <= 4; di++) {
    int ii = i + di;
    if (ii < 0 || ii >= P.nx) continue;
    int kk = cid(P, ii, j);
    int r = B.chi[kk];
    if (alpha_at<D>(P, B, r, kk) > 0.0) b |= 1u << r;
  }
  B.nrow[k] = (uint8_t)b;
}
template <int D>
MMD void b_near_col(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  if (B.dcut[k] > 4) return;
  unsigned b = 0;
  if (D == 1) {
    b = B.nrow[k];
  } else {
    for (int dj = -4; dj <= 4; dj++) {
      int jj = j + dj;
      if (jj < 0 || jj >= P.ny) continue;
      b |= B.nrow[cid(P, i, jj)];
    }
  }
  B.near4[k] = (uint8_t)b;
  if (B.glist) {
    // queue the (cell, material) pairs of the ghost band that have no state
    for (int r = 0; r < P.M; r++) {
      bool take = (b >> r) & 1;
      take = take && !(!B.cut[k] && B.chi[k] == r) && B.Wit[(size_t)r * P.NC + k] == 0;
      long long at = wave_slot(&B.ctr[C_NGHOST], take);
      if (take) B.glist[at] = k * 8 + r;
    }
  }
}

// ---------------------------------------------------------------------------
// Geometry of cut cells (Sec. 2.3) + volume-fraction correction (Eq.
// vol_corr2).  mass: partial densities from state buffer midx, or (init)
// alpha * rho of the initial primitive field Win.
// ---------------------------------------------------------------------------
template <int D>
MMD void b_geom(const Params& P, const Bufs& B, int i, int j, int midx, const double* Win) {
  int k = cid(P, i, j);
  (void)k;
  if (!B.cut[k]) return;
  const double* phi = B.phi;
  const uint8_t* chi = B.chi;
  double al[MAXM];
  for (int r = 0; r < P.M; r++) {
    if (D == 1) {
      int kl = cid(P, i - 1, j), kr = cid(P, i + 1, j);
      double c = lsv(phi, chi, r, k);
      double fl = (lsv(phi, chi, r, kl) + c) * 0.5;
      double fr = (c + lsv(phi, chi, r, kr)) * 0.5;
      int ol = chi[kl] < chi[k] ? chi[kl] : chi[k];
      int orr = chi[k] < chi[kr] ? chi[k] : chi[kr];
      bool il = inside(fl, ol, r), ir = inside(fr, orr, r), ic = inside(c, chi[k], r);
      double Al = il ? 1.0 : 0.0, Ar = ir ? 1.0 : 0.0;
      al[r] = (seg_frac(fl, il, c, ic) + seg_frac(c, ic, fr, ir)) * 0.5;
      B.ax[(size_t)r * P.NC + k] = Ar;
      if (i == 0) B.ax[(size_t)r * P.NC + kl] = Al;
      B.cx[(size_t)r * P.NC + k] = Ar - Al;
      if (P.coord == 1)
        // cylindrical: interface area per cell volume r_i dx from the faces'
        // areas and the volume fraction (alpha dx = r_s - r_{i-1/2} for a
        // material on the inner side), so that a uniform pressure balances
        // faces, geometric source and exchange
        B.cx[(size_t)r * P.NC + k] =
            ((Ar * rad(P, i + 1) - Al * rad(P, i)) - al[r] * P.dx) / rad(P, i + 0.5);
      B.cy[(size_t)r * P.NC + k] = 0.0;
      continue;
    }
    // corner (i+a-1/2, j+b-1/2) for a, b in {0, 1}: cells (i+a-1 .. i+a,
    // j+b-1 .. j+b)
    double cv[2][2];
    int co[2][2];
    for (int b = 0; b < 2; b++)
      for (int a = 0; a < 2; a++) {
        int ci = i + a - 1, cj = j + b - 1;
        int k00 = cid(P, ci, cj), k10 = cid(P, ci + 1, cj),
            k01 = cid(P, ci, cj + 1), k11 = cid(P, ci + 1, cj + 1);
        cv[b][a] = ((lsv(phi, chi, r, k00) + lsv(phi, chi, r, k11)) +
                    (lsv(phi, chi, r, k10) + lsv(phi, chi, r, k01))) * 0.25;
        int o = chi[k00];
        if (chi[k10] < o) o = chi[k10];
        if (chi[k01] < o) o = chi[k01];
        if (chi[k11] < o) o = chi[k11];
        co[b][a] = o;
      }
    double vsw = cv[0][0], vse = cv[0][1], vnw = cv[1][0], vne = cv[1][1];
    bool isw = inside(vsw, co[0][0], r), ise = inside(vse, co[0][1], r),
         inw = inside(vnw, co[1][0], r), ine = inside(vne, co[1][1], r);
    double c = lsv(phi, chi, r, k);
    bool ic = inside(c, chi[k], r);
    double Ar = seg_frac(vse, ise, vne, ine);  // x-face i+1/2
    double Al = seg_frac(vsw, isw, vnw, inw);  // x-face i-1/2
    double At = seg_frac(vnw, inw, vne, ine);  // y-face j+1/2
    double Ab = seg_frac(vsw, isw, vse, ise);  // y-face j-1/2
    double tl = tri_frac(vsw, isw, vnw, inw, c, ic);
    double tr = tri_frac(vse, ise, vne, ine, c, ic);
    double tb = tri_frac(vsw, isw, vse, ise, c, ic);
    double tt = tri_frac(vnw, inw, vne, ine, c, ic);
    al[r] = ((tl + tr) + (tb + tt)) * 0.25;
    size_t o = (size_t)r * P.NC;
    B.ax[o + k] = Ar;
    B.ay[o + k] = At;
    if (i == 0) B.ax[o + cid(P, -1, j)] = Al;
    if (j == 0) B.ay[o + cid(P, i, -1)] = Ab;
    B.cx[o + k] = (Ar - Al) * P.dy;
    B.cy[o + k] = (At - Ab) * P.dx;
  }
  // volume-fraction correction in cells with three or more materials
  int n = 0;
  unsigned vfc_f = 0xff, vfc_z = 0;
  for (int r = 0; r < P.M; r++)
    if (al[r] > 0.0) n++;
  if (n >= 3) {
    double mass[MAXM];
    for (int r = 0; r < P.M; r++) {
      if (Win) {
        size_t plane = (size_t)P.nx * P.ny;
        mass[r] = al[r] * Win[((size_t)r * (D + 2)) * plane + (size_t)j * P.nx + i];
      } else {
        mass[r] = loadQ<D>(P, B.Q[midx], B.occ[midx], r, 0, k);
      }
    }
    double sum = 0.0;
    for (int r = 0; r < P.M; r++) sum += al[r];
    double d = 1.0 - sum;
    unsigned used = 0;
    int prim = chi[k];
    while (d != 0.0) {
      int best = -1;
      for (int r = 0; r < P.M; r++) {
        if (r == prim || ((used >> r) & 1) || !(al[r] > 0.0)) continue;
        if (best < 0 || mass[r] < mass[best]) best = r;
      }
      if (best < 0) break;
      used |= 1u << best;
      double nv = al[best] + d;
      if (nv < 0.0) {
        al[best] = 0.0;
        d = nv;
        vfc_z |= 1u << best;
      } else {
        al[best] = nv;
        d = 0.0;
        vfc_f = (unsigned)best;
      }
    }
  }
  for (int r = 0; r < P.M; r++) B.al[(size_t)r * P.NC + k] = al[r];
  if (B.vfc) B.vfc[k] = (uint16_t)(vfc_f | (vfc_z << 8));
}
template <int D>
__global__ void k_geom(Params P, Bufs B, int midx, const double* Win) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  b_geom<D>(P, B, i, j, midx, Win);
}

// initial conserved state Q0 = alpha U(W) in buffer 0
template <int D>
MMD void b_init_Q(const Params& P, const Bufs& B, int i, int j, const double* Win) {
  int k = cid(P, i, j);
  (void)k;
  size_t plane = (size_t)P.nx * P.ny, q = (size_t)j * P.nx + i;
  unsigned occ = 0;
  for (int r = 0; r < P.M; r++) {
    double a = alpha_at<D>(P, B, r, k);
    double w0 = Win[((size_t)r * (D + 2) + 0) * plane + q];
    double w1 = Win[((size_t)r * (D + 2) + 1) * plane + q];
    double w2 = D == 2 ? Win[((size_t)r * (D + 2) + 2) * plane + q] : 0.0;
    double w3 = Win[((size_t)r * (D + 2) + D + 1) * plane + q];
    if (a > 0.0 && (!(w0 > 0.0) || !(w3 + P.pinf[r] > 0.0) || !isfinite(w1) ||
                    !isfinite(w2)))
      flag_error(P, B, i, j);
    double U[4];
    U[0] = w0;
    U[1] = w0 * w1;
    U[2] = w0 * w2;
    U[3] = total_energy(w0, w1, w2, w3, P.gamma[r], P.pinf[r], P.igm1[r]);
    bool nz = false;
    for (int v = 0; v < 4; v++) {
      double x = a > 0.0 ? a * U[v] : 0.0;
      storeQ<D>(P, B.Q[0], r, v, k, x);
      if (x != 0.0) nz = true;
    }
    if (nz) occ |= 1u << r;
  }
  B.occ[0][k] = (uint8_t)occ;
}
template <int D>
__global__ void k_init_Q(Params P, Bufs B, const double* Win) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  b_init_Q<D>(P, B, i, j, Win);
}

// ---------------------------------------------------------------------------
// Real states of cut cells, reset of ghost validity in the extension region
// ---------------------------------------------------------------------------
template <int D>
MMD void b_real(const Params& P, const Bufs& B, int i, int j, int sidx) {
  int k = cid(P, i, j);
  if (errored(B) || B.dcut[k] > 7) return;
  for (int r = 0; r < P.M; r++) B.Wit[(size_t)r * P.NC + k] = 0;
  int r = B.chi[k];
  if (passive(P, r)) return;  // set by the ambient pass
  double a = B.cut[k] ? B.al[(size_t)r * P.NC + k] : 1.0;
  if (!(a > 0.0)) return;
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  double U0 = loadQ<D>(P, Q, occ, r, 0, k) / a;
  double U1 = loadQ<D>(P, Q, occ, r, 1, k) / a;
  double U2 = loadQ<D>(P, Q, occ, r, 2, k) / a;
  double U3 = loadQ<D>(P, Q, occ, r, 3, k) / a;
  Prim w = prim_from_U(U0, U1, U2, U3, eos_of(P, r));
  // pure cells are checked where they are updated; cut cells here
  if (B.cut[k] && nonphys(w, P.pinf[r])) flag_error(P, B, i, j);
  size_t o = (size_t)r * 4 * P.NC;
  B.W[o + k] = w.r;
  B.W[o + (size_t)P.NC + k] = w.u;
  B.W[o + (size_t)2 * P.NC + k] = w.v;
  B.W[o + (size_t)3 * P.NC + k] = w.p;
  B.Wit[(size_t)r * P.NC + k] = 1;
}

// CFL step size from the time-n state: max over real cells of
// max(|u| + c, |v| + c); positive doubles order like their bit patterns
template <int D>
MMD double b_dt_cell(const Params& P, const Bufs& B, int i, int j, int sidx) {
  int k = cid(P, i, j), r = B.chi[k];
  double w = 0.0;
  if (alpha_at<D>(P, B, r, k) > 0.0 && !passive(P, r)) {
    bool valid;
    Prim s = Wget<D>(P, B, B.Q[sidx], B.occ[sidx], r, i, j, valid);
    double c = sqrt(P.gamma[r] * (s.p + P.pinf[r]) / s.r);
    double a = fabs(s.u) + c, b = fabs(s.v) + c;
    w = a > b ? a : b;
    if (!(w > 0.0)) w = 0.0;
    // a free surface in the cell: its wave against the prescribed pressure
    // (time t_n) bounds the step too
    if (P.fs_on && ((B.xs[k] >> P.fs_mat) & 1) && ((B.xs[k] >> r) & 1)) {
      double f = fs_speed(P, r, s, fs_pressure(P, B.scal[S_T]));
      if (f > w) w = f;
    }
  }
  return w;
}
template <int D>
MMD void dt_finish(const Params& P, const Bufs& B, double smax) {
  // a fixed step size first, then the schedule's next entry, else CFL
  double dt;
  if (B.scal[S_DTFIX] > 0.0) {
    dt = B.scal[S_DTFIX];
  } else if (B.scal[S_SPOS] < B.scal[S_SN]) {
    dt = B.dts[(long long)B.scal[S_SPOS]];
    B.scal[S_SPOS] += 1.0;
  } else {
    dt = P.cfl * P.h / smax;
  }
  B.scal[S_DT] = dt;
  B.scal[S_LX] = dt / P.dx;
  B.scal[S_LY] = dt / P.dy;
  B.scal[S_LV] = D == 2 ? dt / (P.dx * P.dy) : dt / P.dx;
}

// ---------------------------------------------------------------------------
// Ghost states: Jacobi sweeps over the ghost band of every material
// ---------------------------------------------------------------------------
// one ghost-extension sweep for material r at cell (i, j)
template <int D>
MMD void ext_one(const Params& P, const Bufs& B, int i, int j, int r, int sidx, int sweep) {
  int k = cid(P, i, j);
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  auto valid_prev = [&](int ii, int jj) -> bool {
    if (!interior(P, ii, jj)) return false;
    int kk = cid(P, ii, jj);
    if (B.dcut[kk] > 7) return B.chi[kk] == r;
    uint8_t it = B.Wit[(size_t)r * P.NC + kk];
    return it != 0 && it <= sweep + 1;
  };
  double out[4];
  bool ok = false;
  if (sweep < P.kext) {
    double gx = lsv(B.phi, B.chi, r, cid(P, i + 1, j)) - lsv(B.phi, B.chi, r, cid(P, i - 1, j));
    double gy = D == 2 ? lsv(B.phi, B.chi, r, cid(P, i, j + 1)) - lsv(B.phi, B.chi, r, cid(P, i, j - 1)) : 0.0;
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
      Prim a = Wget<D>(P, B, Q, occ, r, xi, j, vd);
      Prim b = Wget<D>(P, B, Q, occ, r, i, yj, vd);
      double wx = fabs(gx), wy = fabs(gy);
      out[0] = (wx * a.r + wy * b.r) / (wx + wy);
      out[1] = (wx * a.u + wy * b.u) / (wx + wy);
      out[2] = (wx * a.v + wy * b.v) / (wx + wy);
      out[3] = (wx * a.p + wy * b.p) / (wx + wy);
      ok = true;
    } else if (hx || hy) {
      Prim a = hx ? Wget<D>(P, B, Q, occ, r, xi, j, vd) : Wget<D>(P, B, Q, occ, r, i, yj, vd);
      out[0] = a.r;
      out[1] = a.u;
      out[2] = a.v;
      out[3] = a.p;
      ok = true;
    }
  } else {
    double row[3][4];
    int cnt = 0;
    for (int dj = -1; dj <= 1; dj++) {
      double a[3][4];
      for (int di = -1; di <= 1; di++) {
        bool use = (di != 0 || dj != 0) && (D == 2 || dj == 0) &&
                   valid_prev(i + di, j + dj);
        Prim w;
        w.r = w.u = w.v = w.p = 0.0;
        bool vd;
        if (use) w = Wget<D>(P, B, Q, occ, r, i + di, j + dj, vd);
        a[di + 1][0] = use ? w.r : 0.0;
        a[di + 1][1] = use ? w.u : 0.0;
        a[di + 1][2] = use ? w.v : 0.0;
        a[di + 1][3] = use ? w.p : 0.0;
        cnt += use ? 1 : 0;
      }
      for (int c = 0; c < 4; c++) row[dj + 1][c] = (a[0][c] + a[2][c]) + a[1][c];
    }
    if (cnt > 0) {
      for (int c = 0; c < 4; c++)
        out[c] = ((row[0][c] + row[2][c]) + row[1][c]) / (double)cnt;
      ok = true;
    }
  }
  if (ok) {
    size_t o = (size_t)r * 4 * P.NC;
    for (int c = 0; c < 4; c++) B.W[o + (size_t)c * P.NC + k] = out[c];
    B.Wit[(size_t)r * P.NC + k] = (uint8_t)(sweep + 2);
  }
}
template <int D>
MMD void b_ext(const Params& P, const Bufs& B, int i, int j, int sidx, int sweep) {
  int k = cid(P, i, j);
  if (errored(B) || B.dcut[k] > 4) return;
  for (int r = 0; r < P.M; r++) {
    if (!((B.near4[k] >> r) & 1)) continue;
    if (!B.cut[k] && B.chi[k] == r) continue;  // pure real cell
    if (B.Wit[(size_t)r * P.NC + k] != 0) continue;
    ext_one<D>(P, B, i, j, r, sidx, sweep);
  }
}

// ---------------------------------------------------------------------------
// Reduced interface interaction (Sec. 2.3.2) in cut cells
// ---------------------------------------------------------------------------
template <int D>
MMD void b_iface(const Params& P, const Bufs& B, int i, int j, int sidx, int stage) {
  int k = cid(P, i, j);
  bool stage0 = stage == 0;
  (void)k;
  if (errored(B) || !B.cut[k]) return;
  for (int r = 0; r < P.M; r++)
    for (int v = 0; v < 4; v++) B.X[((size_t)r * 4 + v) * P.NC + k] = 0.0;
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
  if (!va || !vb) {
    wave_count(&B.ctr[C_IFSKIP], 1);
    return;
  }
  double nrm = sqrt(cxa * cxa + cya * cya);
  double nxv = cxa / nrm, nyv = cya / nrm;
  Prim L, R;
  L.r = Wb.r;
  L.u = Wb.u * nxv + Wb.v * nyv;
  L.v = 0.0;
  L.p = Wb.p;
  R.r = Wa.r;
  R.u = Wa.u * nxv + Wa.v * nyv;
  R.v = 0.0;
  R.p = Wa.p;
  double SM, ps;
  bool pa = passive(P, a), pb = passive(P, bb);
  if (pa || pb) {
    // free surface (Sec. 3 Case II): the pressure is prescribed, and the
    // surface moves with the velocity the solved side's wave reaches at it
    // (the solved side is R when it is a, L otherwise, along n)
    ps = fs_pressure(P, stage_time(B, stage));
    SM = pb ? R.u + wave_jump(P, a, R.r, R.p, ps) : L.u - wave_jump(P, bb, L.r, L.p, ps);
  } else {
    double SL, SR;
    wave_speeds(L, eos_of(P, bb), R, eos_of(P, a), SL, SR);
    SM = contact_speed(L, R, SL, SR);
    ps = 0.5 * ((L.p + L.r * (SL - L.u) * (SM - L.u)) +
                (R.p + R.r * (SR - R.u) * (SM - R.u)));
  }
  double X1 = ps * cxa, X2 = ps * cya, X3 = ps * SM * nrm;
  size_t oa = (size_t)a * 4 * P.NC, ob = (size_t)bb * 4 * P.NC;
  // nothing is exchanged with an ambient that is not solved
  B.X[oa + (size_t)1 * P.NC + k] = pa ? 0.0 : X1;
  B.X[oa + (size_t)2 * P.NC + k] = pa ? 0.0 : X2;
  B.X[oa + (size_t)3 * P.NC + k] = pa ? 0.0 : X3;
  B.X[ob + k] = pb ? 0.0 : -0.0;
  B.X[ob + (size_t)1 * P.NC + k] = pb ? 0.0 : -X1;
  B.X[ob + (size_t)2 * P.NC + k] = pb ? 0.0 : -X2;
  B.X[ob + (size_t)3 * P.NC + k] = pb ? 0.0 : -X3;
  if (stage0) {
    B.vx[k] = SM * nxv;
    B.vy[k] = SM * nyv;
    B.vit[k] = 1;
  }
}

// ---------------------------------------------------------------------------
// Level-set advection velocity v^n (stage 0)
// ---------------------------------------------------------------------------
constexpr int RV = 12;  // reach of the level-set band over one step
template <int D>
MMD void b_vreset(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  if (B.dls[k] > RV) return;
  B.vit[k] = 0;
}
template <int D>
MMD void b_vext(const Params& P, const Bufs& B, int i, int j, int sweep) {
  int k = cid(P, i, j);
  (void)k;
  if (errored(B) || B.dls[k] != 0 || !(B.phi[k] < P.bls) || B.vit[k] != 0) return;
  auto valid_prev = [&](int ii, int jj) -> bool {
    if (!interior(P, ii, jj)) return false;
    uint8_t it = B.vit[cid(P, ii, jj)];
    return it != 0 && it <= sweep + 1;
  };
  double gx = B.phi[cid(P, i + 1, j)] - B.phi[cid(P, i - 1, j)];
  double gy = D == 2 ? B.phi[cid(P, i, j + 1)] - B.phi[cid(P, i, j - 1)] : 0.0;
  int kx = -1, ky = -1;
  if (gx != 0.0) {
    int ii = i - (gx > 0.0 ? 1 : -1);
    if (valid_prev(ii, j)) kx = cid(P, ii, j);
  }
  if (gy != 0.0) {
    int jj = j - (gy > 0.0 ? 1 : -1);
    if (valid_prev(i, jj)) ky = cid(P, i, jj);
  }
  double ox, oy;
  if (kx >= 0 && ky >= 0) {
    double wx = fabs(gx), wy = fabs(gy);
    ox = (wx * B.vx[kx] + wy * B.vx[ky]) / (wx + wy);
    oy = (wx * B.vy[kx] + wy * B.vy[ky]) / (wx + wy);
  } else if (kx >= 0) {
    ox = B.vx[kx];
    oy = B.vy[kx];
  } else if (ky >= 0) {
    ox = B.vx[ky];
    oy = B.vy[ky];
  } else {
    return;
  }
  B.vx[k] = ox;
  B.vy[k] = oy;
  B.vit[k] = (uint8_t)(sweep + 2);
}
// remaining cells: velocity of the cell's own material; also keep the
// time-n level set for the whole reach of this step's band
template <int D>
MMD void b_vfill(const Params& P, const Bufs& B, int i, int j, int sidx) {
  int k = cid(P, i, j);
  (void)k;
  if (B.dls[k] > RV) return;
  B.phin[k] = B.phi[k];
  B.chin[k] = B.chi[k];
  if (B.vit[k] != 0) return;
  bool valid;
  Prim w = Wget<D>(P, B, B.Q[sidx], B.occ[sidx], B.chi[k], i, j, valid);
  B.vx[k] = valid ? w.u : 0.0;
  B.vy[k] = valid ? w.v : 0.0;
}

// ---------------------------------------------------------------------------
// Fluxes and RK stage update
// ---------------------------------------------------------------------------
template <int D>
MMD bool is_bulk(const Params& P, const Bufs& B, int k, int sidx, int nidx) {
  uint8_t own = (uint8_t)(1u << B.chi[k]);
  return B.dcut[k] > 3 && B.occ[sidx][k] == own && B.occ[nidx][k] == own;
}
template <int D>
MMD void b_bulkflag(const Params& P, const Bufs& B, int i, int j, int sidx, int nidx) {
  int k = cid(P, i, j);
  B.bulk[k] = is_bulk<D>(P, B, k, sidx, nidx) ? 1 : 0;
}
// Bulk flags of a block of 256 cells (bw x 256 / bw; workgroup (bx, by) of
// nblk), their compact list of all other cells, and (at stage 0) the CFL
// maximum and from it, in the last workgroup to finish, the step size.  Every
// thread reaches the barriers.
template <int D>
MMD void bulkflag_block(const Params& P, const Bufs& B, int sidx, int nidx, int with_dt, int bx,
                        int by, int bw, int gx) {
  __shared__ int s_cnt, s_base;
  __shared__ double red[256];
  int tid = threadIdx.x;
  int i = bx * bw + tid % bw;
  int j = by * (256 / bw) + tid / bw;
  bool inb = i < P.nx && j < P.ny;
  int k = inb ? cid(P, i, j) : 0;
  bool band = false;
  if (inb) {
    bool bk = is_bulk<D>(P, B, k, sidx, nidx);
    B.bulk[k] = bk ? 1 : 0;
    band = !bk;
  }
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  int my = band ? atomicAdd(&s_cnt, 1) : 0;
  __syncthreads();
  if (tid == 0 && s_cnt) s_base = (int)atomicAdd(&B.ctr[C_NBAND], (unsigned long long)s_cnt);
  __syncthreads();
  if (band) B.blist[s_base + my] = k;
  if (with_dt) {
    // the workgroup's maximum wave speed; a workgroup of the next launch
    // combines them into the step size (a maximum: order-independent)
    red[tid] = inb ? b_dt_cell<D>(P, B, i, j, sidx) : 0.0;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
      __syncthreads();
    }
    if (tid == 0) B.dtpart[by * gx + bx] = red[0];
  }
}

// step size from the workgroup maxima of bulkflag_block (one workgroup of
// 256 threads)
template <int D>
MMD void dt_reduce_block(const Params& P, const Bufs& B, int nblk) {
  __shared__ double red[256];
  int tid = threadIdx.x;
  double m = 0.0;
  for (int q = tid; q < nblk; q += 256) m = fmax(m, B.dtpart[q]);
  red[tid] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  if (tid == 0) dt_finish<D>(P, B, red[0]);
}

// flux of material r across the face between cell (i, j) and its +1
// neighbour in direction dir (0: x, 1: y); stencil of six cells
// FLUX: the face-flux variant fixed at compile time (FLUX_HLLC, FLUX_ROE) or
// chosen from the parameters (-1, for the less frequent callers)
template <int D, int FLUX = -1>
MMD void face_flux(const Params& P, const Bufs& B, const double* Q,
                   const uint8_t* occ, int r, int i, int j, int dir,
                   bool count, double F[4]) {
  Prim Wc[6];
  bool vc[6];
  bool ok = true;
  for (int q = 0; q < 6; q++) {
    int ii = dir == 0 ? i - 2 + q : i, jj = dir == 0 ? j : j - 2 + q;
    Wc[q] = Wget<D>(P, B, Q, occ, r, ii, jj, vc[q]);
    if (!vc[q]) ok = false;
  }
  if (!vc[2] || !vc[3]) {
    wave_count(&B.ctr[C_FLUXSKIP], count ? 1 : 0);
    F[0] = F[1] = F[2] = F[3] = 0.0;
    return;
  }
  double pinf = P.pinf[r];
  Prim L, R;
  auto nrm = [&](const Prim& w) { return dir == 0 ? w.u : w.v; };
  auto tng = [&](const Prim& w) { return dir == 0 ? w.v : w.u; };
  if (FLUX == FLUX_ROE || (FLUX < 0 && P.flux == FLUX_ROE)) {
    Prim Ws[6];
    for (int q = 0; q < 6; q++) {
      Ws[q].r = Wc[q].r;
      Ws[q].u = nrm(Wc[q]);
      Ws[q].v = D == 2 ? tng(Wc[q]) : 0.0;
      Ws[q].p = Wc[q].p;
    }
    double G[4];
    bool good = roe_face(Ws, ok, eos_of(P, r), P.igm1[r], G);
    wave_count(&B.ctr[C_POSFIX], count && !good ? 1 : 0);
    F[0] = G[0];
    F[1] = dir == 0 ? G[1] : G[2];
    F[2] = dir == 0 ? G[2] : G[1];
    F[3] = G[3];
    return;
  }
  if (ok) {
    L.r = weno5(Wc[0].r, Wc[1].r, Wc[2].r, Wc[3].r, Wc[4].r);
    L.u = weno5(nrm(Wc[0]), nrm(Wc[1]), nrm(Wc[2]), nrm(Wc[3]), nrm(Wc[4]));
    L.v = D == 2 ? weno5(tng(Wc[0]), tng(Wc[1]), tng(Wc[2]), tng(Wc[3]), tng(Wc[4])) : 0.0;
    L.p = weno5(Wc[0].p, Wc[1].p, Wc[2].p, Wc[3].p, Wc[4].p);
    R.r = weno5(Wc[5].r, Wc[4].r, Wc[3].r, Wc[2].r, Wc[1].r);
    R.u = weno5(nrm(Wc[5]), nrm(Wc[4]), nrm(Wc[3]), nrm(Wc[2]), nrm(Wc[1]));
    R.v = D == 2 ? weno5(tng(Wc[5]), tng(Wc[4]), tng(Wc[3]), tng(Wc[2]), tng(Wc[1])) : 0.0;
    R.p = weno5(Wc[5].p, Wc[4].p, Wc[3].p, Wc[2].p, Wc[1].p);
    if (!(L.r > 0.0) || !(R.r > 0.0) || !(L.p + pinf > 0.0) || !(R.p + pinf > 0.0))
      ok = false;
  }
  if (!ok) {
    wave_count(&B.ctr[C_POSFIX], count ? 1 : 0);
    L.r = Wc[2].r; L.u = nrm(Wc[2]); L.v = tng(Wc[2]); L.p = Wc[2].p;
    R.r = Wc[3].r; R.u = nrm(Wc[3]); R.v = tng(Wc[3]); R.p = Wc[3].p;
  }
  double G[4];
  hllc_flux(L, R, eos_of(P, r), P.igm1[r], G);
  F[0] = G[0];
  F[1] = dir == 0 ? G[1] : G[2];
  F[2] = dir == 0 ? G[2] : G[1];
  F[3] = G[3];
}

// general update of every material in cells next to interfaces
template <int D>
MMD void b_flux_band(const Params& P, const Bufs& B, int i, int j, int sidx, int nidx, int didx,
                            double bcoef, double ccoef) {
  int k = cid(P, i, j);
  (void)k;
  if (errored(B) || B.bulk[k]) return;
  const double* Qs = B.Q[sidx];
  const double* Qn = B.Q[nidx];
  const uint8_t* os = B.occ[sidx];
  const uint8_t* on = B.occ[nidx];
  double lx = B.scal[S_LX], ly = B.scal[S_LY], lv = B.scal[S_LV];
  // non-cut cells are real cells of their material: check them here
  if (!B.cut[k] && !passive(P, B.chi[k])) {
    bool vd;
    int r = B.chi[k];
    Prim w = Wget<D>(P, B, Qs, os, r, i, j, vd);
    if (nonphys(w, P.pinf[r])) flag_error(P, B, i, j);
  }
  double out[MAXM][4];
  unsigned occ = 0;
  unsigned long long nact = 0;
  for (int r = 0; r < P.M; r++)
    if (alpha_at<D>(P, B, r, k) > 0.0 && !passive(P, r)) nact++;
  wave_count(&B.ctr[C_UPD], (unsigned)nact);
  for (int r = 0; r < P.M; r++) {
    if (passive(P, r)) {
      // an ambient that is not solved: the stage leaves it as it is
      bool nz = false;
      for (int v = 0; v < 4; v++) {
        out[r][v] = loadQ<D>(P, Qs, os, r, v, k);
        if (out[r][v] != 0.0 && !(D == 1 && v == 2)) nz = true;
      }
      if (nz) occ |= 1u << r;
      continue;
    }
    double Fl[4] = {0, 0, 0, 0}, Fr[4] = {0, 0, 0, 0}, Fb[4] = {0, 0, 0, 0},
           Ft[4] = {0, 0, 0, 0};
    double Al = apx<D>(P, B, r, i - 1, j), Ar = apx<D>(P, B, r, i, j);
    double Ab = 0.0, At = 0.0;
    if (Al > 0.0) face_flux<D>(P, B, Qs, os, r, i - 1, j, 0, i == 0, Fl);
    if (Ar > 0.0) face_flux<D>(P, B, Qs, os, r, i, j, 0, true, Fr);
    if (D == 2) {
      Ab = apy(P, B, r, i, j - 1);
      At = apy(P, B, r, i, j);
      if (Ab > 0.0) face_flux<D>(P, B, Qs, os, r, i, j - 1, 1, j == 0, Fb);
      if (At > 0.0) face_flux<D>(P, B, Qs, os, r, i, j, 1, true, Ft);
    }
    bool nz = false;
    for (int v = 0; v < 4; v++) {
      if (D == 1 && v == 2) {
        out[r][v] = 0.0;
        continue;
      }
      double fl = Al > 0.0 ? Al * Fl[v] : 0.0;
      double fr = Ar > 0.0 ? Ar * Fr[v] : 0.0;
      double rhs = lx * (fl - fr);
      if (D == 1 && P.coord == 1) {
        // cylindrical: face areas per cell volume, geometric source
        double ri = rad(P, i + 0.5);
        rhs = lx * (fl * rad(P, i) - fr * rad(P, i + 1)) / ri;
        bool vd;
        Prim w = Wget<D>(P, B, Qs, os, r, i, j, vd);
        if (v == 1 && vd) rhs = rhs + B.scal[S_DT] * (alpha_at<D>(P, B, r, k) * w.p / ri);
      }
      if (D == 2) {
        double fb = Ab > 0.0 ? Ab * Fb[v] : 0.0;
        double ft = At > 0.0 ? At * Ft[v] : 0.0;
        rhs = rhs + ly * (fb - ft);
      }
      double X = B.cut[k] ? B.X[((size_t)r * 4 + v) * P.NC + k] : 0.0;
      rhs = rhs + lv * X;
      double qn = loadQ<D>(P, Qn, on, r, v, k);
      double qs = loadQ<D>(P, Qs, os, r, v, k);
      double x = bcoef * qn + ccoef * (qs + rhs);
      out[r][v] = x;
      if (x != 0.0) nz = true;
    }
    if (nz) occ |= 1u << r;
  }
  for (int r = 0; r < P.M; r++)
    if ((occ >> r) & 1)
      for (int v = 0; v < 4; v++) storeQ<D>(P, B.Q[didx], r, v, k, out[r][v]);
  B.occ[didx][k] = (uint8_t)occ;
}

// Bulk update: cells with no cut cell within three cells and only their own
// material present.  There alpha = A = 1 and the exchange term vanishes
// (Sec. 2.4: the single-material block degenerates to standard finite
// volumes).  A workgroup of NT threads updates a BX x BY tile: the primitive
// states of the tile and a 3-cell frame are staged in LDS once; the x-face
// fluxes are computed (each once), shared through LDS by the face's two
// cells and reduced into per-cell sums, then the y-faces reuse the same LDS.
template <int BX, int BY>
struct BulkTile {
  static constexpr int WX = BX + 6, WY = BY + 6;
  static constexpr int NFX = (BX + 1) * BY, NFY = BX * (BY + 1);
  static constexpr int NFM = NFX > NFY ? NFX : NFY;
  double W[4][WY][WX];
  double F[4][NFM];
  uint8_t chi[WY][WX];
  uint8_t bulk[BY + 2][BX + 2];
};

// flux across face (fi, fj) of the tile in direction dir (0: the left face of
// tile cell (fi, fj), 1: its bottom face), rotated back to (rho, x, y, E)
// momentum order; false when neither cell of the face is a bulk cell
template <int BX, int BY, int FLUX>
MMD bool bulk_face(const Params& P, const Bufs& B, const BulkTile<BX, BY>& sm, int dir,
                   int fi, int fj, double G[4]) {
  // the two cells of the face in tile coordinates: (fi-1, fj) | (fi, fj)
  // or (fi, fj-1) | (fi, fj); the bulk marks are offset by one
  bool need = dir == 0 ? (sm.bulk[fj + 1][fi] || sm.bulk[fj + 1][fi + 1])
                       : (sm.bulk[fj][fi + 1] || sm.bulk[fj + 1][fi + 1]);
  if (!need) return false;
  int m = dir == 0 ? (sm.bulk[fj + 1][fi + 1] ? sm.chi[fj + 3][fi + 3] : sm.chi[fj + 3][fi + 2])
                   : (sm.bulk[fj + 1][fi + 1] ? sm.chi[fj + 3][fi + 3] : sm.chi[fj + 2][fi + 3]);
  // stencil cell q (0..5: cells fi-3 .. fi+2 along dir) of component v in
  // face-normal order (rho, normal velocity, tangential velocity, p), read
  // from LDS where it is used so that few values stay live in registers
  int bx = dir == 0 ? fi : fi + 3, by = dir == 0 ? fj + 3 : fj;
  int sx = dir == 0 ? 1 : 0, sy = dir == 0 ? 0 : 1;
  int vn = dir == 0 ? 1 : 2, vt = dir == 0 ? 2 : 1;
  auto c = [&](int q, int v) -> double {
    int comp = v == 1 ? vn : v == 2 ? vt : v;
    return sm.W[comp][by + q * sy][bx + q * sx];
  };
  if (FLUX == FLUX_ROE) {
    Prim Ws[6];
    for (int q = 0; q < 6; q++) {
      Ws[q].r = c(q, 0);
      Ws[q].u = c(q, 1);
      Ws[q].v = c(q, 2);
      Ws[q].p = c(q, 3);
    }
    double Gf[4];
    if (!roe_face(Ws, true, eos_of(P, m), P.igm1[m], Gf)) atomicAdd(&B.ctr[C_POSFIX], 1ull);
    G[0] = Gf[0];
    G[1] = dir == 0 ? Gf[1] : Gf[2];
    G[2] = dir == 0 ? Gf[2] : Gf[1];
    G[3] = Gf[3];
    return true;
  }
  double pinf = P.pinf[m];
  Prim L, R;
  L.r = weno5(c(0, 0), c(1, 0), c(2, 0), c(3, 0), c(4, 0));
  L.u = weno5(c(0, 1), c(1, 1), c(2, 1), c(3, 1), c(4, 1));
  L.v = weno5(c(0, 2), c(1, 2), c(2, 2), c(3, 2), c(4, 2));
  L.p = weno5(c(0, 3), c(1, 3), c(2, 3), c(3, 3), c(4, 3));
  R.r = weno5(c(5, 0), c(4, 0), c(3, 0), c(2, 0), c(1, 0));
  R.u = weno5(c(5, 1), c(4, 1), c(3, 1), c(2, 1), c(1, 1));
  R.v = weno5(c(5, 2), c(4, 2), c(3, 2), c(2, 2), c(1, 2));
  R.p = weno5(c(5, 3), c(4, 3), c(3, 3), c(2, 3), c(1, 3));
  if (!(L.r > 0.0) || !(R.r > 0.0) || !(L.p + pinf > 0.0) || !(R.p + pinf > 0.0)) {
    atomicAdd(&B.ctr[C_POSFIX], 1ull);
    L.r = c(2, 0); L.u = c(2, 1); L.v = c(2, 2); L.p = c(2, 3);
    R.r = c(3, 0); R.u = c(3, 1); R.v = c(3, 2); R.p = c(3, 3);
  }
  double Gf[4];
  hllc_flux(L, R, eos_of(P, m), P.igm1[m], Gf);
  G[0] = Gf[0];
  G[1] = dir == 0 ? Gf[1] : Gf[2];
  G[2] = dir == 0 ? Gf[2] : Gf[1];
  G[3] = Gf[3];
  return true;
}

// Tiles of the bulk kernel: 28 x 16 cells with 512 threads, so that both
// face sets (29 x 16 and 28 x 17) take one pass (40.7 KB of LDS), for grids
// of a few tiles per compute unit (896 x 384: three); 28 x 32 cells with
// 1024 threads (73.6 KB) for larger grids, where the smaller frame overhead
// wins once every CU has several tiles to work through (measured crossover
// between 3 and 9 tiles of 28 x 16 per CU; 30 x 33 tiles, whose face sets
// fill all 1024 threads, measured no faster).  The register budget is left
// to the compiler: a tighter one spills to scratch, and the spill traffic
// outweighs the extra waves.
constexpr int BULK_BX = 28, BULK_BY = 16, BULK_NT = 512;
constexpr int BULK_BXW = 28, BULK_BYW = 32, BULK_NTW = 1024;
constexpr int BULK_WIDE_TILES_PER_CU = 6;

template <int BX, int BY, int NT, int FLUX>
__global__ void __launch_bounds__(NT)
k_flux_bulk2(Params P, Bufs B, int sidx, int nidx, int didx, double bcoef,
             double ccoef, int stage0) {
  using T = BulkTile<BX, BY>;
  constexpr int WX = T::WX, WY = T::WY, NFX = T::NFX, NFY = T::NFY;
  static_assert(NT >= BX * BY, "one thread per tile cell");
  __shared__ T sm;
  int tid = threadIdx.x;
  int tx = tid % BX, ty = tid / BX;
  int i0 = blockIdx.x * BX, j0 = blockIdx.y * BY;
  int i = i0 + tx, j = j0 + ty;
  bool inb = tid < BX * BY && i < P.nx && j < P.ny;
  int k = inb ? cid(P, i, j) : 0;
  bool isb = inb && B.bulk[k];
  int nb = __syncthreads_count(isb);
  if (nb == 0 || errored(B)) return;
  if (tid == 0) {
    atomicAdd(&B.ctr[C_UPD], (unsigned long long)nb);
    atomicAdd(&B.ctr[stage0 ? C_UPDB0 : C_UPDB1], (unsigned long long)nb);
  }
  const double* Qs = B.Q[sidx];
  const double* Qn = B.Q[nidx];
  // stage the tile + 3-cell frame: pure cells from Q, frame cells outside the
  // domain from the boundary states.  Every load of the thread's cells (and
  // of its own cell's Q^(s), Q^n for the update) is issued before any value
  // is used, so that their latencies overlap.
  constexpr int NS = (WX * WY + NT - 1) / NT;
  constexpr int NB = ((BX + 2) * (BY + 2) + NT - 1) / NT;
  int kk[NS];
  uint8_t ch[NS], oc[NS], bf[NB];
  bool inr[NS], ind[NS];
#pragma unroll
  for (int n = 0; n < NS; n++) {
    int q = tid + n * NT;
    int ci = i0 - 3 + q % WX, cj = j0 - 3 + q / WX;
    inr[n] = q < WX * WY && ci >= -H && ci < P.nx + H && cj >= -H && cj < P.ny + H;
    ind[n] = inr[n] && ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny;
    kk[n] = inr[n] ? cid(P, ci, cj) : 0;
    ch[n] = inr[n] ? B.chi[kk[n]] : 0;
    oc[n] = ind[n] ? B.occ[sidx][kk[n]] : 0;
  }
#pragma unroll
  for (int n = 0; n < NB; n++) {
    int q = tid + n * NT;
    int ci = i0 - 1 + q % (BX + 2), cj = j0 - 1 + q / (BX + 2);
    bool in = q < (BX + 2) * (BY + 2) && ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny;
    bf[n] = in ? B.bulk[cid(P, ci, cj)] : 0;
  }
  int m = isb ? B.chi[k] : 0;
  double U[NS][4];
#pragma unroll
  for (int n = 0; n < NS; n++) {
    size_t o = (size_t)ch[n] * 4 * P.NC + kk[n];
    bool has = (oc[n] >> ch[n]) & 1;
    if (ind[n]) {
      for (int v = 0; v < 4; v++) U[n][v] = has ? Qs[o + (size_t)v * P.NC] : 0.0;
    } else if (inr[n]) {
      for (int v = 0; v < 4; v++) U[n][v] = B.W[o + (size_t)v * P.NC];
    } else {
      U[n][0] = 1.0; U[n][1] = 0.0; U[n][2] = 0.0; U[n][3] = 1.0;
    }
  }
  size_t om = (size_t)m * 4 * P.NC + k;
  double qs_own[4], qn_own[4];
  for (int v = 0; v < 4; v++) {
    qs_own[v] = isb ? Qs[om + (size_t)v * P.NC] : 0.0;
    qn_own[v] = isb && !stage0 ? Qn[om + (size_t)v * P.NC] : 0.0;
  }
#pragma unroll
  for (int n = 0; n < NS; n++) {
    int q = tid + n * NT;
    if (q >= WX * WY) continue;
    double r_ = U[n][0], u_ = U[n][1], v_ = U[n][2], p_ = U[n][3];
    if (ind[n]) {
      Prim w = prim_from_U(U[n][0], U[n][1], U[n][2], U[n][3], eos_of(P, ch[n]));
      r_ = w.r; u_ = w.u; v_ = w.v; p_ = w.p;
    }
    int lx = q % WX, ly = q / WX;
    sm.W[0][ly][lx] = r_;
    sm.W[1][ly][lx] = u_;
    sm.W[2][ly][lx] = v_;
    sm.W[3][ly][lx] = p_;
    sm.chi[ly][lx] = ch[n];
  }
#pragma unroll
  for (int n = 0; n < NB; n++) {
    int q = tid + n * NT;
    if (q < (BX + 2) * (BY + 2)) sm.bulk[q / (BX + 2)][q % (BX + 2)] = bf[n];
  }
  __syncthreads();
  double lx = B.scal[S_LX], ly = B.scal[S_LY];
  // x-faces: face f is the left face of tile cell (f % (BX+1), f / (BX+1))
#pragma unroll 1
  for (int f = tid; f < NFX; f += NT) {
    double G[4];
    if (bulk_face<BX, BY, FLUX>(P, B, sm, 0, f % (BX + 1), f / (BX + 1), G))
      for (int v = 0; v < 4; v++) sm.F[v][f] = G[v];
  }
  __syncthreads();
  double acc[4];
  if (isb) {
    int fl = ty * (BX + 1) + tx, fr = fl + 1;
    for (int v = 0; v < 4; v++) acc[v] = lx * (sm.F[v][fl] - sm.F[v][fr]);
  }
  __syncthreads();
  // y-faces: face f is the bottom face of tile cell (f % BX, f / BX)
#pragma unroll 1
  for (int f = tid; f < NFY; f += NT) {
    double G[4];
    if (bulk_face<BX, BY, FLUX>(P, B, sm, 1, f % BX, f / BX, G))
      for (int v = 0; v < 4; v++) sm.F[v][f] = G[v];
  }
  __syncthreads();
  if (!isb) return;
  {
    Prim w;
    w.r = sm.W[0][ty + 3][tx + 3];
    w.u = sm.W[1][ty + 3][tx + 3];
    w.v = sm.W[2][ty + 3][tx + 3];
    w.p = sm.W[3][ty + 3][tx + 3];
    if (nonphys(w, P.pinf[m])) flag_error(P, B, i, j);
  }
  int fb = ty * BX + tx, ft = fb + BX;
  double* Qd = B.Q[didx];
  for (int v = 0; v < 4; v++) {
    double rhs = acc[v] + ly * (sm.F[v][fb] - sm.F[v][ft]);
    double qs = qs_own[v];
    double x = stage0 ? (qs + rhs) : (bcoef * qn_own[v] + ccoef * (qs + rhs));
    Qd[om + (size_t)v * P.NC] = x;
  }
  B.occ[didx][k] = (uint8_t)(1u << m);
}

// 1D bulk update of one tile of T = blockDim.x cells starting at i0, with a
// 3-cell frame staged in LDS; every thread of the workgroup must call it.
// LDS arrays are sized for T <= T1MAX.
constexpr int T1MAX = 1024;
struct Bulk1Smem {
  double W[3][T1MAX + 6];
  double F[3][T1MAX + 1];
  uint8_t chi[T1MAX + 6];
  uint8_t bulk[T1MAX + 2];
};
MMD void bulk1_tile(const Params& P, const Bufs& B, Bulk1Smem& S, int i0, int sidx,
                    int nidx, int didx, double bcoef, double ccoef, int stage0) {
  int T = blockDim.x, tid = threadIdx.x;
  int i = i0 + tid;
  bool inb = i < P.nx;
  int k = inb ? cid(P, i, 0) : 0;
  bool isb = inb && B.bulk[k];
  int nb = __syncthreads_count(isb);
  if (nb == 0 || errored(B)) return;  // uniform across the workgroup
  // updates of solved materials (an ambient that is not solved is copied)
  int nu = P.fs_on ? __syncthreads_count(isb && B.chi[k] != P.fs_mat) : nb;
  if (tid == 0) {
    atomicAdd(&B.ctr[C_UPD], (unsigned long long)nu);
    atomicAdd(&B.ctr[stage0 ? C_UPDB0 : C_UPDB1], (unsigned long long)nu);
  }
  const double* Qs = B.Q[sidx];
  for (int q = tid; q < T + 6; q += T) {
    int ci = i0 - 3 + q;
    double r_ = 1.0, u_ = 0.0, p_ = 1.0;
    uint8_t ch = 0;
    if (ci >= -H && ci < P.nx + H) {
      int kk = cid(P, ci, 0);
      ch = B.chi[kk];
      if (ci >= 0 && ci < P.nx) {
        size_t o = (size_t)ch * 3 * P.NC + kk;
        bool has = (B.occ[sidx][kk] >> ch) & 1;
        double U0 = has ? Qs[o] / 1.0 : 0.0, U1 = has ? Qs[o + P.NC] / 1.0 : 0.0,
               U3 = has ? Qs[o + 2 * (size_t)P.NC] / 1.0 : 0.0;
        Prim w = prim_from_U(U0, U1, 0.0, U3, eos_of(P, ch));
        r_ = w.r; u_ = w.u; p_ = w.p;
      } else {
        size_t o = (size_t)ch * 4 * P.NC + kk;
        r_ = B.W[o];
        u_ = B.W[o + P.NC];
        p_ = B.W[o + 3 * (size_t)P.NC];
      }
    }
    S.W[0][q] = r_;
    S.W[1][q] = u_;
    S.W[2][q] = p_;
    S.chi[q] = ch;
  }
  for (int q = tid; q < T + 2; q += T) {
    int ci = i0 - 1 + q;
    S.bulk[q] = (ci >= 0 && ci < P.nx) ? B.bulk[cid(P, ci, 0)] : 0;
  }
  __syncthreads();
  for (int f = tid; f < T + 1; f += T) {
    // face f: between tile cells f-1 and f
    if (!(S.bulk[f] || S.bulk[f + 1])) continue;
    int m = S.bulk[f + 1] ? S.chi[f + 3] : S.chi[f + 2];
    if (passive(P, m)) continue;  // no fluxes of an ambient that is not solved
    double pinf = P.pinf[m];
    const double* R0 = S.W[0];
    const double* U0 = S.W[1];
    const double* P0 = S.W[2];
    if (P.flux == FLUX_ROE) {
      Prim Ws[6];
      for (int q = 0; q < 6; q++) {
        Ws[q].r = R0[f + q];
        Ws[q].u = U0[f + q];
        Ws[q].v = 0.0;
        Ws[q].p = P0[f + q];
      }
      double G[4];
      if (!roe_face(Ws, true, eos_of(P, m), P.igm1[m], G)) atomicAdd(&B.ctr[C_POSFIX], 1ull);
      S.F[0][f] = G[0];
      S.F[1][f] = G[1];
      S.F[2][f] = G[3];
      continue;
    }
    Prim L, R;
    L.r = weno5(R0[f], R0[f + 1], R0[f + 2], R0[f + 3], R0[f + 4]);
    L.u = weno5(U0[f], U0[f + 1], U0[f + 2], U0[f + 3], U0[f + 4]);
    L.v = 0.0;
    L.p = weno5(P0[f], P0[f + 1], P0[f + 2], P0[f + 3], P0[f + 4]);
    R.r = weno5(R0[f + 5], R0[f + 4], R0[f + 3], R0[f + 2], R0[f + 1]);
    R.u = weno5(U0[f + 5], U0[f + 4], U0[f + 3], U0[f + 2], U0[f + 1]);
    R.v = 0.0;
    R.p = weno5(P0[f + 5], P0[f + 4], P0[f + 3], P0[f + 2], P0[f + 1]);
    if (!(L.r > 0.0) || !(R.r > 0.0) || !(L.p + pinf > 0.0) || !(R.p + pinf > 0.0)) {
      atomicAdd(&B.ctr[C_POSFIX], 1ull);
      L.r = R0[f + 2]; L.u = U0[f + 2]; L.p = P0[f + 2];
      R.r = R0[f + 3]; R.u = U0[f + 3]; R.p = P0[f + 3];
    }
    double G[4];
    hllc_flux(L, R, eos_of(P, m), P.igm1[m], G);
    S.F[0][f] = G[0];
    S.F[1][f] = G[1];
    S.F[2][f] = G[3];
  }
  __syncthreads();
  if (isb && passive(P, S.chi[tid + 3])) {
    // an ambient that is not solved: the stage leaves it as it is
    int m = S.chi[tid + 3];
    size_t o = (size_t)m * 3 * P.NC + k;
    for (int v = 0; v < 3; v++) B.Q[didx][o + (size_t)v * P.NC] = Qs[o + (size_t)v * P.NC];
    B.occ[didx][k] = (uint8_t)(1u << m);
  } else if (isb) {
    int m = S.chi[tid + 3];
    Prim w;
    w.r = S.W[0][tid + 3];
    w.u = S.W[1][tid + 3];
    w.v = 0.0;
    w.p = S.W[2][tid + 3];
    if (nonphys(w, P.pinf[m])) flag_error(P, B, i, 0);
    double lx = B.scal[S_LX], lv = B.scal[S_LV];
    size_t o = (size_t)m * 3 * P.NC + k;
    const double* Qn = B.Q[nidx];
    double* Qd = B.Q[didx];
    for (int v = 0; v < 3; v++) {
      double rhs = lx * (S.F[v][tid] - S.F[v][tid + 1]);
      if (P.coord == 1) {
        // cylindrical: face areas r_{i-1/2}, r_{i+1/2} per volume r_i dx,
        // and the geometric source alpha p / r_i of the radial momentum
        double ri = rad(P, i + 0.5);
        rhs = lx * (S.F[v][tid] * rad(P, i) - S.F[v][tid + 1] * rad(P, i + 1)) / ri;
        if (v == 1) rhs = rhs + B.scal[S_DT] * (1.0 * w.p / ri);
      }
      rhs = rhs + lv * 0.0;
      double qs = Qs[o + (size_t)v * P.NC];
      double x = stage0 ? (qs + rhs) : (bcoef * Qn[o + (size_t)v * P.NC] + ccoef * (qs + rhs));
      Qd[o + (size_t)v * P.NC] = x;
    }
    B.occ[didx][k] = (uint8_t)(1u << m);
  }
  __syncthreads();  // the LDS tile is reused by the next call
}

constexpr int T1 = 256;
__global__ void __launch_bounds__(256)
k_flux_bulk1(Params P, Bufs B, int sidx, int nidx, int didx, double bcoef,
             double ccoef, int stage0) {
  __shared__ Bulk1Smem S;
  bulk1_tile(P, B, S, blockIdx.x * blockDim.x, sidx, nidx, didx, bcoef, ccoef, stage0);
}

// ---------------------------------------------------------------------------
// Level-set stage (Sec. 2.2): construct, HJ-WENO5 upwind, RK, reconstruct
// ---------------------------------------------------------------------------
template <int D>
MMD double hj_deriv(const Params& P, const Bufs& B, int r, int i, int j,
                    int dir, double vel) {
  double d[6];
  double ih = dir == 0 ? P.idx : P.idy;
  for (int q = 0; q < 6; q++) {
    int o = q - 2;
    int k1 = dir == 0 ? cid(P, i + o, j) : cid(P, i, j + o);
    int k0 = dir == 0 ? cid(P, i + o - 1, j) : cid(P, i, j + o - 1);
    d[q] = (lsv(B.phi, B.chi, r, k1) - lsv(B.phi, B.chi, r, k0)) * ih;
  }
  if (vel > 0.0) return weno5(d[0], d[1], d[2], d[3], d[4]);
  if (vel < 0.0) return weno5(d[5], d[4], d[3], d[2], d[1]);
  return 0.0;
}

template <int D>
MMD void b_ls(const Params& P, const Bufs& B, int i, int j, double bcoef, double ccoef) {
  int k = cid(P, i, j);
  (void)k;
  if (errored(B) || B.dls[k] > 3) return;
  double dt = B.scal[S_DT];
  double best = 0.0;
  int br = -1;
  unsigned xs = B.xs[k];
  for (int r = 0; r < P.M; r++) {
    if (!((xs >> r) & 1)) continue;
    double gx = hj_deriv<D>(P, B, r, i, j, 0, B.vx[k]);
    double adv = B.vx[k] * gx;
    if (D == 2) {
      double gy = hj_deriv<D>(P, B, r, i, j, 1, B.vy[k]);
      adv = adv + B.vy[k] * gy;
    }
    double val = lsv(B.phi, B.chi, r, k) - dt * adv;
    double nv = bcoef * lsv(B.phin, B.chin, r, k) + ccoef * val;
    if (br < 0 || nv > best) {
      best = nv;
      br = r;
    }
  }
  double a = fabs(best);
  B.ptmp[k] = a < P.bls ? a : P.bls;
  B.ctmp[k] = (uint8_t)br;
}
template <int D>
MMD void b_ls_commit(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  (void)k;
  if (errored(B) || B.dls[k] > 3) return;
  B.phi[k] = B.ptmp[k];
  B.chi[k] = B.ctmp[k];
}

// ---------------------------------------------------------------------------
// Mixing (Sec. 2.3.2, after each sub-step): exchanges from sources, then a
// gather that applies them in place
// ---------------------------------------------------------------------------
// loadQ with the word read in any case (k in range), then chosen
template <int D>
MMD double loadQ_u(const Params& P, const double* Q, const uint8_t* occ, int r, int v, int k) {
  int vv = D == 1 && v == 3 ? 2 : v;
  double q = Q[((size_t)r * (D + 2) + vv) * P.NC + k];
  bool has = (occ[k] >> r) & 1;
  return has && !(D == 1 && v == 2) ? q : 0.0;
}
// alpha_at with every word read in any case (k in range), then chosen
MMD double alpha_u(const Params& P, const Bufs& B, int r, int k) {
  uint8_t c = B.cut[k], h = B.chi[k];
  double a = B.al[(size_t)r * P.NC + k];
  return c ? a : (h == r ? 1.0 : 0.0);
}
template <int D>
MMD void b_mix1(const Params& P, const Bufs& B, int i, int j, int didx, uint32_t stamp,
                int r0, int r1) {
  int k = cid(P, i, j);
  (void)k;
  if (errored(B)) return;
  const double* Q = B.Q[didx];
  const uint8_t* occ = B.occ[didx];
  uint8_t own = (uint8_t)(1u << B.chi[k]);
  if (!B.cut[k] && occ[k] == own) return;
  double amix = P.amix;
  // neighbour n = 3 (dj + 1) + di + 1 (4 is the cell itself; 1D: row dj = 0)
  constexpr int NN = 9;
  int kn[NN];
  bool inn[NN];
  for (int dj = -1; dj <= 1; dj++)
    for (int di = -1; di <= 1; di++) {
      int n = 3 * (dj + 1) + di + 1;
      bool row = D == 2 || dj == 0;
      kn[n] = row ? cid(P, i + di, j + dj) : k;
      inn[n] = row && interior(P, i + di, j + dj);
    }
  uint8_t chk = B.chi[k];
  // cylindrical: volumes and contents carry the cells' radii (the exchange
  // is of content: alpha r and Q r in place of alpha and Q)
  bool cyl = D == 1 && P.coord == 1;
  double rs = cyl ? rad(P, i + 0.5) : 1.0;
  for (int r = r0; r < r1; r++) {
    if (passive(P, r)) continue;  // an ambient that is not solved
    // every load of this material that does not depend on a decision below,
    // issued together: the cell's volume fraction and state, the level set
    // of the four face neighbours, volume fraction and indicator of all eight
    double as = alpha_u(P, B, r, k);
    double qk[4];
    for (int v = 0; v < 4; v++) qk[v] = loadQ_u<D>(P, Q, occ, r, v, k);
    double an[NN];
    uint8_t hn[NN];
    double pn[NN];
    for (int n = 0; n < NN; n++) {
      an[n] = alpha_u(P, B, r, kn[n]);
      hn[n] = B.chi[kn[n]];
      pn[n] = B.phi[kn[n]];
    }
    // a part of the cell's own material with a volume fraction but nothing
    // in it (left so by a move between materials) is filled like a new
    // cell; so is a part with 0 < alpha < 1 and no mass (a partial density
    // of zero or roundoff of either sign: an interface that crossed a face
    // that had no aperture yet for this material)
    bool nz = false;
    for (int v = 0; v < 4; v++)
      if (qk[v] != 0.0) nz = true;
    bool nomass = !nz || (!(qk[0] > 0.0) && as < 1.0);
    if (!(as < amix) && chk == r && !(nomass && as > 0.0)) continue;
    if (!(as > 0.0) && !nz) continue;
    wave_count(&B.ctr[C_MIXSRC], 1);
    auto lsn = [&](int n) { return hn[n] == r ? pn[n] : -pn[n]; };
    double gx = lsn(5) - lsn(3);
    double gy = D == 2 ? lsn(7) - lsn(1) : 0.0;
    int sx = gx > 0.0 ? 1 : (gx < 0.0 ? -1 : 0);
    int sy = gy > 0.0 ? 1 : (gy < 0.0 ? -1 : 0);
    int tn[3] = {-1, -1, -1};
    double w[3] = {0.0, 0.0, 0.0};
    auto eligible = [&](int n) -> bool { return inn[n] && an[n] >= amix && hn[n] == r; };
    int nx_ = 4 + sx, ny_ = 4 + 3 * sy, nxy = 4 + sx + 3 * sy;
    if (sx != 0 && eligible(nx_)) {
      tn[0] = nx_;
      w[0] = gx * gx * an[nx_];
    }
    if (sy != 0 && eligible(ny_)) {
      tn[1] = ny_;
      w[1] = gy * gy * an[ny_];
    }
    if (sx != 0 && sy != 0 && eligible(nxy)) {
      tn[2] = nxy;
      w[2] = fabs(gx * gy) * an[nxy];
    }
    double wsum = (w[0] + w[1]) + w[2];
    double beta[3] = {0.0, 0.0, 0.0};
    if (wsum > 0.0) {
      for (int q = 0; q < 3; q++)
        if (w[q] > 0.0)
          beta[q] = w[q] / wsum;
        else
          tn[q] = -1;
    } else {
      tn[0] = tn[1] = tn[2] = -1;
      double bestA = -1.0;
      int bt = -1;
      for (int dj = -(D == 2); dj <= (D == 2); dj++)
        for (int di = -1; di <= 1; di++) {
          if (di == 0 && dj == 0) continue;
          int n = 3 * (dj + 1) + di + 1;
          if (eligible(n) && an[n] > bestA) {
            bestA = an[n];
            bt = n;
          }
        }
      if (bt < 0) {
        // stranded: marked for the absorb pass (after every material's
        // exchanges); a fragment of the cell's own material also decides
        // the cell's new material, the other of largest volume fraction
        B.strStamp[(size_t)r * P.NC + k] = stamp;
        if (chk == r) {
          double ba = 0.0;
          int to = -1;
          for (int m = 0; m < P.M; m++) {
            double am = alpha_u(P, B, m, k);
            if (m != r && am > ba) {
              ba = am;
              to = m;
            }
          }
          if (to >= 0) {
            B.rlTo[k] = (uint8_t)to;
            B.rlStamp[k] = stamp;
          }
        }
        if (B.abList && atomicExch(&B.abMark[k], stamp) != stamp) {
          unsigned long long at = atomicAdd(&B.ctr[C_NAB], 1ull);
          B.abList[at] = k;
        }
        continue;
      }
      tn[0] = bt;
      beta[0] = 1.0;
    }
    int tk[3], last = -1;
    for (int q = 0; q < 3; q++) tk[q] = tn[q] >= 0 ? kn[tn[q]] : -1;
    // states of the targets (needed only where the cell holds material r)
    double qt[3][4];
    for (int q = 0; q < 3; q++)
      for (int v = 0; v < 4; v++)
        qt[q][v] = as > 0.0 && tk[q] >= 0 ? loadQ_u<D>(P, Q, occ, r, v, tk[q]) : 0.0;
    for (int q = 0; q < 3; q++) {
      B.mixT[((size_t)r * 3 + q) * P.NC + k] = tk[q];
      if (tk[q] >= 0) {
        last = q;
        B.tgtStamp[(size_t)r * P.NC + tk[q]] = stamp;
      }
    }
    B.srcStamp[(size_t)r * P.NC + k] = stamp;
    for (int v = 0; v < 4; v++) {
      // a vanishing cell sends its content (Q r in cylindrical geometry)
      double Qs = qk[v];
      if (cyl && !(as > 0.0)) Qs = Qs * rs;
      double acc = Qs;
      for (int q = 0; q < 3; q++) {
        if (tk[q] < 0) continue;
        double m;
        if (as > 0.0) {
          double at2 = an[tn[q]];
          double Qt = qt[q][v];
          if (cyl) {
            double rt = rad(P, (i + (tn[q] % 3 - 1)) + 0.5);
            double aS = as * rs, aT = at2 * rt, qS = Qs * rs, qT = Qt * rt;
            m = beta[q] * ((aS * qT - aT * qS) / (aS + aT));
          } else {
            m = beta[q] * ((as * Qt - at2 * Qs) / (as + at2));
          }
        } else {
          m = q == last ? -acc : -(beta[q] * Qs);
          acc = acc + m;
        }
        B.mixM[(((size_t)r * 3 + q) * 4 + v) * P.NC + k] = m;
      }
    }
  }
}

// Stranded mixing sources of cell k (after every material's exchanges): the
// cell takes the new material decided by a stranded fragment of its own
// material, then each stranded material's conserved quantities join the
// cell's material (a stranded source of that material itself stays), in
// material order.  Returns whether the cell was relabelled.
template <int D>
MMD bool b_absorb(const Params& P, const Bufs& B, int k, int didx, uint32_t stamp) {
  double* Q = B.Q[didx];
  uint8_t* occp = B.occ[didx];
  bool rel = B.rlStamp[k] == stamp;
  int to = rel ? (int)B.rlTo[k] : (int)B.chi[k];
  unsigned occ = occp[k];
  for (int r = 0; r < P.M; r++) {
    if (B.strStamp[(size_t)r * P.NC + k] != stamp) continue;
    if (r == to) {
      atomicAdd(&B.ctr[C_STRANDED], 1ull);
      continue;
    }
    bool nz = false;
    for (int v = 0; v < 4; v++) {
      if (D == 1 && v == 2) continue;
      double q = loadQ<D>(P, Q, (const uint8_t*)occp, r, v, k);
      double t = loadQ<D>(P, Q, (const uint8_t*)occp, to, v, k);
      double n = t + q;
      storeQ<D>(P, Q, to, v, k, n);
      storeQ<D>(P, Q, r, v, k, 0.0);
      if (n != 0.0) nz = true;
    }
    // occupancy read by loadQ above: update it only after both loads
    occ &= ~(1u << r);
    if (nz) occ |= 1u << to;
    occp[k] = (uint8_t)occ;
    atomicAdd(&B.ctr[C_ABSORB], 1ull);
  }
  if (rel) {
    B.chi[k] = (uint8_t)to;
    atomicAdd(&B.ctr[C_RELABEL], 1ull);
  }
  return rel;
}

// y sides of the level-set frame: columns i in [-H, nx+H), frame cell t
MMD void b_bc_ls_y(const Params& P, int t, double* phi, uint8_t* chi) {
  int i = t / (2 * H) - H, q = t % (2 * H);
  int j, sj;
  if (q < H) {
    j = -1 - q;
    sj = src_lo(j, P.bc[2]);
  } else {
    j = P.ny + (q - H);
    sj = src_hi(j, P.ny, P.bc[3]);
  }
  int k = cid(P, i, j), ks = cid(P, i, sj);
  phi[k] = phi[ks];
  chi[k] = chi[ks];
}

// ---------------------------------------------------------------------------
// Interface scale separation (Sec. 2.3.3), after every time step when
// enabled: oddball cells (cut cells whose material has no cell crossed by its
// eps-inner contour, eps = 0.75 h, in the 3 x 3 block) go to the other
// material of largest volume fraction, provided that one is resolved there
// (has such a cell in the block); their distance becomes |d_min - eps| with
// d_min the distance to the eps-grown boundary of the new material, found
// from the crossed cells within 3 cells; conserved quantities follow.
// ---------------------------------------------------------------------------
// does the contour phi^r = off cross cell (i, j)?  Centre and four corners
// (means of the four cells around each corner) on both sides of off
template <int D>
MMD bool crosses(const Params& P, const Bufs& B, int r, int i, int j, double off) {
  double c = lsv(B.phi, B.chi, r, cid(P, i, j)) - off;
  double mn = c, mx = c;
  for (int cj = 0; cj < (D == 2 ? 2 : 1); cj++)
    for (int ci = 0; ci < 2; ci++) {
      int x0 = i - 1 + ci, y0 = D == 2 ? j - 1 + cj : 0;
      double v;
      if (D == 2)
        v = (lsv(B.phi, B.chi, r, cid(P, x0, y0)) + lsv(B.phi, B.chi, r, cid(P, x0 + 1, y0)) +
             lsv(B.phi, B.chi, r, cid(P, x0, y0 + 1)) +
             lsv(B.phi, B.chi, r, cid(P, x0 + 1, y0 + 1))) * 0.25 - off;
      else
        v = (lsv(B.phi, B.chi, r, cid(P, x0, 0)) + lsv(B.phi, B.chi, r, cid(P, x0 + 1, 0))) * 0.5 - off;
      if (v < mn) mn = v;
      if (v > mx) mx = v;
    }
  return mn <= 0.0 && mx > 0.0;
}
template <int D>
MMD bool resolved_near(const Params& P, const Bufs& B, int r, int i, int j, double eps) {
  for (int dj = -(D == 2); dj <= (D == 2); dj++)
    for (int di = -1; di <= 1; di++)
      if (crosses<D>(P, B, r, i + di, j + dj, eps)) return true;
  return false;
}
// oddball test of cell (i, j); an oddball cell is listed with its new
// material and distance (the fields themselves change only in k_ss_apply)
template <int D>
MMD void b_ss_detect(const Params& P, const Bufs& B, int i, int j) {
  int k = cid(P, i, j);
  int c1 = B.chi[k];
  if (!(alpha_u(P, B, c1, k) < 1.0)) return;
  double eps = 0.75 * P.h;
  if (resolved_near<D>(P, B, c1, i, j, eps)) return;
  int c2 = -1;
  double ba = 0.0;
  for (int r = 0; r < P.M; r++) {
    double a = alpha_u(P, B, r, k);
    if (r != c1 && a > ba) {
      ba = a;
      c2 = r;
    }
  }
  if (c2 < 0 || !resolved_near<D>(P, B, c2, i, j, eps)) return;
  double dmin = -1.0;
  int R = D == 2 ? 3 : 0;
  for (int dj = -R; dj <= R; dj++)
    for (int di = -3; di <= 3; di++) {
      int ii = i + di, jj = j + dj;
      if (ii < -1 || ii > P.nx || (D == 2 && (jj < -1 || jj > P.ny))) continue;
      if (!crosses<D>(P, B, c2, ii, jj, -eps)) continue;
      int k0 = cid(P, ii, jj);
      double gx = lsv(B.phi, B.chi, c2, cid(P, ii + 1, jj)) - lsv(B.phi, B.chi, c2, cid(P, ii - 1, jj));
      double gy = D == 2 ? lsv(B.phi, B.chi, c2, cid(P, ii, jj + 1)) -
                               lsv(B.phi, B.chi, c2, cid(P, ii, jj - 1))
                         : 0.0;
      double gn = sqrt(gx * gx + gy * gy);
      if (!(gn > 0.0)) continue;
      double f = lsv(B.phi, B.chi, c2, k0) + eps;
      double ex = di * P.dx - f * (gx / gn), ey = dj * P.dy - f * (gy / gn);
      double d = sqrt(ex * ex + ey * ey);
      if (dmin < 0.0 || d < dmin) dmin = d;
    }
  double np = B.phi[k];
  if (dmin >= 0.0) {
    double a = fabs(dmin - eps);
    np = a < P.bls ? a : P.bls;
  }
  B.ssTo[k] = (uint8_t)c2;
  B.ssPhi[k] = np;
  unsigned long long at = atomicAdd(&B.ctr[C_NSS], 1ull);
  B.ssList[at] = k;
  atomicAdd(&B.ctr[C_ODDBALL], 1ull);
}
// an oddball cell takes its new material and distance; the conserved
// quantities of its old material join the new one
template <int D>
MMD void b_ss_apply(const Params& P, const Bufs& B, int k, int didx) {
  double* Q = B.Q[didx];
  uint8_t* occp = B.occ[didx];
  int c1 = B.chi[k], c2 = B.ssTo[k];
  unsigned occ = occp[k];
  bool nz = false;
  for (int v = 0; v < 4; v++) {
    if (D == 1 && v == 2) continue;
    double q = loadQ<D>(P, Q, (const uint8_t*)occp, c1, v, k);
    double t = loadQ<D>(P, Q, (const uint8_t*)occp, c2, v, k);
    double n = t + q;
    storeQ<D>(P, Q, c2, v, k, n);
    storeQ<D>(P, Q, c1, v, k, 0.0);
    if (n != 0.0) nz = true;
  }
  occ &= ~(1u << c1);
  if (nz) occ |= 1u << c2;
  occp[k] = (uint8_t)occ;
  B.chi[k] = (uint8_t)c2;
  B.phi[k] = B.ssPhi[k];
}
template <int D>
// materials r0 <= r < r1 of cell (i, j); with word_occ the occupancy bits
// are set and cleared by atomics on the aligned 32-bit word that holds the
// cell's byte (other materials of the cell may be updated at the same time)
MMD void b_mix2(const Params& P, const Bufs& B, int i, int j, int didx, uint32_t stamp,
                int r0, int r1, bool word_occ) {
  int k = cid(P, i, j);
  double* Q = B.Q[didx];
  uint8_t* occp = B.occ[didx];
  unsigned occ = occp[k];
  bool touched = false;
  // cylindrical: exchanges are of content, the cell's state changes by
  // them over its radius
  bool cyl = D == 1 && P.coord == 1;
  double rc = cyl ? rad(P, i + 0.5) : 1.0;
  for (int r = r0; r < r1; r++) {
    bool src = B.srcStamp[(size_t)r * P.NC + k] == stamp;
    bool tgt = B.tgtStamp[(size_t)r * P.NC + k] == stamp;
    if (!src && !tgt) continue;
    touched = true;
    // exchanges that apply to this cell: its own (as a source) or those its
    // neighbours sent it (as a target); at most one slot per neighbour
    const double* mrow[3][3];
    for (int dj = 0; dj < 3; dj++)
      for (int di = 0; di < 3; di++) mrow[dj][di] = nullptr;
    if (src) {
      for (int q = 0; q < 3; q++)
        if (B.mixT[((size_t)r * 3 + q) * P.NC + k] >= 0)
          mrow[0][q] = B.mixM + ((size_t)r * 3 + q) * 4 * P.NC + k;
    } else {
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) {
          int ii = i + di, jj = j + dj;
          if ((di == 0 && dj == 0) || (D == 1 && dj != 0) || !interior(P, ii, jj)) continue;
          int n = cid(P, ii, jj);
          if (B.srcStamp[(size_t)r * P.NC + n] != stamp) continue;
          for (int q = 0; q < 3; q++)
            if (B.mixT[((size_t)r * 3 + q) * P.NC + n] == k)
              mrow[dj + 1][di + 1] = B.mixM + ((size_t)r * 3 + q) * 4 * P.NC + n;
        }
    }
    double nq[4];
    bool nz = false;
    for (int v = 0; v < 4; v++) {
      double q0 = loadQ<D>(P, Q, (const uint8_t*)occp, r, v, k);
      size_t ov = (size_t)v * P.NC;
      if (src) {
        for (int q = 0; q < 3; q++)
          if (mrow[0][q]) q0 = cyl ? q0 + mrow[0][q][ov] / rc : q0 + mrow[0][q][ov];
      } else {
        double row[3];
        for (int dj = 0; dj < 3; dj++) {
          double a0 = mrow[dj][0] ? mrow[dj][0][ov] : 0.0;
          double a1 = mrow[dj][1] ? mrow[dj][1][ov] : 0.0;
          double a2 = mrow[dj][2] ? mrow[dj][2][ov] : 0.0;
          row[dj] = (a0 + a2) + a1;
        }
        q0 = cyl ? q0 - ((row[0] + row[2]) + row[1]) / rc : q0 - ((row[0] + row[2]) + row[1]);
      }
      nq[v] = q0;
      if (q0 != 0.0 && !(D == 1 && v == 2)) nz = true;
    }
    if (nz) {
      for (int v = 0; v < 4; v++) storeQ<D>(P, Q, r, v, k, nq[v]);
      occ |= 1u << r;
    } else {
      occ &= ~(1u << r);
    }
    if (word_occ) {
      unsigned* w = (unsigned*)(occp + (k & ~3));
      unsigned bit = 1u << (8 * (k & 3) + r);
      if (nz)
        atomicOr(w, bit);
      else
        atomicAnd(w, ~bit);
    }
  }
  if (touched && !word_occ) occp[k] = (uint8_t)occ;
}

// ---------------------------------------------------------------------------
// Output packing: interior Q [M][NV][ny][nx], alpha, phi, chi
// ---------------------------------------------------------------------------
template <int D>
MMD void b_pack(const Params& P, const Bufs& B, int i, int j, int sidx, double* Qo, double* ao,
                       double* po, int32_t* co) {
  int k = cid(P, i, j);
  (void)k;
  size_t plane = (size_t)P.nx * P.ny, q = (size_t)j * P.nx + i;
  for (int r = 0; r < P.M; r++) {
    if (Qo) {
      Qo[((size_t)r * (D + 2) + 0) * plane + q] = loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, 0, k);
      Qo[((size_t)r * (D + 2) + 1) * plane + q] = loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, 1, k);
      if (D == 2)
        Qo[((size_t)r * (D + 2) + 2) * plane + q] = loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, 2, k);
      Qo[((size_t)r * (D + 2) + D + 1) * plane + q] = loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, 3, k);
    }
    if (ao) ao[(size_t)r * plane + q] = alpha_at<D>(P, B, r, k);
  }
  if (po) po[q] = B.phi[k];
  if (co) co[q] = B.chi[k];
}
template <int D>
__global__ void k_pack(Params P, Bufs B, int sidx, double* Qo, double* ao,
                       double* po, int32_t* co) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  b_pack<D>(P, B, i, j, sidx, Qo, ao, po, co);
}

// initial level set from an interior [ny][nx] array
template <int D>
MMD void b_load_ls(const Params& P, const Bufs& B, int i, int j, const double* phi,
                   const int32_t* chi) {
  int k = cid(P, i, j);
  size_t q = (size_t)j * P.nx + i;
  double p = phi[q];
  int32_t c = chi[q];
  if (c < 0 || c >= P.M || !(p >= 0.0)) {
    // counted (the call then fails); the stored values stay in range
    atomicAdd(&B.ctr[C_BADIN], 1ull);
    c = 0;
    p = 0.0;
  }
  B.phi[k] = p;
  B.chi[k] = (uint8_t)c;
}
__global__ void k_load_ls(Params P, Bufs B, const double* phi, const int32_t* chi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= P.nx || j >= P.ny) return;
  b_load_ls<2>(P, B, i, j, phi, chi);
}


// ---------------------------------------------------------------------------
// General update of the listed (non-bulk) cells: one lane per face of a cell
// computes that face's aperture-weighted flux for every material; the lane
// of the left face then combines them into the stage update.
// ---------------------------------------------------------------------------
template <int D, int FLUX = -1>
MMD void flux_list_blocks(const Params& P, const Bufs& B, int sidx, int nidx, int didx,
                          double bcoef, double ccoef, int bx, int nbx) {
  // threads are (cell, material, face): the aperture-scaled flux of one
  // material across one face of one listed cell goes through LDS to the
  // thread that combines the faces of (cell, material) into its update
  constexpr int FPC = D == 2 ? 4 : 2;  // faces per cell
  __shared__ double sF[256][4];
  __shared__ unsigned sOcc[256];
  const int tpc = FPC * P.M, cpb = 256 / tpc;  // threads and cells per block
  int tid = threadIdx.x, c = tid / tpc, rem = tid % tpc, r = rem / FPC, f = rem % FPC;
  int nb = (int)B.ctr[C_NBAND];
  if (errored(B)) return;
  const double* Qs = B.Q[sidx];
  const uint8_t* os = B.occ[sidx];
  for (int base = bx * cpb; base < nb; base += nbx * cpb) {
    int idx = base + c;
    bool act = c < cpb && idx < nb;
    int k = act ? B.blist[idx] : 0;
    int i = k % P.NX - H, j = k / P.NX - P.HY;
    if (tid < cpb) sOcc[tid] = 0;
    if (act) {
      // face f: 0 low x, 1 high x, 2 low y, 3 high y
      int dir = f >> 1, fi = f == 0 ? i - 1 : i, fj = f == 2 ? j - 1 : j;
      bool count = f == 0 ? i == 0 : (f == 2 ? j == 0 : true);
      // no fluxes of an ambient that is not solved
      double A = passive(P, r) ? 0.0 : apd(P, B, r, fi, fj, dir);
      double F[4] = {0.0, 0.0, 0.0, 0.0};
      if (A > 0.0) face_flux<D, FLUX>(P, B, Qs, os, r, fi, fj, dir, count, F);
      for (int v = 0; v < 4; v++) sF[tid][v] = A > 0.0 ? A * F[v] : 0.0;
    }
    __syncthreads();
    if (act && f == 0) {
      const double* Qn = B.Q[nidx];
      const uint8_t* on = B.occ[nidx];
      double lx = B.scal[S_LX], ly = B.scal[S_LY], lv = B.scal[S_LV];
      bool pas = passive(P, r);
      // non-cut cells are real cells of their material: checked by that
      // material's thread
      if (!B.cut[k] && r == B.chi[k] && !pas) {
        bool vd;
        Prim w = Wget<D>(P, B, Qs, os, r, i, j, vd);
        if (nonphys(w, P.pinf[r])) flag_error(P, B, i, j);
      }
      // cylindrical: radii of the faces and the centre, and the state whose
      // pressure gives the geometric source
      double rl = 0.0, rr = 0.0, ri = 1.0, src = 0.0;
      bool hsrc = false;
      if (D == 1 && P.coord == 1 && !pas) {
        rl = rad(P, i);
        rr = rad(P, i + 1);
        ri = rad(P, i + 0.5);
        Prim w = Wget<D>(P, B, Qs, os, r, i, j, hsrc);
        if (hsrc) src = B.scal[S_DT] * (alpha_at<D>(P, B, r, k) * w.p / ri);
      }
      double out[4];
      bool nz = false;
      for (int v = 0; v < 4; v++) {
        if (D == 1 && v == 2) {
          out[v] = 0.0;
          continue;
        }
        double qs = loadQ<D>(P, Qs, os, r, v, k);
        if (pas) {
          // an ambient that is not solved: the stage leaves it as it is
          out[v] = qs;
          if (qs != 0.0) nz = true;
          continue;
        }
        double rhs = lx * (sF[tid][v] - sF[tid + 1][v]);
        if (D == 1 && P.coord == 1) {
          rhs = lx * (sF[tid][v] * rl - sF[tid + 1][v] * rr) / ri;
          if (v == 1 && hsrc) rhs = rhs + src;
        }
        if (D == 2) rhs = rhs + ly * (sF[tid + 2][v] - sF[tid + FPC - 1][v]);
        double X = B.cut[k] ? B.X[((size_t)r * 4 + v) * P.NC + k] : 0.0;
        rhs = rhs + lv * X;
        double qn = loadQ<D>(P, Qn, on, r, v, k);
        double x = bcoef * qn + ccoef * (qs + rhs);
        out[v] = x;
        if (x != 0.0) nz = true;
      }
      if (nz) {
        atomicOr(&sOcc[c], 1u << r);
        for (int v = 0; v < 4; v++) storeQ<D>(P, B.Q[didx], r, v, k, out[v]);
      }
      wave_count(&B.ctr[C_UPD], alpha_at<D>(P, B, r, k) > 0.0 && !pas ? 1u : 0u);
    }
    __syncthreads();
    if (tid < cpb && base + tid < nb) B.occ[didx][B.blist[base + tid]] = (uint8_t)sOcc[tid];
    __syncthreads();
  }
}

// one ghost-extension sweep over the queued (cell, material) pairs
template <int D>
__global__ void __launch_bounds__(256) k_ext_list(Params P, Bufs B, int sidx, int sweep) {
  int n = (int)B.ctr[C_NGHOST];
  if (errored(B)) return;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    int e = B.glist[q];
    int k = e >> 3, r = e & 7;
    if (B.Wit[(size_t)r * P.NC + k] != 0) continue;
    ext_one<D>(P, B, k % P.NX - H, k / P.NX - P.HY, r, sidx, sweep);
  }
}

// ---------------------------------------------------------------------------
// Active tiles.  Work near interfaces touches a few percent of the cells;
// after each level-set update the tiles (16 x 16 cells in 2D, 256 in 1D)
// that hold, within one cell of the tile, a cell within 8 of a cut cell,
// within 12 of the level-set band, or a material state other than its own,
// are listed, and the near-interface kernels walk that list.  Every cell
// those kernels act on lies in a listed tile, so results do not change.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Conservation book-keeping (Eq. discretized_equ: a material's total changes
// only by the fluxes through the domain boundary and by its exchange term):
// per stage, the net boundary inflow and the exchange total of every
// material and component, weighted by the stage's share of the full step
// and added to compensated (Neumaier) running sums; on demand, the sums of
// Q.  Partial sums are formed per workgroup over fixed index ranges and
// combined in a fixed order, so the results do not depend on scheduling.
// ---------------------------------------------------------------------------
MMD double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// sums of v[0..7] over the workgroup (blockDim.x a multiple of 64, at most
// 1024) in a fixed order; the results are left in thread 0's v.  red holds
// 8 doubles per wavefront.
MMD void block_sum8(double v[8], double* red) {
  int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int x = 0; x < 8; x++) v[x] = wave_sum(v[x]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int x = 0; x < 8; x++) red[w * 8 + x] = v[x];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int x = 0; x < 8; x++) {
      double t = 0.0;
      for (int q = 0; q < nw; q++) t += red[q * 8 + x];
      v[x] = t;
    }
}

MMD void neumaier_add(double* sum, double* comp, double x) {
  double t = *sum + x;
  if (fabs(*sum) >= fabs(x))
    *comp += (*sum - t) + x;
  else
    *comp += (x - t) + *sum;
  *sum = t;
}

// add one stage's totals of material r (t[0..3] boundary inflow, t[4..7]
// exchange), weighted by the stage's share w of the step
MMD void cons_accumulate(const Bufs& B, int r, const double t[8], double w) {
  for (int v = 0; v < 4; v++) {
    neumaier_add(&B.cons[(CONS_BND * MAXM + r) * 4 + v], &B.cons[(CONS_BNDC * MAXM + r) * 4 + v],
                 w * t[v]);
    neumaier_add(&B.cons[(CONS_X * MAXM + r) * 4 + v], &B.cons[(CONS_XC * MAXM + r) * 4 + v],
                 w * t[4 + v]);
  }
}

// flux term of one domain-boundary face of material r: side 0 is the low
// face of row/column q (x-face i-1/2 of row q, or y-face j-1/2 of column q),
// side 1 the high face; out = A F (0 where A = 0)
template <int D, int FLUX = -1>
MMD void cons_face(const Params& P, const Bufs& B, const double* Qs, const uint8_t* os, int r,
                   int dir, int q, int side, double out[4]) {
  double F[4] = {0, 0, 0, 0};
  double A;
  if (dir == 0) {
    int i = side == 0 ? -1 : P.nx - 1;
    A = apx<D>(P, B, r, i, q);
    if (A > 0.0) face_flux<D, FLUX>(P, B, Qs, os, r, i, q, 0, false, F);
  } else {
    int j = side == 0 ? -1 : P.ny - 1;
    A = apy(P, B, r, q, j);
    if (A > 0.0) face_flux<D, FLUX>(P, B, Qs, os, r, q, j, 1, false, F);
  }
  for (int v = 0; v < 4; v++) out[v] = A > 0.0 ? A * F[v] : 0.0;
}

// net inflow of material r through the two boundary faces of row q
// (q < ny) or of column q - ny (2D, ny <= q < ny + nx)
template <int D>
MMD void cons_boundary(const Params& P, const Bufs& B, const double* Qs, const uint8_t* os,
                       int r, long q, double out[4]) {
  int dir = q < P.ny ? 0 : 1;
  int qq = dir == 0 ? (int)q : (int)(q - P.ny);
  double lo[4], hi[4];
  cons_face<D>(P, B, Qs, os, r, dir, qq, 0, lo);
  cons_face<D>(P, B, Qs, os, r, dir, qq, 1, hi);
  double l = dir == 0 ? B.scal[S_LX] : B.scal[S_LY];
  for (int v = 0; v < 4; v++) out[v] = l * (lo[v] - hi[v]);
}

MMD int cons_rows(const Params& P) { return P.dim == 2 ? P.ny + P.nx : 1; }

// Workgroup x of material r (x in [0, nbb + ncb)): x < nbb takes 128
// boundary rows/columns (one thread per boundary face), the others CONS_CH
// cells each (exchange).  Partials cpart[x][r][8]: net boundary inflow,
// exchange.
constexpr int CONS_ROWS = 128;

template <int D, int FLUX = -1>
MMD void cons_part_block(const Params& P, const Bufs& B, int sidx, int nbb, int bx, int r) {
  __shared__ double red[4 * 8];
  __shared__ double face[CONS_ROWS][2][4];
  const double* Qs = B.Q[sidx];
  const uint8_t* os = B.occ[sidx];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double* part = B.cpart + ((size_t)bx * P.M + r) * 8;
  bool any = true;
  if (passive(P, r)) {
    // an ambient that is not solved has no fluxes and exchanges nothing
    if (threadIdx.x == 0)
      for (int v = 0; v < 8; v++) part[v] = 0.0;
    return;
  }
  if (bx < nbb) {
    // thread t: face (side t & 1) of row/column q
    int t = threadIdx.x, row = t >> 1, side = t & 1;
    long q = (long)bx * CONS_ROWS + row;
    bool ok = q < cons_rows(P);
    double f[4] = {0, 0, 0, 0};
    int dir = q < P.ny ? 0 : 1;
    if (ok) cons_face<D, FLUX>(P, B, Qs, os, r, dir, dir == 0 ? (int)q : (int)(q - P.ny), side, f);
    for (int v = 0; v < 4; v++) face[row][side][v] = f[v];
    __syncthreads();
    if (ok && side == 0) {
      double l = dir == 0 ? B.scal[S_LX] : B.scal[S_LY];
      // cylindrical: the faces' radii (totals of r_i Q_i)
      double rlo = P.coord == 1 ? rad(P, 0) : 1.0, rhi = P.coord == 1 ? rad(P, P.nx) : 1.0;
      for (int v = 0; v < 4; v++)
        acc[v] = P.coord == 1 ? l * (face[row][0][v] * rlo - face[row][1][v] * rhi)
                              : l * (face[row][0][v] - face[row][1][v]);
    }
  } else {
    // cell indices fit 32 bits (the cell count NC is an int); the cut flags
    // of a thread's cells are all loaded before the first is tested
    constexpr int NQ = CONS_CH / 256;
    int q0 = (bx - nbb) * CONS_CH, n = P.nx * P.ny;
    int kq[NQ];
    uint8_t cq[NQ];
#pragma unroll
    for (int u = 0; u < NQ; u++) {
      int q = q0 + (int)threadIdx.x + u * 256;
      bool ok = q < n;
      kq[u] = cid(P, ok ? q % P.nx : 0, ok ? q / P.nx : 0);
      cq[u] = B.cut[kq[u]] & (ok ? 0xff : 0);
    }
    bool mine = false;
    double lv = B.scal[S_LV];
    if (D == 1 && P.coord == 1) {
      // cylindrical: r-weighted exchange of the cut cells and the geometric
      // source alpha p dt of every cell where the material has a state
      double dt = B.scal[S_DT];
      for (int u = 0; u < NQ; u++) {
        int q = q0 + (int)threadIdx.x + u * 256;
        if (q >= n) continue;
        double ri = rad(P, q + 0.5);
        if (cq[u]) {
          mine = true;
          for (int v = 0; v < 4; v++) acc[4 + v] += lv * B.X[((size_t)r * 4 + v) * P.NC + kq[u]] * ri;
        }
        double a = alpha_at<D>(P, B, r, kq[u]);
        if (a > 0.0) {
          bool vd;
          Prim w = Wget<D>(P, B, Qs, os, r, q, 0, vd);
          if (vd) {
            acc[5] += dt * (a * w.p);
            mine = true;
          }
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < NQ; u++) {
        if (!cq[u]) continue;
        mine = true;
        for (int v = 0; v < 4; v++) acc[4 + v] += lv * B.X[((size_t)r * 4 + v) * P.NC + kq[u]];
      }
    }
    any = __syncthreads_or(mine);
  }
  if (any) block_sum8(acc, red);
  if (threadIdx.x == 0)
    for (int v = 0; v < 8; v++) part[v] = any ? acc[v] : 0.0;
}


// combine the partials of nblk workgroups for (material r, quantity v),
// x = 8 r + v, in a fixed order (64 interleaved running sums, then a
// butterfly whose lane 0 result has a fixed order, so runs are reproducible)
// and add the stage total, weighted by w, to the running sums; one wavefront
MMD void cons_fin_wave(const Params& P, const Bufs& B, int nblk, double w, int x, int lane) {
  int r = x / 8, v = x % 8;
  double a = 0.0;
  for (int b = lane; b < nblk; b += 64) a += B.cpart[((size_t)b * P.M + r) * 8 + v];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane != 0) return;
  if (v < 4)
    neumaier_add(&B.cons[(CONS_BND * MAXM + r) * 4 + v], &B.cons[(CONS_BNDC * MAXM + r) * 4 + v],
                 w * a);
  else
    neumaier_add(&B.cons[(CONS_X * MAXM + r) * 4 + v - 4],
                 &B.cons[(CONS_XC * MAXM + r) * 4 + v - 4], w * a);
}
// one wavefront per (material, quantity); with advance, the time moves on by
// the step size (after the last stage of a step)
__global__ void __launch_bounds__(64) k_cons_fin(Params P, Bufs B, int nblk, double w,
                                                 int advance) {
  int x = blockIdx.x, t = threadIdx.x;
  if (advance && x == 0 && t == 0) {
    B.scal[S_T] += B.scal[S_DT];
    B.ctr[C_STEPNO] += 1;
  }
  if (x < P.M * 8) cons_fin_wave(P, B, nblk, w, x, t);
}

// this thread's part of the sums of Q (state buffer sidx) of material r over
// cells q0 + tid, q0 + tid + T, ... below q1; out[4..7] = 0
template <int D>
MMD void qsum_range(const Params& P, const Bufs& B, int sidx, int r, long q0, long q1, int tid,
                    int T, double acc[8]) {
  for (int v = 0; v < 8; v++) acc[v] = 0.0;
  for (long q = q0 + tid; q < q1; q += T) {
    int k = cid(P, (int)(q % P.nx), (int)(q / P.nx));
    // cylindrical: totals of r_i Q_i
    double ri = P.coord == 1 ? rad(P, (double)q + 0.5) : 1.0;
    for (int v = 0; v < 4; v++)
      acc[v] += P.coord == 1 ? loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, v, k) * ri
                             : loadQ<D>(P, B.Q[sidx], B.occ[sidx], r, v, k);
  }
}

// sums of Q per material and component: partials over CONS_CH cells per
// workgroup, then k_qsum_fin
template <int D>
__global__ void __launch_bounds__(256) k_qsum_part(Params P, Bufs B, int sidx) {
  __shared__ double red[4 * 8];
  long q0 = (long)blockIdx.x * CONS_CH, n = (long)P.nx * P.ny;
  long q1 = q0 + CONS_CH < n ? q0 + CONS_CH : n;
  for (int r = 0; r < P.M; r++) {
    double acc[8];
    qsum_range<D>(P, B, sidx, r, q0, q1, threadIdx.x, 256, acc);
    block_sum8(acc, red);
    if (threadIdx.x == 0)
      for (int v = 0; v < 4; v++) B.cpart[((size_t)blockIdx.x * P.M + r) * 4 + v] = acc[v];
  }
}
__global__ void __launch_bounds__(256) k_qsum_fin(Params P, Bufs B, int nblk) {
  __shared__ double red[4 * 8];
  for (int r = 0; r < P.M; r++) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
      for (int v = 0; v < 4; v++) a[v] += B.cpart[((size_t)b * P.M + r) * 4 + v];
    block_sum8(a, red);
    if (threadIdx.x == 0)
      for (int v = 0; v < 4; v++) B.cons[(CONS_Q * MAXM + r) * 4 + v] = a[v];
  }
}

MMD int tile_w(const Params& P) { return P.dim == 2 ? 16 : 256; }
MMD int tile_h(const Params& P) { return P.dim == 2 ? 16 : 1; }
MMD int tiles_x(const Params& P) { return (P.nx + tile_w(P) - 1) / tile_w(P); }


MMD void tile_flag(const Params& P, const Bufs& B, int didx, int nidx, int tile, int tid,
                   int nthr) {
  int tw = tile_w(P), th = tile_h(P);
  int i0 = (tile % tiles_x(P)) * tw, j0 = (tile / tiles_x(P)) * th;
  int ew = tw + 2, eh = P.dim == 2 ? th + 2 : 1;
  bool f = false;
  for (int q = tid; q < ew * eh; q += nthr) {
    int i = i0 - 1 + q % ew, j = P.dim == 2 ? j0 - 1 + q / ew : 0;
    if (!interior(P, i, j)) continue;
    int k = cid(P, i, j);
    uint8_t own = (uint8_t)(1u << B.chi[k]);
    if (B.dcut[k] <= 8 || B.dls[k] <= RV || B.occ[didx][k] != own || B.occ[nidx][k] != own)
      f = true;
  }
  if (__syncthreads_or(f) && tid == 0) {
    unsigned long long at = atomicAdd(&B.ctr[C_NTILES], 1ull);
    B.tiles[at] = tile;
  }
}
__global__ void __launch_bounds__(256) k_tiles(Params P, Bufs B, int didx, int nidx) {
  tile_flag(P, B, didx, nidx, (int)blockIdx.x, (int)threadIdx.x, (int)blockDim.x);
}
// Tile list (workgroups below nb, each flagging every nb-th of the nt tiles)
// beside the geometry and volume-fraction correction of every cut cell (the
// next nb workgroups, likewise over all tiles, without the list: every cut
// cell lies in a listed tile).  The geometry reads the level set and the
// densities, the list the distances and occupancy, and neither writes what
// the other reads.  With save_Q (the adjoint's recompute), workgroups from
// 2 nb on copy the updated state and its occupancy, before the mixing
// changes them, to save_Q / save_occ.
template <int D>
__global__ void __launch_bounds__(256) k_tiles_geom(Params P, Bufs B, int didx, int nidx,
                                                    int nt, int nb, double* save_Q,
                                                    uint8_t* save_occ, int gate) {
  if (gated_off(B, gate)) return;
  int b = blockIdx.x;
  if (b < nb) {
    for (int t = b; t < nt; t += nb) tile_flag(P, B, didx, nidx, t, (int)threadIdx.x, (int)blockDim.x);
    return;
  }
  if (b >= 2 * nb) {
    size_t nq = (size_t)P.M * (D + 2) * P.NC, nthr = (size_t)(gridDim.x - 2 * nb) * blockDim.x;
    const double* Q = B.Q[didx];
    for (size_t w = (size_t)(b - 2 * nb) * blockDim.x + threadIdx.x; w < nq + P.NC; w += nthr)
      if (w < nq)
        save_Q[w] = Q[w];
      else
        save_occ[w - nq] = B.occ[didx][w - nq];
    return;
  }
  b -= nb;
  int tw = tile_w(P), th = tile_h(P), ntx = tiles_x(P);
  for (int t = b; t < nt; t += nb) {
    int i = (t % ntx) * tw + (int)threadIdx.x % tw;
    int j = (t / ntx) * th + (int)threadIdx.x / tw;
    if (i < P.nx && j < P.ny) b_geom<D>(P, B, i, j, didx, nullptr);
  }
}

// run body(i, j) over the cells of the listed tiles, workgroup bx of nbx;
// 256 threads per workgroup
template <typename F>
MMD void for_tiles_n(const Params& P, const Bufs& B, int bx, int nbx, F body) {
  int ntile = (int)B.ctr[C_NTILES];
  int tw = tile_w(P), th = tile_h(P), ntx = tiles_x(P);
  for (int t = bx; t < ntile; t += nbx) {
    int tile = B.tiles[t];
    int i = (tile % ntx) * tw + (int)threadIdx.x % tw;
    int j = (tile / ntx) * th + (int)threadIdx.x / tw;
    if (i < P.nx && j < P.ny) body(i, j);
  }
}
template <typename F>
MMD void for_tiles(const Params& P, const Bufs& B, F body) {
  for_tiles_n(P, B, (int)blockIdx.x, (int)gridDim.x, body);
}

#define TILE_KERNEL(name, body, decl, ...)                                   \
  template <int D>                                                          \
  __global__ void __launch_bounds__(256) name(Params P, Bufs B decl) {     \
    for_tiles(P, B, [&](int i, int j) { body<D>(P, B, i, j __VA_ARGS__); }); \
  }
#define COMMA ,
// Real states of the listed tiles (workgroups below ntb) and the row pass of
// the ghost-band membership (the other ntb): the row pass reads only the
// classification and the volume fractions, which the real states leave alone.
// Workgroups from 2 ntb on run the copies of cl (the adjoint's recompute: the
// stage's input snapshot, which neither part writes).
template <int D>
__global__ void __launch_bounds__(256) t_real_near_row(Params P, Bufs B, int sidx, int ntb,
                                                       CopyList cl) {
  if ((int)blockIdx.x >= 2 * ntb) {
    copy_list_part(cl, (int)blockIdx.x - 2 * ntb, (int)gridDim.x - 2 * ntb);
    return;
  }
  // a new mixing stamp per stage (the previous stage's mixing is complete)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    B.ctr[C_STAMP] += 1;
    B.ctr[C_NGHOST] = 0;  // refilled by the column pass
    B.ctr[C_NBAND] = 0;   // the band list is rebuilt with the bulk flags
  }
  if ((int)blockIdx.x < ntb)
    for_tiles_n(P, B, (int)blockIdx.x, ntb, [&](int i, int j) { b_real<D>(P, B, i, j, sidx); });
  else
    for_tiles_n(P, B, (int)blockIdx.x - ntb, ntb,
                [&](int i, int j) { b_near_row<D>(P, B, i, j); });
}
// Column pass of the ghost-band membership (with the ghost queue) and, at
// stage 0, the reset of the level-set velocity validity, over the listed
// tiles (workgroups below ntb), beside the bulk flags and band list of the
// stage (the other gx * gy, blocks of bw x 256 / bw cells): the flags read
// only the classification and the occupancy, and the step size the real
// states, all complete before this launch.
template <int D>
__global__ void __launch_bounds__(256) t_near_col_flags(Params P, Bufs B, int sidx, int nidx,
                                                        int stage0, int ntb, int gx, int gy,
                                                        int bw) {
  int b = blockIdx.x;
  if (b < ntb) {
    for_tiles_n(P, B, b, ntb, [&](int i, int j) {
      if (stage0) b_vreset<D>(P, B, i, j);
      b_near_col<D>(P, B, i, j);
    });
    return;
  }
  b -= ntb;
  bulkflag_block<D>(P, B, sidx, nidx, stage0, b % gx, b / gx, bw, gx);
}
// Interface exchange of the listed tiles (workgroups below ntb) beside the
// frame of the state buffer (the others, one thread per frame cell): the
// exchange reads the states of its own cut cell only, the frame neither the
// exchange terms nor the velocities it writes.
template <int D>
__global__ void __launch_bounds__(256) t_iface_frame(Params P, Bufs B, int sidx, int stage,
                                                     int ntb, int ndt) {
  // with ndt > 0 the last workgroup sets the step size from the ndt wave-speed
  // maxima of the bulk-flag workgroups (nothing else in this launch reads it)
  if (ndt > 0 && (int)blockIdx.x == (int)gridDim.x - 1) {
    dt_reduce_block<D>(P, B, ndt);
    return;
  }
  if ((int)blockIdx.x < ntb) {
    for_tiles_n(P, B, (int)blockIdx.x, ntb,
                [&](int i, int j) { b_iface<D>(P, B, i, j, sidx, stage); });
    return;
  }
  int t = ((int)blockIdx.x - ntb) * (int)blockDim.x + (int)threadIdx.x;
  if (D == 2)
    bc_W2_cell(P, B, sidx, t);
  else if (t < P.ny * 2 * H * P.M)
    b_bc_W_x<D>(P, B, t, sidx);
}
TILE_KERNEL(t_vext, b_vext, COMMA int sweep, COMMA sweep)

// Level-set velocity of one listed tile at stage 0 (2D): the four sweeps of
// b_vext in LDS over the tile and a frame of four cells (the reach of four
// sweeps), then the fill of b_vfill for the tile's own cells; only the own
// cells are written back.  Other workgroups write back their tiles while
// this one reads its frame, so a cell enters with stamp 1 (interface
// velocities, final before this launch) or 0, and every swept velocity is
// computed here, never read.  Near the frame's outer edge the sweeps miss
// neighbours outside it; that reaches the own cells only after the fourth
// sweep.
constexpr int VF = 4, VT = 16, VW = VT + 2 * VF, VP = VW + 2;
struct VextSmem {
  double vx[VW * VW], vy[VW * VW], phi[VP * VP];
  uint8_t vit[VW * VW], vit0[VW * VW], cand[VW * VW];
};
__global__ void __launch_bounds__(256) k_vext_tiles(Params P, Bufs B, int sidx) {
  __shared__ VextSmem S;
  int ntile = (int)B.ctr[C_NTILES], ntx = tiles_x(P);
  bool err = errored(B);
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    int tile = B.tiles[t];
    int i0 = (tile % ntx) * VT - VF, j0 = (tile / ntx) * VT - VF;
    // level set over the region and one more cell (clamped into the frame:
    // only interior cells take differences of it)
    for (int q = threadIdx.x; q < VP * VP; q += blockDim.x) {
      int gi = i0 - 1 + q % VP, gj = j0 - 1 + q / VP;
      gi = gi < -1 ? -1 : (gi > P.nx ? P.nx : gi);
      gj = gj < -1 ? -1 : (gj > P.ny ? P.ny : gj);
      S.phi[q] = B.phi[cid(P, gi, gj)];
    }
    for (int q = threadIdx.x; q < VW * VW; q += blockDim.x) {
      int gi = i0 + q % VW, gj = j0 + q / VW;
      bool in = interior(P, gi, gj);
      int k = cid(P, in ? gi : 0, in ? gj : 0);
      uint8_t it = B.vit[k], dl = B.dls[k];
      double vx = B.vx[k], vy = B.vy[k];
      S.vit[q] = S.vit0[q] = in && it == 1 ? 1 : 0;
      S.vx[q] = vx;
      S.vy[q] = vy;
      S.cand[q] = in && !err && dl == 0;
    }
    __syncthreads();
    for (int sw = 0; sw < 4; sw++) {
      for (int q = threadIdx.x; q < VW * VW; q += blockDim.x) {
        int x = q % VW, y = q / VW, pq = (y + 1) * VP + x + 1;
        if (!S.cand[q] || !(S.phi[pq] < P.bls) || S.vit[q] != 0) continue;
        // a state of an earlier sweep (stamps of this sweep are sw + 2); a
        // cell with one is never written again, so its values are final
        auto valid_prev = [&](int xx, int yy) -> bool {
          if (xx < 0 || xx >= VW || yy < 0 || yy >= VW) return false;
          uint8_t it = S.vit[yy * VW + xx];
          return it != 0 && it <= sw + 1;
        };
        double gx = S.phi[pq + 1] - S.phi[pq - 1];
        double gy = S.phi[pq + VP] - S.phi[pq - VP];
        int kx = -1, ky = -1;
        if (gx != 0.0) {
          int xx = x - (gx > 0.0 ? 1 : -1);
          if (valid_prev(xx, y)) kx = y * VW + xx;
        }
        if (gy != 0.0) {
          int yy = y - (gy > 0.0 ? 1 : -1);
          if (valid_prev(x, yy)) ky = yy * VW + x;
        }
        double ox, oy;
        if (kx >= 0 && ky >= 0) {
          double wx = fabs(gx), wy = fabs(gy);
          ox = (wx * S.vx[kx] + wy * S.vx[ky]) / (wx + wy);
          oy = (wx * S.vy[kx] + wy * S.vy[ky]) / (wx + wy);
        } else if (kx >= 0) {
          ox = S.vx[kx];
          oy = S.vy[kx];
        } else if (ky >= 0) {
          ox = S.vx[ky];
          oy = S.vy[ky];
        } else {
          continue;
        }
        S.vx[q] = ox;
        S.vy[q] = oy;
        S.vit[q] = (uint8_t)(sw + 2);
      }
      __syncthreads();
    }
    // own cells: the swept states, then the fill and the time-n level set
    {
      int x = VF + (int)threadIdx.x % VT, y = VF + (int)threadIdx.x / VT;
      int i = i0 + x, j = j0 + y, q = y * VW + x;
      if (threadIdx.x < VT * VT && i < P.nx && j < P.ny) {
        int k = cid(P, i, j);
        if (S.vit[q] != S.vit0[q]) {
          B.vx[k] = S.vx[q];
          B.vy[k] = S.vy[q];
          B.vit[k] = S.vit[q];
        }
        if (B.dls[k] <= RV) {
          B.phin[k] = B.phi[k];
          B.chin[k] = B.chi[k];
          if (S.vit[q] == 0) {
            bool valid;
            Prim w = Wget<2>(P, B, B.Q[sidx], B.occ[sidx], B.chi[k], i, j, valid);
            B.vx[k] = valid ? w.u : 0.0;
            B.vy[k] = valid ? w.v : 0.0;
          }
        }
      }
    }
    __syncthreads();
  }
}
TILE_KERNEL(t_vfill, b_vfill, COMMA int sidx, COMMA sidx)

// ---------------------------------------------------------------------------
// Redistancing of the regional level set after a time step (2D).  Per listed
// 16 x 16 tile, in LDS over the tile and a frame of band_ls + 2 cells: the
// interface distances of the band cells from the crossings with their
// 4-neighbours of another material, then band_ls + 1 Jacobi sweeps of the
// 8-neighbour path distance within the material (each sweep reaches one
// cell further, so the tile's own cells are exact after the last one); the
// tile's band cells go to ptmp, committed by k_reinit_commit (other tiles
// read the old level set of their frames meanwhile).
// ---------------------------------------------------------------------------
constexpr int RI_T = 16, RI_FMAX = 12, RI_W = RI_T + 2 * RI_FMAX;
struct ReinitSmem {
  double a[RI_W * RI_W], b[RI_W * RI_W], phi[RI_W * RI_W];
  uint8_t chi[RI_W * RI_W], in[RI_W * RI_W], nb[RI_W * RI_W];
  uint16_t list[RI_W * RI_W];
  int nlist;
};
__global__ void __launch_bounds__(256) k_reinit_tiles(Params P, Bufs B) {
  __shared__ ReinitSmem S;
  int tid = threadIdx.x;
  int ntile = (int)B.ctr[C_NTILES], ntx = tiles_x(P);
  const int FR = P.nband + 2;  // frame: band_ls + 2 <= RI_FMAX
  const int W = RI_T + 2 * FR, nsw = FR - 1;
  double bls = P.bls;
  // neighbour n of the 8 (dj, di) in row-major order without the centre:
  // its offset in the window and its centre distance
  int off[8];
  double dist[8];
  for (int n = 0, q = 0; q < 9; q++) {
    if (q == 4) continue;
    int di = q % 3 - 1, dj = q / 3 - 1;
    double ex = di * P.dx, ey = dj * P.dy;
    off[n] = dj * W + di;
    dist[n] = sqrt(ex * ex + ey * ey);
    n++;
  }
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    int tile = B.tiles[t];
    int i0 = (tile % ntx) * RI_T - FR, j0 = (tile / ntx) * RI_T - FR;
    if (tid == 0) S.nlist = 0;
    for (int q = tid; q < W * W; q += 256) {
      int ci = i0 + q % W, cj = j0 + q / W;
      bool in = ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny;
      int k = in ? cid(P, ci, cj) : 0;
      S.in[q] = in ? 1 : 0;
      S.phi[q] = in ? B.phi[k] : bls;
      S.chi[q] = in ? B.chi[k] : 0;
    }
    __syncthreads();
    // interface distances; the band cells away from the window's outer ring
    // are listed with the mask of their same-material interior neighbours
    // (cells of the ring have no full neighbourhood and are never read for
    // the tile's own cells)
    for (int q = tid; q < W * W; q += 256) {
      int lx = q % W, ly = q / W;
      double best = bls;
      double pc = S.phi[q];
      if (S.in[q] && pc < bls && lx > 0 && ly > 0 && lx < W - 1 && ly < W - 1) {
        double dxm = -1.0, dym = -1.0;
        for (int n = 0; n < 4; n++) {
          int o = n == 0 ? -1 : (n == 1 ? 1 : (n == 2 ? -W : W));
          int qn = q + o;
          if (!S.in[qn] || S.chi[qn] == S.chi[q]) continue;
          double pn = S.phi[qn], sum = pc + pn;
          double hh = n < 2 ? P.dx : P.dy;
          double d = sum > 0.0 ? hh * (pc / sum) : 0.5 * hh;
          if (n < 2) {
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
        unsigned m = 0;
        for (int n = 0; n < 8; n++) {
          int qn = q + off[n];
          if (S.in[qn] && S.chi[qn] == S.chi[q]) m |= 1u << n;
        }
        S.nb[q] = (uint8_t)m;
        int at = atomicAdd(&S.nlist, 1);
        S.list[at] = (uint16_t)q;
      }
      S.a[q] = best;
      S.b[q] = best;
    }
    __syncthreads();
    // Jacobi sweeps over the listed band cells (every other cell keeps its
    // value, the band width, in both buffers)
    double* src = S.a;
    double* dst = S.b;
    int nl = S.nlist;
    for (int sw = 0; sw < nsw; sw++) {
      for (int e = tid; e < nl; e += 256) {
        int q = S.list[e];
        unsigned m = S.nb[q];
        double v = src[q];
        for (int n = 0; n < 8; n++) {
          if (!((m >> n) & 1)) continue;
          double cand = src[q + off[n]] + dist[n];
          if (cand < v) v = cand;
        }
        dst[q] = v < bls ? v : bls;
      }
      __syncthreads();
      double* tmp = src;
      src = dst;
      dst = tmp;
    }
    for (int q = tid; q < RI_T * RI_T; q += 256) {
      int lx = FR + q % RI_T, ly = FR + q / RI_T, lq = ly * W + lx;
      int ci = i0 + lx, cj = j0 + ly;
      if (ci < P.nx && cj < P.ny) B.ptmp[cid(P, ci, cj)] = src[lq];
    }
    __syncthreads();  // the LDS window is reused by the next tile
  }
}
// commit of the redistanced band cells of the listed tiles
__global__ void __launch_bounds__(256) k_reinit_commit(Params P, Bufs B) {
  for_tiles(P, B, [&](int i, int j) {
    int k = cid(P, i, j);
    if (B.phi[k] < P.bls) B.phi[k] = B.ptmp[k];
  });
}

// 1D: every ghost-extension sweep of a stage in one workgroup, a barrier
// between sweeps (each sweep reads the states the previous ones left, as
// separate launches would; the queue of a 1D problem is short)
__global__ void __launch_bounds__(1024) k_ext_all1(Params P, Bufs B, int sidx) {
  int n = (int)B.ctr[C_NGHOST];
  if (errored(B)) return;
  for (int sw = 0; sw < P.kext + 4; sw++) {
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
      int e = B.glist[q];
      int k = e >> 3, r = e & 7;
      if (B.Wit[(size_t)r * P.NC + k] != 0) continue;
      ext_one<1>(P, B, k % P.NX - H, 0, r, sidx, sw);
    }
    __syncthreads();
  }
}
// 1D, stage 0: the four level-set velocity sweeps and the fill over the
// listed tiles in one workgroup, a barrier after each pass
__global__ void __launch_bounds__(1024) k_vel_all1(Params P, Bufs B, int sidx) {
  int ncell = (int)B.ctr[C_NTILES] * 256;
  for (int pass = 0; pass < 5; pass++) {
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
      int i = B.tiles[q / 256] * 256 + q % 256;
      if (i >= P.nx) continue;
      if (pass < 4)
        b_vext<1>(P, B, i, 0, pass);
      else
        b_vfill<1>(P, B, i, 0, sidx);
    }
    __syncthreads();
  }
}
TILE_KERNEL(t_ls_commit, b_ls_commit, )

// Commit of the new level set and its frame in one launch (2D), with the
// book-keeping totals of the stage in its last workgroups (from ntb + nfr
// on).  Workgroups below ntb commit the listed tiles; the next nfr fill the
// ghost frame (x sides
// of rows [0, ny), then y sides of columns [-H, nx + H), a corner from the
// source cell of both maps) from the committed value of the source cell: the
// new one where the commit writes it (band cells, dls <= 3, always inside a
// listed tile), the old one elsewhere.  A frame thread therefore reads only
// words that no commit thread writes.
__global__ void __launch_bounds__(256) k_ls_commit_bc(Params P, Bufs B, int ntb, int nfr,
                                                      int nblk, double w, int advance) {
  if ((int)blockIdx.x >= ntb + nfr) {
    // the book-keeping totals of the stage: one wavefront per (material,
    // quantity), independent of the level set
    int x = ((int)blockIdx.x - ntb - nfr) * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (advance && x == 0 && lane == 0) {
      B.scal[S_T] += B.scal[S_DT];
      B.ctr[C_STEPNO] += 1;
    }
    if (x < P.M * 8) cons_fin_wave(P, B, nblk, w, x, lane);
    return;
  }
  if ((int)blockIdx.x < ntb) {
    int ntile = (int)B.ctr[C_NTILES];
    int tw = tile_w(P), th = tile_h(P), ntx = tiles_x(P);
    for (int t = blockIdx.x; t < ntile; t += ntb) {
      int tile = B.tiles[t];
      int i = (tile % ntx) * tw + (int)threadIdx.x % tw;
      int j = (tile / ntx) * th + (int)threadIdx.x / tw;
      if (i < P.nx && j < P.ny) b_ls_commit<2>(P, B, i, j);
    }
    return;
  }
  int t = ((int)blockIdx.x - ntb) * (int)blockDim.x + (int)threadIdx.x;
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
  bool upd = !errored(B) && B.dls[ks] <= 3;
  B.phi[k] = upd ? B.ptmp[ks] : B.phi[ks];
  B.chi[k] = upd ? B.ctmp[ks] : B.chi[ks];
}

// Band fluxes and updates together with the book-keeping partials and the
// level-set stage, in one launch: workgroups below ncons * M compute
// partials (workgroup x of material r), the next nls the level-set stage of
// the listed tiles, the other nfb the band list.  The partials read only the
// stage's source state, fluxes and exchange terms, the level-set stage only
// the level sets, the velocity and the step size: none of it is written by
// the band update, so their latency hides behind the band work.
template <int D, int FLUX>
__global__ void __launch_bounds__(256) k_flux_list_cons(Params P, Bufs B, int sidx, int nidx,
                                                        int didx, double bcoef, double ccoef,
                                                        int nfb, int nbb, int ncons, int nls) {
  int b = blockIdx.x, nc = ncons * P.M;
  if (b < nc)
    cons_part_block<D, FLUX>(P, B, sidx, nbb, b % ncons, b / ncons);
  else if (b < nc + nls)
    for_tiles_n(P, B, b - nc, nls, [&](int i, int j) { b_ls<D>(P, B, i, j, bcoef, ccoef); });
  else
    flux_list_blocks<D, FLUX>(P, B, sidx, nidx, didx, bcoef, ccoef, b - nc - nls, nfb);
}
template <int D>
__global__ void __launch_bounds__(256) t_mix1(Params P, Bufs B, int didx) {
  // one material per grid row: the sources of different materials are
  // independent
  uint32_t st = (uint32_t)B.ctr[C_STAMP];
  int r = blockIdx.y;
  for_tiles(P, B, [&](int i, int j) { b_mix1<D>(P, B, i, j, didx, st, r, r + 1); });
}
template <int D>
__global__ void __launch_bounds__(256) t_mix2(Params P, Bufs B, int didx, CopyList cl) {
  // grid slice z = 1: the copies of cl (the adjoint's recompute: states the
  // stage read, which the mixing leaves alone)
  if (blockIdx.z == 1) {
    copy_list_part(cl, (int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    return;
  }
  // one material per grid row, occupancy bits by word atomics
  uint32_t st = (uint32_t)B.ctr[C_STAMP];
  int r = blockIdx.y;
  for_tiles(P, B, [&](int i, int j) { b_mix2<D>(P, B, i, j, didx, st, r, r + 1, true); });
}
// is cell k within H cells of the domain boundary (its level set and
// indicator are copied into the frame)?
MMD bool near_edge(const Params& P, int k) {
  int i = k % P.NX - H, j = k / P.NX - P.HY;
  return i < H || i >= P.nx - H || (P.dim == 2 && (j < H || j >= P.ny - H));
}
// both sides of the level-set frame again, by the whole workgroup
template <int D>
MMD void refill_ls_frame(const Params& P, const Bufs& B) {
  for (int t = threadIdx.x; t < P.ny * 2 * H; t += blockDim.x) b_bc_ls_x(P, t, B.phi, B.chi);
  __syncthreads();
  if (D == 2)
    for (int t = threadIdx.x; t < (P.nx + 2 * H) * 2 * H; t += blockDim.x)
      b_bc_ls_y(P, t, B.phi, B.chi);
}

// The stage's stranded sources, listed by the mixing (one workgroup): when a
// cell was relabelled the level-set frame is filled again and the stage's
// stamp recorded, so that the classification and geometry launched next run
// again (with the masses after mixing); the list is emptied for the next
// stage.
template <int D>
__global__ void __launch_bounds__(256) k_absorb(Params P, Bufs B, int didx) {
  int n = (int)B.ctr[C_NAB];
  if (n == 0) return;
  uint32_t st = (uint32_t)B.ctr[C_STAMP];
  bool rel = false, edge = false;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int k = B.abList[e];
    if (b_absorb<D>(P, B, k, didx, st)) {
      rel = true;
      edge |= near_edge(P, k);
    }
  }
  if (__syncthreads_or(rel)) {
    if (__syncthreads_or(edge)) refill_ls_frame<D>(P, B);
    if (threadIdx.x == 0) B.ctr[C_RLSTAMP] = st;
  }
  if (threadIdx.x == 0) B.ctr[C_NAB] = 0;
}

template <int D>
__global__ void __launch_bounds__(256) t_ss_detect(Params P, Bufs B) {
  for_tiles(P, B, [&](int i, int j) { b_ss_detect<D>(P, B, i, j); });
}
// the step's oddball cells (one workgroup), then the level-set frame and
// the stamp that runs the classification and geometry launched next
template <int D>
__global__ void __launch_bounds__(256) k_ss_apply(Params P, Bufs B, int didx) {
  int n = (int)B.ctr[C_NSS];
  if (n == 0) return;
  bool edge = false;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    b_ss_apply<D>(P, B, B.ssList[e], didx);
    edge |= near_edge(P, B.ssList[e]);
  }
  if (__syncthreads_or(edge)) refill_ls_frame<D>(P, B);
  if (threadIdx.x == 0) {
    B.ctr[C_SSSTAMP] = B.ctr[C_STAMP];
    B.ctr[C_NSS] = 0;
  }
}

// All ghost-extension sweeps of one material on one active 16 x 16 tile in
// one launch (2D).  A sweep reaches one cell further, so the tile and a frame
// of EXR >= k_ext + 4 cells determine the tile's ghost states exactly: the
// sweeps run in LDS over that region with the same stamps as the global
// sweeps (a neighbour counts if it had a state before the sweep began), and
// only the tile's own queued pairs are written back.  Frame cells whose
// neighbours lie outside the region can come out differently; their effect
// travels one cell per sweep and does not reach the tile.
constexpr int EXR = 12, EXT = 16, EXW = EXT + 2 * EXR, EXG = EXW + 2;
struct ExtSmem {
  double W[4][EXW * EXW];
  double lphi[EXG * EXG];  // local level set of the material, region + ring
  uint8_t st[EXW * EXW];   // sweep stamp: 0 no state, 1 real, s + 2 sweep s
  uint8_t pend[EXW * EXW]; // queued ghost pair
  uint16_t list[EXW * EXW];  // the region's queued pairs
  int nlist;
};
__global__ void __launch_bounds__(256) k_ext_tiles(Params P, Bufs B, int sidx) {
  __shared__ ExtSmem S;
  __shared__ int any;
  const int r = blockIdx.y, tid = threadIdx.x, ntx = tiles_x(P);
  if (errored(B)) return;
  const int ntile = (int)B.ctr[C_NTILES], nsw = P.kext + 4;
  const double* Q = B.Q[sidx];
  const uint8_t* occ = B.occ[sidx];
  // Other workgroups write back their tiles while this one reads its frame:
  // a queued pair is recognised by its stamp not being 1 (real states have
  // 1 throughout; queued pairs 0 until written back, then the sweep stamp),
  // and its state is always recomputed here, never read.
  auto pending = [&](int k) -> bool {
    uint8_t dc = B.dcut[k], n4 = B.near4[k], ct = B.cut[k], ch = B.chi[k],
            it = B.Wit[(size_t)r * P.NC + k];  // all loads issued together
    return dc <= 4 && ((n4 >> r) & 1) && !(!ct && ch == r) && it != 1;
  };
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    int tile = B.tiles[t];
    int ti0 = (tile % ntx) * EXT, tj0 = (tile / ntx) * EXT;
    int x0 = ti0 - EXR, y0 = tj0 - EXR;
    if (tid == 0) {
      any = 0;
      S.nlist = 0;
    }
    __syncthreads();
    {
      int i = ti0 + tid % EXT, j = tj0 + tid / EXT;
      if (i < P.nx && j < P.ny && pending(cid(P, i, j))) any = 1;
    }
    __syncthreads();
    if (!any) continue;  // the same for the whole workgroup
    // the region's states (loads of all the thread's cells in flight
    // together): real states from the buffer, far pure cells from Q
    constexpr int NQ = (EXW * EXW + 255) / 256, NG = (EXG * EXG + 255) / 256;
    int kq[NQ];
    uint8_t dcq[NQ], chq[NQ], itq[NQ], n4q[NQ], ctq[NQ], ocq[NQ];
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int q = tid + n * 256;
      int ci = x0 + q % EXW, cj = y0 + q / EXW;
      bool in = q < EXW * EXW && interior(P, ci, cj);
      int k = in ? cid(P, ci, cj) : -1, ks = in ? k : cid(P, 0, 0);
      kq[n] = k;
      // unconditional loads from an in-range cell, selected afterwards, so
      // that no load waits for the previous one
      uint8_t a0 = B.dcut[ks], a1 = B.chi[ks], a2 = B.Wit[(size_t)r * P.NC + ks],
              a3 = B.near4[ks], a4 = B.cut[ks], a5 = occ[ks];
      dcq[n] = in ? a0 : 0;
      chq[n] = in ? a1 : 0;
      itq[n] = in ? a2 : 0;
      n4q[n] = in ? a3 : 0;
      ctq[n] = in ? a4 : 0;
      ocq[n] = in ? a5 : 0;
    }
    double U[NQ][4];
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int k = kq[n];
      bool far = dcq[n] > 7 && chq[n] == r;
      bool need = k >= 0 && (far || (dcq[n] <= 7 && itq[n] == 1));
      const double* base = far ? Q : B.W;
      size_t o = (size_t)r * 4 * P.NC + (k >= 0 ? k : cid(P, 0, 0));
      for (int c = 0; c < 4; c++) {
        double u = base[o + (size_t)c * P.NC];
        U[n][c] = need ? u : 0.0;
      }
    }
#pragma unroll
    for (int n = 0; n < NQ; n++) {
      int q = tid + n * 256;
      if (q >= EXW * EXW) continue;
      int k = kq[n];
      uint8_t st = 0, pd = 0;
      double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
      if (k >= 0) {
        if (dcq[n] > 7) {
          if (chq[n] == r) {
            st = 1;
            bool has = (ocq[n] >> r) & 1;
            double U0 = has ? U[n][0] / 1.0 : 0.0, U1 = has ? U[n][1] / 1.0 : 0.0,
                   U2 = has ? U[n][2] / 1.0 : 0.0, U3 = has ? U[n][3] / 1.0 : 0.0;
            Prim w = prim_from_U(U0, U1, U2, U3, eos_of(P, r));
            w0 = w.r; w1 = w.u; w2 = w.v; w3 = w.p;
          }
        } else {
          st = itq[n] == 1 ? 1 : 0;
          if (st) {
            w0 = U[n][0]; w1 = U[n][1]; w2 = U[n][2]; w3 = U[n][3];
          }
          pd = dcq[n] <= 4 && ((n4q[n] >> r) & 1) && !(!ctq[n] && chq[n] == r) && itq[n] != 1;
        }
      }
      S.st[q] = st;
      S.pend[q] = pd;
      S.W[0][q] = w0; S.W[1][q] = w1; S.W[2][q] = w2; S.W[3][q] = w3;
      if (pd) S.list[atomicAdd(&S.nlist, 1)] = (uint16_t)q;
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
    // a region cell's state counts in sweep s if it had one before the sweep
    auto valid = [&](int lx, int ly, int ci, int cj, int s) -> bool {
      if (lx < 0 || lx >= EXW || ly < 0 || ly >= EXW || !interior(P, ci, cj)) return false;
      int it = S.st[ly * EXW + lx];
      return it != 0 && it <= s + 1;
    };
    const int nl = S.nlist;
    for (int s = 0; s < nsw; s++) {
      bool open = false;
      for (int e = tid; e < nl; e += 256) {
        int q = S.list[e];
        if (S.st[q] != 0) continue;
        open = true;
        int lx = q % EXW, ly = q / EXW, ci = x0 + lx, cj = y0 + ly;
        double out[4];
        bool ok = false;
        if (s < P.kext) {
          int g = (ly + 1) * EXG + lx + 1;  // the cell in the ring-padded level set
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
            double wx = fabs(gx), wy = fabs(gy);
            for (int c = 0; c < 4; c++) out[c] = (wx * S.W[c][a] + wy * S.W[c][b]) / (wx + wy);
            ok = true;
          } else if (hx || hy) {
            int a = hx ? ly * EXW + lx + sx : (ly + sy) * EXW + lx;
            for (int c = 0; c < 4; c++) out[c] = S.W[c][a];
            ok = true;
          }
        } else {
          double row[3][4];
          int cnt = 0;
          for (int dj = -1; dj <= 1; dj++) {
            double a[3][4];
            for (int di = -1; di <= 1; di++) {
              bool use = (di != 0 || dj != 0) && valid(lx + di, ly + dj, ci + di, cj + dj, s);
              int n = use ? (ly + dj) * EXW + lx + di : q;  // in range even when unused
              for (int c = 0; c < 4; c++) a[di + 1][c] = use ? S.W[c][n] : 0.0;
              cnt += use ? 1 : 0;
            }
            for (int c = 0; c < 4; c++) row[dj + 1][c] = (a[0][c] + a[2][c]) + a[1][c];
          }
          if (cnt > 0) {
            for (int c = 0; c < 4; c++)
              out[c] = ((row[0][c] + row[2][c]) + row[1][c]) / (double)cnt;
            ok = true;
          }
        }
        if (ok) {
          for (int c = 0; c < 4; c++) S.W[c][q] = out[c];
          S.st[q] = (uint8_t)(s + 2);
        }
      }
      // once every queued pair of the region has a state, later sweeps
      // change nothing
      if (!__syncthreads_or(open)) break;
    }
    // the tile's own pairs go back to the state buffer
    {
      int lx = EXR + tid % EXT, ly = EXR + tid / EXT, i = x0 + lx, j = y0 + ly;
      int q = ly * EXW + lx;
      if (i < P.nx && j < P.ny && S.pend[q] && S.st[q] != 0) {
        int k = cid(P, i, j);
        size_t o = (size_t)r * 4 * P.NC + k;
        for (int c = 0; c < 4; c++) B.W[o + (size_t)c * P.NC] = S.W[c][q];
        B.Wit[(size_t)r * P.NC + k] = S.st[q];
      }
    }
    __syncthreads();
  }
}

#undef TILE_KERNEL
#undef COMMA

// ---------------------------------------------------------------------------
// Batched 1D instances: one workgroup advances one instance through all
// steps; every phase of the step is a loop of the workgroup's threads over
// the instance's cells followed by a workgroup barrier.  Instances are
// independent, so no grid-wide synchronisation is needed.
// ---------------------------------------------------------------------------
#define PHASE(call)                                       \
  do {                                                    \
    for (int i_ = tid; i_ < P.nx; i_ += T) { call; }      \
    __syncthreads();                                      \
  } while (0)

struct BatchSmem {
  Params P;
  Bufs B;
  Bulk1Smem S;
  double red[T1MAX];
};

MMD void batch_load(const Params* Pa, const Bufs* Ba, BatchSmem& sm) {
  if (threadIdx.x == 0) {
    sm.P = Pa[blockIdx.x];
    sm.B = Ba[blockIdx.x];
  }
  __syncthreads();
}

// MAXT: the largest workgroup the variant runs with (its register budget
// follows from it: 128 registers at 1024 threads, 256 at 512, 512 at 256)
template <int MAXT>
__global__ void __launch_bounds__(MAXT)
k_batch1d(const Params* Pa, const Bufs* Ba, int nsteps, int rk_order) {
  __shared__ BatchSmem sm;
  batch_load(Pa, Ba, sm);
  const Params& P = sm.P;
  const Bufs& B = sm.B;
  int tid = threadIdx.x, T = blockDim.x;
  double bc[3], cc[3], wc[3];
  int ns;
  if (rk_order == 2) {
    ns = 2;
    bc[0] = 0.0; bc[1] = 0.5;
    cc[0] = 1.0; cc[1] = 0.5;
    wc[0] = 0.5; wc[1] = 0.5;
  } else {
    ns = 3;
    bc[0] = 0.0; bc[1] = 0.75; bc[2] = 1.0 / 3.0;
    cc[0] = 1.0; cc[1] = 0.25; cc[2] = 2.0 / 3.0;
    wc[0] = 1.0 / 6.0; wc[1] = 1.0 / 6.0; wc[2] = 2.0 / 3.0;
  }
  uint32_t stamp = (uint32_t)B.ctr[C_STAMP];
  for (int n = 0; n < nsteps; n++) {
    __syncthreads();
    if (errored(B)) break;
    int sidx = 0;
    for (int s = 0; s < ns; s++) {
      int didx = s == ns - 1 ? 0 : s + 1;
      PHASE(b_real<1>(P, B, i_, 0, sidx));
      if (P.fs_on) {
        for (int k = tid; k < P.NC; k += T) b_ambient<1>(P, B, k, sidx, s);
        __syncthreads();
      }
      if (s == 0) {
        double w = 0.0;
        for (int i = tid; i < P.nx; i += T) w = fmax(w, b_dt_cell<1>(P, B, i, 0, sidx));
        sm.red[tid] = w;
        __syncthreads();
        for (int h = T / 2; h > 0; h >>= 1) {
          if (tid < h) sm.red[tid] = fmax(sm.red[tid], sm.red[tid + h]);
          __syncthreads();
        }
        if (tid == 0) dt_finish<1>(P, B, sm.red[0]);
        __syncthreads();
      }
      PHASE(b_near_row<1>(P, B, i_, 0));
      PHASE(b_near_col<1>(P, B, i_, 0));
      for (int sw = 0; sw < P.kext + 4; sw++) PHASE(b_ext<1>(P, B, i_, 0, sidx, sw));
      for (int t = tid; t < 2 * H * P.M; t += T) b_bc_W_x<1>(P, B, t, sidx);
      __syncthreads();
      if (s == 0) PHASE(b_vreset<1>(P, B, i_, 0));
      PHASE(b_iface<1>(P, B, i_, 0, sidx, s));
      if (s == 0) {
        for (int sw = 0; sw < 4; sw++) PHASE(b_vext<1>(P, B, i_, 0, sw));
        PHASE(b_vfill<1>(P, B, i_, 0, sidx));
      }
      PHASE(b_bulkflag<1>(P, B, i_, 0, sidx, 0));
      for (int i0 = 0; i0 < P.nx; i0 += T)
        bulk1_tile(P, B, sm.S, i0, sidx, 0, didx, bc[s], cc[s], s == 0 ? 1 : 0);
      PHASE(b_flux_band<1>(P, B, i_, 0, sidx, 0, didx, bc[s], cc[s]));
      {
        // conservation book-keeping: the 2 M boundary faces in parallel,
        // then the exchange of the cut cells, one material at a time
        double* fb = sm.red;  // [2 M][4] boundary face terms A F
        if (tid < 2 * P.M)
          cons_face<1>(P, B, B.Q[sidx], B.occ[sidx], tid >> 1, 0, 0, tid & 1, fb + tid * 4);
        __syncthreads();
        double lv = B.scal[S_LV], lx = B.scal[S_LX], dt = B.scal[S_DT];
        bool cyl = P.coord == 1;
        for (int r = 0; r < P.M; r++) {
          // an ambient that is not solved: nothing to book
          if (passive(P, r)) continue;
          double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int i = tid; i < P.nx; i += T) {
            int k = cid(P, i, 0);
            double ri = cyl ? rad(P, i + 0.5) : 1.0;
            if (B.cut[k])
              for (int v = 0; v < 4; v++)
                acc[4 + v] += cyl ? lv * B.X[((size_t)r * 4 + v) * P.NC + k] * ri
                                  : lv * B.X[((size_t)r * 4 + v) * P.NC + k];
            // cylindrical: geometric source of the radial momentum
            double a = cyl ? alpha_at<1>(P, B, r, k) : 0.0;
            if (a > 0.0) {
              bool vd;
              Prim w = Wget<1>(P, B, B.Q[sidx], B.occ[sidx], r, i, 0, vd);
              if (vd) acc[5] += dt * (a * w.p);
            }
          }
          if (tid == 0)
            for (int v = 0; v < 4; v++)
              acc[v] = cyl ? lx * (fb[2 * r * 4 + v] * rad(P, 0) - fb[(2 * r + 1) * 4 + v] * rad(P, P.nx))
                           : lx * (fb[2 * r * 4 + v] - fb[(2 * r + 1) * 4 + v]);
          block_sum8(acc, sm.red + 64);
          if (tid == 0) cons_accumulate(B, r, acc, wc[s]);
        }
      }
      PHASE(b_ls<1>(P, B, i_, 0, bc[s], cc[s]));
      PHASE(b_ls_commit<1>(P, B, i_, 0));
      for (int t = tid; t < 2 * H; t += T) b_bc_ls_x(P, t, B.phi, B.chi);
      __syncthreads();
      PHASE(b_classify<1>(P, B, i_, 0));
      PHASE(b_dist_row<1>(P, B, i_, 0));
      PHASE(b_geom<1>(P, B, i_, 0, didx, (const double*)nullptr));
      PHASE(b_mix1<1>(P, B, i_, 0, didx, stamp, 0, P.M));
      PHASE(b_mix2<1>(P, B, i_, 0, didx, stamp, 0, P.M, false));
      {
        // stranded sources; a relabelled cell: frame, classification and
        // geometry once more (masses after mixing)
        int nab = (int)B.ctr[C_NAB];
        bool rel = false;
        for (int e = tid; e < nab; e += T) rel |= b_absorb<1>(P, B, B.abList[e], didx, stamp);
        if (__syncthreads_or(rel)) {
          for (int t = tid; t < 2 * H; t += T) b_bc_ls_x(P, t, B.phi, B.chi);
          __syncthreads();
          PHASE(b_classify<1>(P, B, i_, 0));
          PHASE(b_dist_row<1>(P, B, i_, 0));
          PHASE(b_geom<1>(P, B, i_, 0, didx, (const double*)nullptr));
        }
        if (tid == 0) B.ctr[C_NAB] = 0;
        __syncthreads();
      }
      stamp++;
      sidx = didx;
    }
    if (P.scale_sep) {
      PHASE(b_ss_detect<1>(P, B, i_, 0));
      int nss = (int)B.ctr[C_NSS];
      for (int e = tid; e < nss; e += T) b_ss_apply<1>(P, B, B.ssList[e], 0);
      __syncthreads();
      if (nss > 0) {
        for (int t = tid; t < 2 * H; t += T) b_bc_ls_x(P, t, B.phi, B.chi);
        __syncthreads();
        PHASE(b_classify<1>(P, B, i_, 0));
        PHASE(b_dist_row<1>(P, B, i_, 0));
        PHASE(b_geom<1>(P, B, i_, 0, 0, (const double*)nullptr));
      }
      if (tid == 0) B.ctr[C_NSS] = 0;
      __syncthreads();
    }
    if (tid == 0) {
      B.scal[S_T] += B.scal[S_DT];
      B.ctr[C_STEPNO] += 1;
    }
  }
  __syncthreads();
  if (tid == 0) B.ctr[C_STAMP] = stamp;
}

// initial state of every instance; arrays are the concatenation of the
// instances' interior cells (offset off[q] cells for instance q)
__global__ void __launch_bounds__(1024)
k_batch1d_init(const Params* Pa, const Bufs* Ba, const double* phi, const int32_t* chi,
               const double* W, const int64_t* off) {
  __shared__ BatchSmem sm;
  batch_load(Pa, Ba, sm);
  const Params& P = sm.P;
  const Bufs& B = sm.B;
  int tid = threadIdx.x, T = blockDim.x;
  int64_t o = off[blockIdx.x];
  const double* Wq = W + (size_t)P.M * 3 * o;
  PHASE(b_load_ls<1>(P, B, i_, 0, phi + o, chi + o));
  for (int t = tid; t < 2 * H; t += T) b_bc_ls_x(P, t, B.phi, B.chi);
  __syncthreads();
  PHASE(b_classify<1>(P, B, i_, 0));
  PHASE(b_dist_row<1>(P, B, i_, 0));
  PHASE(b_geom<1>(P, B, i_, 0, 0, Wq));
  PHASE(b_init_Q<1>(P, B, i_, 0, Wq));
}

__global__ void __launch_bounds__(1024)
k_batch1d_pack(const Params* Pa, const Bufs* Ba, double* Q, double* alpha, double* phi,
               int32_t* chi, const int64_t* off) {
  __shared__ BatchSmem sm;
  batch_load(Pa, Ba, sm);
  const Params& P = sm.P;
  const Bufs& B = sm.B;
  int tid = threadIdx.x, T = blockDim.x;
  int64_t o = off[blockIdx.x];
  PHASE(b_pack<1>(P, B, i_, 0, 0, Q ? Q + (size_t)P.M * 3 * o : nullptr,
                  alpha ? alpha + (size_t)P.M * o : nullptr, phi ? phi + o : nullptr,
                  chi ? chi + o : nullptr));
}

// sums of Q per material and component of every instance (one workgroup
// per instance)
__global__ void __launch_bounds__(1024) k_batch1d_qsum(const Params* Pa, const Bufs* Ba) {
  __shared__ BatchSmem sm;
  batch_load(Pa, Ba, sm);
  const Params& P = sm.P;
  const Bufs& B = sm.B;
  for (int r = 0; r < P.M; r++) {
    double acc[8];
    qsum_range<1>(P, B, 0, r, 0, P.nx, threadIdx.x, blockDim.x, acc);
    block_sum8(acc, sm.red);
    if (threadIdx.x == 0)
      for (int v = 0; v < 4; v++) B.cons[(CONS_Q * MAXM + r) * 4 + v] = acc[v];
  }
}
#undef PHASE

}  // namespace mmfv
