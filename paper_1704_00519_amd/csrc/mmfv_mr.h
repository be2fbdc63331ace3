// Multiresolution analysis of a 2D state (Sec. 2.4): the cell-average
// pyramid of the mixture density and total energy, the details of the
// 5th-order prediction, their level-dependent thresholding, and the block
// structure (refinement, safety zone, grading, existence, leaves) that they
// and the interface position identifier produce.
//
// Levels l = 0 (coarsest) .. L (the solver grid); level l has
// nx / 2^(L-l) x ny / 2^(L-l) cells, dense row-major (no halo), in blocks of
// bs x bs cells.  Flags are 32-bit words, one per block and level.
#pragma once
#include "mmfv_kernels.h"

namespace mmfv {

constexpr int MR_MAXL = 10;
constexpr double MR_G1 = -22.0 / 128.0, MR_G2 = 3.0 / 128.0;

// Flags of the blocks a 16 x 16 tile of cells (origin i0, j0) touches, in
// LDS: at most 9 x 9 blocks (block side >= 2); one atomic per touched,
// flagged block when the tile is done.
constexpr int MR_TILE = 16, MR_LOC = 9;
struct MrTileFlags {
  int bx0, by0, nlx, nly;
  MMD void init(int i0, int j0, int bs) {
    bx0 = i0 / bs;
    by0 = j0 / bs;
    nlx = (i0 + MR_TILE - 1) / bs - bx0 + 1;
    nly = (j0 + MR_TILE - 1) / bs - by0 + 1;
  }
  MMD int local(int i, int j, int bs) const { return (j / bs - by0) * nlx + (i / bs - bx0); }
};

// Level-L fields (the sums over the materials, in material order, of rho
// and rho E), the interface identifier of the solver-grid blocks (a cell in
// the narrow band: level-set value below band), and per workgroup the
// largest magnitudes of the two fields (part[2 b], part[2 b + 1]).  One
// 16 x 16 tile of cells per workgroup.
__global__ void __launch_bounds__(256) k_mr_fields(Params P, Bufs B, double* u0, double* u1,
                                                   uint32_t* iface, int bs, double band,
                                                   double* part) {
  __shared__ uint32_t sf[MR_LOC * MR_LOC];
  __shared__ double r0[4], r1[4];
  int tid = threadIdx.x;
  int i0 = blockIdx.x * MR_TILE, j0 = blockIdx.y * MR_TILE;
  int i = i0 + tid % MR_TILE, j = j0 + tid / MR_TILE;
  MrTileFlags tf;
  tf.init(i0, j0, bs);
  if (tid < MR_LOC * MR_LOC) sf[tid] = 0;
  __syncthreads();
  bool in = i < P.nx && j < P.ny;
  double a0 = 0.0, a1 = 0.0;
  if (in) {
    int k = cid(P, i, j);
    double rho = loadQ<2>(P, B.Q[0], B.occ[0], 0, 0, k);
    double E = loadQ<2>(P, B.Q[0], B.occ[0], 0, 3, k);
    for (int r = 1; r < P.M; r++) {
      rho = rho + loadQ<2>(P, B.Q[0], B.occ[0], r, 0, k);
      E = E + loadQ<2>(P, B.Q[0], B.occ[0], r, 3, k);
    }
    size_t q = (size_t)j * P.nx + i;
    u0[q] = rho;
    u1[q] = E;
    a0 = fabs(rho);
    a1 = fabs(E);
    if (B.phi[k] < band) sf[tf.local(i, j, bs)] = 1;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a0 = fmax(a0, __shfl_xor(a0, o));
    a1 = fmax(a1, __shfl_xor(a1, o));
  }
  if (__lane_id() == 0) {
    r0[tid >> 6] = a0;
    r1[tid >> 6] = a1;
  }
  __syncthreads();
  if (tid < tf.nlx * tf.nly && sf[tid]) {
    int bi = tf.bx0 + tid % tf.nlx, bj = tf.by0 + tid / tf.nlx;
    if (bi < P.nx / bs && bj < P.ny / bs) atomicOr(&iface[(size_t)bj * (P.nx / bs) + bi], 1u);
  }
  if (tid == 0) {
    size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = fmax(fmax(r0[0], r0[1]), fmax(r0[2], r0[3]));
    part[2 * b + 1] = fmax(fmax(r1[0], r1[1]), fmax(r1[2], r1[3]));
  }
}

// the largest magnitudes from the n workgroup pairs, as the bit patterns of
// non-negative doubles; one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) k_mr_max(const double* part, long n,
                                                 unsigned long long* smax) {
  __shared__ double s0[1024], s1[1024];
  int tid = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (long q = tid; q < n; q += 1024) {
    a0 = fmax(a0, part[2 * q]);
    a1 = fmax(a1, part[2 * q + 1]);
  }
  s0[tid] = a0;
  s1[tid] = a1;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (tid < h) {
      s0[tid] = fmax(s0[tid], s0[tid + h]);
      s1[tid] = fmax(s1[tid], s1[tid + h]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    smax[0] = (unsigned long long)__double_as_longlong(s0[0]);
    smax[1] = (unsigned long long)__double_as_longlong(s1[0]);
  }
}

// Projection of both fields from level l+1 (2 nxc x 2 nyc) to level l: the
// mean of the four children, 0.25 ((c00 + c10) + (c01 + c11)).
__global__ void __launch_bounds__(256) k_mr_project(const double* f0, const double* f1,
                                                    double* c0, double* c1, int nxc, int nyc) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long)nxc * nyc) return;
  int i = (int)(q % nxc), j = (int)(q / nxc);
  size_t nxf = 2 * (size_t)nxc;
  size_t a = (size_t)(2 * j) * nxf + 2 * i, b = a + nxf;
  c0[q] = 0.25 * ((f0[a] + f0[a + 1]) + (f0[b] + f0[b + 1]));
  c1[q] = 0.25 * ((f1[a] + f1[a + 1]) + (f1[b] + f1[b + 1]));
}

// 5th-order prediction of child (2 ic + a, 2 jc + b) from the coarse level
// (nxc x nyc; neighbours outside clamped to the edge): u + s_a Q_x + s_b Q_y
// + s_a s_b Q_xy, s = +1 for the left / bottom child, in the evaluation
// order of the definition.
MMD double mr_predict(const double* u, int nxc, int nyc, int ic, int jc, int a, int b) {
  auto at = [&](int dj, int di) -> double {
    int jj = jc + dj, ii = ic + di;
    jj = jj < 0 ? 0 : (jj > nyc - 1 ? nyc - 1 : jj);
    ii = ii < 0 ? 0 : (ii > nxc - 1 ? nxc - 1 : ii);
    return u[(size_t)jj * nxc + ii];
  };
  double qx = MR_G1 * (at(0, 1) - at(0, -1)) + MR_G2 * (at(0, 2) - at(0, -2));
  double qy = MR_G1 * (at(1, 0) - at(-1, 0)) + MR_G2 * (at(2, 0) - at(-2, 0));
  auto t = [&](int m, int n) -> double {
    return (at(n, m) - at(-n, m)) - (at(n, -m) - at(-n, -m));
  };
  constexpr double C11 = MR_G1 * MR_G1, C12 = MR_G1 * MR_G2, C21 = MR_G2 * MR_G1,
                   C22 = MR_G2 * MR_G2;
  double qxy = ((C11 * t(1, 1) + C12 * t(1, 2)) + C21 * t(2, 1)) + C22 * t(2, 2);
  double sa = a == 0 ? 1.0 : -1.0, sb = b == 0 ? 1.0 : -1.0;
  return ((at(0, 0) + sa * qx) + sb * qy) + (sa * sb) * qxy;
}

// Details of level l+1 (fine, 2 nxc x 2 nyc) against the prediction from
// level l (coarse): a level-l block (bs x bs coarse cells, 2 bs x 2 bs fine)
// is flagged when a child cell's |detail| exceeds e times the field's
// largest magnitude, in either field.  One 16 x 16 tile of fine cells per
// workgroup; the flags of the blocks it touches go through LDS.
__global__ void __launch_bounds__(256) k_mr_detail(const double* c0, const double* c1,
                                                   const double* f0, const double* f1, int nxc,
                                                   int nyc, int bs, double e,
                                                   const unsigned long long* smax,
                                                   uint32_t* flag) {
  __shared__ uint32_t sf[MR_LOC * MR_LOC];
  int tid = threadIdx.x;
  int nxf = 2 * nxc, nyf = 2 * nyc, fbs = 2 * bs;
  int i0 = blockIdx.x * MR_TILE, j0 = blockIdx.y * MR_TILE;
  int fi = i0 + tid % MR_TILE, fj = j0 + tid / MR_TILE;
  MrTileFlags tf;
  tf.init(i0, j0, fbs);
  if (tid < MR_LOC * MR_LOC) sf[tid] = 0;
  __syncthreads();
  if (fi < nxf && fj < nyf) {
    double thr0 = e * __longlong_as_double((long long)smax[0]);
    double thr1 = e * __longlong_as_double((long long)smax[1]);
    int ic = fi >> 1, jc = fj >> 1, a = fi & 1, b = fj & 1;
    size_t q = (size_t)fj * nxf + fi;
    double d0 = f0[q] - mr_predict(c0, nxc, nyc, ic, jc, a, b);
    double d1 = f1[q] - mr_predict(c1, nxc, nyc, ic, jc, a, b);
    if (fabs(d0) > thr0 || fabs(d1) > thr1) sf[tf.local(fi, fj, fbs)] = 1;
  }
  __syncthreads();
  if (tid < tf.nlx * tf.nly && sf[tid]) {
    int bi = tf.bx0 + tid % tf.nlx, bj = tf.by0 + tid / tf.nlx;
    if (bi < nxc / bs && bj < nyc / bs) atomicOr(&flag[(size_t)bj * (nxc / bs) + bi], 1u);
  }
}

// Block structure, one workgroup.  Per level l: nbx[l] x nby[l] blocks at
// offset off[l] of the flag arrays; detail (l < L), iface (identifier of
// the solver-grid blocks at level L on entry), refine, exist.  Out: the
// leaf level of every solver-grid block, and per level the counts of
// existing and of leaf blocks.
struct MrLevels {
  int L, nbx[MR_MAXL + 1], nby[MR_MAXL + 1];
  long off[MR_MAXL + 1];
};
__global__ void __launch_bounds__(1024) k_mr_tree(MrLevels V, const uint32_t* detail,
                                                  uint32_t* iface, uint32_t* refine,
                                                  uint32_t* exist, int32_t* leaf,
                                                  unsigned long long* counts) {
  __shared__ unsigned long long s_cnt[2 * (MR_MAXL + 1)];
  int tid = threadIdx.x, T = blockDim.x, L = V.L;
  for (int x = tid; x < 2 * (L + 1); x += T) s_cnt[x] = 0;
  // identifiers of the coarser levels: any child
  for (int l = L - 1; l >= 0; l--) {
    for (int q = tid; q < V.nbx[l] * V.nby[l]; q += T) {
      int bi = q % V.nbx[l], bj = q / V.nbx[l], w = V.nbx[l + 1];
      const uint32_t* c = iface + V.off[l + 1];
      size_t a = (size_t)(2 * bj) * w + 2 * bi, b = a + w;
      iface[V.off[l] + q] = (c[a] | c[a + 1]) | (c[b] | c[b + 1]);
    }
    __syncthreads();
  }
  // refinement: identifier, or significant details in the 3 x 3 neighbourhood
  for (int l = 0; l < L; l++) {
    for (int q = tid; q < V.nbx[l] * V.nby[l]; q += T) {
      int bi = q % V.nbx[l], bj = q / V.nbx[l];
      uint32_t d = 0;
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) {
          int ii = bi + di, jj = bj + dj;
          if (ii >= 0 && ii < V.nbx[l] && jj >= 0 && jj < V.nby[l])
            d |= detail[V.off[l] + (size_t)jj * V.nbx[l] + ii];
        }
      refine[V.off[l] + q] = d | iface[V.off[l] + q];
    }
  }
  __syncthreads();
  // grading, from level L-1 up to level 1: the 3 x 3 neighbourhood of a
  // refined block must exist, so its members' parents are refined
  for (int l = L - 1; l >= 1; l--) {
    for (int q = tid; q < V.nbx[l] * V.nby[l]; q += T) {
      int bi = q % V.nbx[l], bj = q / V.nbx[l];
      uint32_t need = 0;
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) {
          int ii = bi + di, jj = bj + dj;
          if (ii >= 0 && ii < V.nbx[l] && jj >= 0 && jj < V.nby[l])
            need |= refine[V.off[l] + (size_t)jj * V.nbx[l] + ii];
        }
      if (need) refine[V.off[l - 1] + (size_t)(bj / 2) * V.nbx[l - 1] + bi / 2] = 1;
    }
    __syncthreads();
  }
  // existence, from the coarsest level down
  for (int q = tid; q < V.nbx[0] * V.nby[0]; q += T) exist[V.off[0] + q] = 1;
  __syncthreads();
  for (int l = 0; l < L; l++) {
    for (int q = tid; q < V.nbx[l + 1] * V.nby[l + 1]; q += T) {
      int bi = q % V.nbx[l + 1], bj = q / V.nbx[l + 1];
      size_t p = V.off[l] + (size_t)(bj / 2) * V.nbx[l] + bi / 2;
      exist[V.off[l + 1] + q] = refine[p] & exist[p];
    }
    __syncthreads();
  }
  // counts per level, and the leaf level of every solver-grid block
  for (int l = 0; l <= L; l++)
    for (int q = tid; q < V.nbx[l] * V.nby[l]; q += T) {
      uint32_t e = exist[V.off[l] + q];
      uint32_t lf = e && (l == L || !refine[V.off[l] + q]);
      if (e) atomicAdd(&s_cnt[2 * l], 1ull);
      if (lf) atomicAdd(&s_cnt[2 * l + 1], 1ull);
    }
  for (int q = tid; q < V.nbx[L] * V.nby[L]; q += T) {
    int bi = q % V.nbx[L], bj = q / V.nbx[L];
    int lv = 0;
    for (int l = L; l >= 0; l--) {
      int sh = L - l;
      if (exist[V.off[l] + (size_t)(bj >> sh) * V.nbx[l] + (bi >> sh)]) {
        lv = l;
        break;
      }
    }
    leaf[q] = lv;
  }
  __syncthreads();
  for (int x = tid; x < 2 * (L + 1); x += T) counts[x] = s_cnt[x];
}

}  // namespace mmfv
