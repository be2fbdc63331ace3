"""Multiresolution analysis of a 2D state (Sec. 2.4): the cell-average
pyramid, the prediction details, their level-dependent thresholding, and the
block structure they and the interface network produce.

TEST INFRASTRUCTURE ONLY: plain numpy in FP64, for the tests to check the
library's multiresolution kernels against.  Every array expression is
written in the evaluation order the definitions below state.

Definitions (Sec. 2.4 and the readings noted):

* Levels l = 0 (coarsest) .. L (the solver grid, nx x ny cells); level l has
  nx / 2^(L-l) x ny / 2^(L-l) cells, in blocks of B x B cells.
* Fields: the mixture density and total energy of a cell, the sums over the
  materials (in material order) of their conserved rho and rho E.
* Projection (the paper's P_{l+1 -> l}, tensor product in 2D): a coarse cell
  is the mean of its four children, 0.25 ((c00 + c10) + (c01 + c11)).
* Prediction (P_{l -> l+1}, 5th order, tensor product of the 1D operator):
  the child (2i + a, 2j + b) of coarse cell (i, j) is predicted as
  u + s_a Q_x + s_b Q_y + s_a s_b Q_xy, s = +1 for the left/bottom child and
  -1 for the right/top one, with
  Q_x = g1 (u[i+1] - u[i-1]) + g2 (u[i+2] - u[i-2]) (likewise Q_y) and
  Q_xy = sum over m, n in {1, 2} of g_m g_n (u[i+m, j+n] - u[i+m, j-n]
  - (u[i-m, j+n] - u[i-m, j-n])), g1 = -22/128, g2 = 3/128.  Reading: the
  paper prints the sums of the neighbours u[i+m] + u[i-m]; only their
  differences preserve constants and reproduce linear data, so the
  differences are meant (the operator of its reference).  Coarse neighbours
  outside the domain take the nearest cell's value (zero gradient).
* Detail of a level-(l+1) cell: d = u - prediction.  Reading: it is
  significant when |d| > eps_{l+1} s_v, with Harten's level-dependent
  threshold eps_l = 2^(2 (l - L)) eps and s_v the largest |value| of field v
  over the solver grid.
* A level-l block (l < L) has significant details when any of its 2B x 2B
  children cells at level l+1 has one (either field).
* Interface position identifier: a block of the solver grid is 1 when one
  of its cells lies in the narrow band of the interface network (level-set
  value below the band width); a block at a coarser level is 1 when any of
  its descendant blocks is (reading: such blocks are refined down to L).
* Refinement: a level-l block (l < L) is refined when it has identifier 1
  or when a block of its 3 x 3 neighbourhood at level l (itself included)
  has significant details (Harten's safety zone for waves that move; the
  band of the interface identifier is its own margin: reading).  Grading
  (reading): a refined block's 3 x 3 neighbourhood must exist, so the
  parents of those neighbours are refined too, from level L-1 up to
  level 1.  A block exists at level 0,
  and at level l+1 when its parent exists and is refined.
* Output: for every block of the solver grid, the level of the leaf that
  covers it; per level the counts of existing and of leaf blocks; the
  compression (leaf cells over solver cells).
"""
from __future__ import annotations

import numpy as np

G1 = -22.0 / 128.0
G2 = 3.0 / 128.0


def fields(Q):
    """Mixture density and total energy: sums over materials in material
    order of Q[r, 0] and Q[r, -1] ([M, nv, ny, nx] -> two [ny, nx])."""
    rho = Q[0, 0].copy()
    E = Q[0, -1].copy()
    for r in range(1, Q.shape[0]):
        rho = rho + Q[r, 0]
        E = E + Q[r, -1]
    return [rho, E]


def project(u):
    """Level l+1 -> l: the mean of the four children."""
    return 0.25 * ((u[0::2, 0::2] + u[0::2, 1::2]) + (u[1::2, 0::2] + u[1::2, 1::2]))


def predict(u):
    """Level l -> l+1 prediction of every child cell of u ([ny, nx] ->
    [2 ny, 2 nx]), neighbours outside clamped to the edge."""
    ny, nx = u.shape
    up = np.pad(u, 2, mode="edge")

    def at(dj, di):
        return up[2 + dj:2 + dj + ny, 2 + di:2 + di + nx]

    qx = G1 * (at(0, 1) - at(0, -1)) + G2 * (at(0, 2) - at(0, -2))
    qy = G1 * (at(1, 0) - at(-1, 0)) + G2 * (at(2, 0) - at(-2, 0))

    def t(m, n):
        return (at(n, m) - at(-n, m)) - (at(n, -m) - at(-n, -m))

    qxy = (((G1 * G1) * t(1, 1) + (G1 * G2) * t(1, 2)) + (G2 * G1) * t(2, 1)) + (G2 * G2) * t(2, 2)
    out = np.empty((2 * ny, 2 * nx))
    for b in (0, 1):
        for a in (0, 1):
            sa = 1.0 if a == 0 else -1.0
            sb = 1.0 if b == 0 else -1.0
            out[b::2, a::2] = ((u + sa * qx) + sb * qy) + (sa * sb) * qxy
    return out


def pyramid(u, L):
    """[level 0, ..., level L] of one field."""
    lev = [u]
    for _ in range(L):
        lev.append(project(lev[-1]))
    return lev[::-1]


def details(lev):
    """details[l] for l = 1..L (index l): u_l - predict(u_{l-1})."""
    return [None] + [lev[l] - predict(lev[l - 1]) for l in range(1, len(lev))]


def block_any(mask, B):
    """Per B x B block: any of its cells."""
    ny, nx = mask.shape
    return mask.reshape(ny // B, B, nx // B, B).any(axis=(1, 3))


def dilate(mask):
    """3 x 3 dilation inside the array."""
    ny, nx = mask.shape
    p = np.pad(mask, 1)
    out = np.zeros_like(mask)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            out |= p[1 + dj:1 + dj + ny, 1 + di:1 + di + nx]
    return out


def analyse(Q, phi, band, B=16, L=3, eps=1e-3):
    """The block structure of the state Q ([M, nv, ny, nx]) with level set
    phi ([ny, nx]); returns dict(leaf=[ny/B, nx/B] leaf level of every
    solver-grid block, detail=[per level l < L: [blocks] significant
    details], iface=[per level: identifier], refine, exist, counts)."""
    ny, nx = phi.shape
    if nx % (B << L) or ny % (B << L):
        raise ValueError("grid not divisible into blocks at every level")
    fl = fields(Q)
    scale = [float(np.abs(f).max()) for f in fl]
    det = [details(pyramid(f, L)) for f in fl]
    detail = []
    for l in range(L):
        e = (2.0 ** (2 * (l + 1 - L))) * eps
        sig = np.zeros((ny >> (L - l - 1), nx >> (L - l - 1)), bool)
        for v in range(len(fl)):
            sig |= np.abs(det[v][l + 1]) > e * scale[v]
        # children cells of a level-l block: 2B x 2B cells of level l+1
        detail.append(block_any(sig, 2 * B))
    iface = [None] * (L + 1)
    iface[L] = block_any(phi < band, B)
    for l in range(L - 1, -1, -1):
        m = iface[l + 1]
        iface[l] = (m[0::2, 0::2] | m[0::2, 1::2]) | (m[1::2, 0::2] | m[1::2, 1::2])
    out = build_tree(detail, iface, L, B, nx * ny)
    out.update(detail=detail, iface=iface, scale=scale)
    return out


def build_tree(detail, iface, L, B=16, cells=None):
    """Refinement, grading, existence and leaves from the per-level block
    flags: detail[l] (l < L) and iface[l] (l <= L)."""
    refine = [dilate(detail[l]) | iface[l] for l in range(L)] + [None]
    for l in range(L - 1, 0, -1):
        need = dilate(refine[l])
        par = (need[0::2, 0::2] | need[0::2, 1::2]) | (need[1::2, 0::2] | need[1::2, 1::2])
        refine[l - 1] = refine[l - 1] | par
    exist = [np.ones_like(iface[0])]
    for l in range(L):
        r = refine[l] & exist[l]
        exist.append(np.repeat(np.repeat(r, 2, axis=0), 2, axis=1))
    leaf = np.zeros(iface[L].shape, np.int32)
    counts = []
    for l in range(L + 1):
        e = exist[l]
        isleaf = e if l == L else e & ~refine[l]
        counts.append((int(e.sum()), int(isleaf.sum())))
        rep = 1 << (L - l)
        leaf[np.repeat(np.repeat(e, rep, axis=0), rep, axis=1)] = l
    if cells is None:
        cells = iface[L].size * B * B
    comp = sum(c[1] for c in counts) * B * B / float(cells)
    return dict(leaf=leaf, refine=refine[:L], exist=exist, counts=counts, compression=comp)
