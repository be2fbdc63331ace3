"""Pins of the oracle's cut-cell geometry (Sec. 2.3: volume fractions,
apertures, interface segment; Sec. 2.3.1: volume-fraction correction).

Straight interfaces with exact signed distance are reproduced exactly by the
piecewise-linear geometry, so volume fractions, apertures and the interface
closure vector are compared against polygon clipping written here.  Circles
converge at second order.  Face-aligned interfaces exercise the tie rule
(values derived by hand)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def clip_halfplane(poly, n, d):
    """Sutherland-Hodgman: part of polygon with n.x < d."""
    out = []
    m = len(poly)
    for k in range(m):
        P, Q = poly[k], poly[(k + 1) % m]
        fp, fq = d - (n[0] * P[0] + n[1] * P[1]), d - (n[0] * Q[0] + n[1] * Q[1])
        if fp >= 0:
            out.append(P)
        if (fp > 0 > fq) or (fp < 0 < fq):
            t = fp / (fp - fq)
            out.append((P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1])))
    return out


def area(poly):
    if len(poly) < 3:
        return 0.0
    s = 0.0
    for k in range(len(poly)):
        (x0, y0), (x1, y1) = poly[k], poly[(k + 1) % len(poly)]
        s += x0 * y1 - x1 * y0
    return 0.5 * abs(s)


def seg_inside(a, b, n, d):
    fa, fb = d - (n[0] * a[0] + n[1] * a[1]), d - (n[0] * b[0] + n[1] * b[1])
    if fa >= 0 and fb >= 0:
        return 1.0
    if fa <= 0 and fb <= 0:
        return 0.0
    return max(fa, fb) / abs(fa - fb)


def line_case(theta, offset, nx=24, ny=20):
    L = 1.0
    h = L / nx
    cfg = wl.base_config(dim=2, nx=nx, ny=ny, x0=0.0, x1=L, y0=0.0, y1=ny * h,
                         n_mat=2, gamma=[1.4, 1.4], pinf=[0.0, 0.0],
                         bc=[wl.BC_TRANSMISSIVE] * 4, band_ls=40)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    n = (math.cos(theta), math.sin(theta))
    s = n[0] * X + n[1] * Y - offset
    phi = np.abs(s)
    chi = (s > 0).astype(np.int32)
    W = np.ones((2, 4, ny, nx))
    W[:, 1:3] = 0.0
    o = oracle.Oracle(cfg)
    assert o.init(phi, chi, W) == 0
    return o, n, offset, h, X, Y


@pytest.mark.parametrize("theta,offset", [(0.3, 0.47), (1.1, 0.52), (2.5, -0.2),
                                          (-0.7, 0.05), (0.7853981, 0.49)])
def test_straight_line_exact(theta, offset):
    o, n, d, h, X, Y = line_case(theta, offset)
    g = o.get()
    Ax, Ay = o.apertures()
    cx, cy = o.closure()
    ny, nx = X.shape
    worst = 0.0
    for j in range(2, ny - 2):  # keep away from the domain frame
        for i in range(2, nx - 2):
            x0, y0 = X[j, i] - h / 2, Y[j, i] - h / 2
            sq = [(x0, y0), (x0 + h, y0), (x0 + h, y0 + h), (x0, y0 + h)]
            a0 = area(clip_halfplane(sq, n, d)) / (h * h)
            worst = max(worst, abs(g["alpha"][0, j, i] - a0),
                        abs(g["alpha"][1, j, i] - (1 - a0)))
            # apertures of the west and south faces
            aw = seg_inside((x0, y0), (x0, y0 + h), n, d)
            as_ = seg_inside((x0, y0), (x0 + h, y0), n, d)
            worst = max(worst, abs(Ax[0, j, i] - aw), abs(Ay[0, j, i] - as_))
            assert Ax[0, j, i] + Ax[1, j, i] == pytest.approx(1.0, abs=2e-16)
            # closure vector of material 0: inward normal (-n) times chord
            poly = clip_halfplane(sq, n, d)
            chord = 0.0
            for k in range(len(poly)):
                P, Q = poly[k], poly[(k + 1) % len(poly)]
                on = lambda q: abs(n[0] * q[0] + n[1] * q[1] - d) < 1e-12
                if on(P) and on(Q):
                    chord = math.hypot(Q[0] - P[0], Q[1] - P[1])
            worst = max(worst, abs(cx[0, j, i] + n[0] * chord),
                        abs(cy[0, j, i] + n[1] * chord) / 1.0)
    assert worst < 1e-13


def test_circle_area_second_order():
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        cfg = wl.base_config(dim=2, nx=n, ny=n, x0=0, x1=1, y0=0, y1=1, n_mat=2,
                             gamma=[1.4, 1.4], pinf=[0, 0], band_ls=8)
        x = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x, x)
        dd = np.hypot(X - 0.51, Y - 0.47)
        phi = np.minimum(np.abs(dd - 0.3), 8 * h)
        chi = (dd <= 0.3).astype(np.int32)
        W = np.ones((2, 4, n, n))
        W[:, 1:3] = 0
        o = oracle.Oracle(cfg)
        assert o.init(phi, chi, W) == 0
        a = o.get()["alpha"][1].sum() * h * h
        errs.append(abs(a - math.pi * 0.09))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_1d_face_aligned_tie_rule():
    # interface exactly on the face x = 0.5 of an 8-cell grid (dyadic values,
    # so the zero is exact): the face is owned by the smaller indicator (0),
    # so A^0 = 1 there and A^1 = 0; alpha is 1/0 on either side, and the
    # interface segment lives in the first cell of material 1
    cfg = wl.base_config(dim=1, nx=8, n_mat=2, gamma=[1.4, 1.4], pinf=[0, 0],
                         band_ls=8)
    x = (np.arange(8) + 0.5) / 8
    phi = np.abs(x - 0.5).reshape(1, 8)
    chi = (x > 0.5).astype(np.int32).reshape(1, 8)
    W = np.ones((2, 3, 1, 8))
    W[:, 1] = 0
    o = oracle.Oracle(cfg)
    assert o.init(phi, chi, W) == 0
    g = o.get()
    Ax, _ = o.apertures()
    assert g["alpha"][0, 0].tolist() == [1.0] * 4 + [0.0] * 4
    assert g["alpha"][1, 0].tolist() == [0.0] * 4 + [1.0] * 4
    assert Ax[0, 0].tolist() == [1.0] * 5 + [0.0] * 4
    assert Ax[1, 0].tolist() == [0.0] * 5 + [1.0] * 4
    cx, _ = o.closure()
    assert cx[0, 0, 4] == -1.0 and cx[1, 0, 4] == 1.0
    assert cx[0, 0, 3] == 0.0 and cx[1, 0, 3] == 0.0


def test_1d_interface_mid_cell():
    # interface at x = 17/32, a quarter into cell 4 (dyadic, exact)
    cfg = wl.base_config(dim=1, nx=8, n_mat=2, gamma=[1.4, 1.4], pinf=[0, 0],
                         band_ls=8)
    x = (np.arange(8) + 0.5) / 8
    phi = np.abs(x - 17 / 32).reshape(1, 8)
    chi = (x > 17 / 32).astype(np.int32).reshape(1, 8)
    W = np.ones((2, 3, 1, 8))
    W[:, 1] = 0
    o = oracle.Oracle(cfg)
    assert o.init(phi, chi, W) == 0
    g = o.get()
    assert g["alpha"][0, 0, 4] == 0.25
    assert g["alpha"][1, 0, 4] == 0.75
    cx, _ = o.closure()
    assert cx[0, 0, 4] == -1.0 and cx[1, 0, 4] == 1.0


def y_junction(n=16, rho=(1.0, 2.0, 0.5)):
    """Three sectors meeting at a point inside a cell, rays 120 deg apart."""
    h = 1.0 / n
    cfg = wl.base_config(dim=2, nx=n, ny=n, x0=0, x1=1, y0=0, y1=1, n_mat=3,
                         gamma=[1.4, 1.5, 1.6], pinf=[0, 0, 0], band_ls=8)
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    c = (0.5 + 0.3 * h, 0.5 + 0.2 * h)
    ang = np.arctan2(Y - c[1], X - c[0])
    rays = [0.1, 0.1 + 2 * np.pi / 3, 0.1 + 4 * np.pi / 3]
    d = np.full(X.shape, np.inf)
    for t in rays:
        ux, uy = np.cos(t), np.sin(t)
        s_ = np.maximum((X - c[0]) * ux + (Y - c[1]) * uy, 0.0)
        d = np.minimum(d, np.hypot(X - c[0] - s_ * ux, Y - c[1] - s_ * uy))
    sector = np.mod(ang - 0.1, 2 * np.pi) // (2 * np.pi / 3)
    chi = sector.astype(np.int32)
    W = np.zeros((3, 4, n, n))
    for m in range(3):
        W[m, 0] = rho[m]
        W[m, 3] = 1.0
    return cfg, np.minimum(d, 8 * h), chi, W


def test_three_material_correction():
    # a junction inside a cell: cells holding three materials end with
    # sum(alpha) = 1; the cell's own material is never changed, and the
    # defect goes to the non-primary material of least mass alpha*rho
    cfg, phi, chi, W = y_junction()
    o1 = oracle.Oracle(cfg)
    assert o1.init(phi, chi, W) == 0
    a1 = o1.get()["alpha"]
    three = (a1 > 0).sum(0) >= 3
    assert three.any()
    assert np.all(np.abs(a1.sum(0)[three] - 1.0) <= 4e-16)
    # two runs that differ only in which non-primary material is the
    # lightest: each correction changes exactly that material, by the same
    # defect 1 - sum(uncorrected alpha), and never the primary
    for prim in range(3):
        o1_, o2_ = [m for m in range(3) if m != prim]
        runs = []
        for light in (o1_, o2_):
            rho = [1.0, 1.0, 1.0]
            rho[light] = 1e-3
            rho[o2_ if light == o1_ else o1_] = 5.0
            _, _, _, W2 = y_junction(rho=tuple(rho))
            o2 = oracle.Oracle(cfg)
            assert o2.init(phi, chi, W2) == 0
            runs.append(o2.get()["alpha"])
        aA, aB = runs
        for j, i in zip(*np.where(three & (chi == prim))):
            assert aA[prim, j, i] == aB[prim, j, i] == a1[prim, j, i]
            dA = aA[o1_, j, i] - aB[o1_, j, i]
            dB = aB[o2_, j, i] - aA[o2_, j, i]
            assert dA == pytest.approx(dB, abs=1e-15)
