"""Pins of the oracle's redistancing of the regional level set (a reading:
the paper describes no reinitialisation; the pass after every time step
keeps the distance field from degenerating in stretched layers).

* a straight interface at any angle, given its exact distance: the
  interface cells get the exact distance back (the distance to the line
  through the two axis crossings is exact for a straight interface), and
  the band beyond stays within the 8-neighbour path bias of the exact one;
* a degenerate field (all zero in the band of a vertical interface) gets
  the exact distances h/2, 3h/2, ... back, and the crossing between the two
  materials stays where the linear interpolation put it;
* the conserved state and the material indicator are untouched, the volume
  fractions follow the new level set;
* the whole step with the pass on keeps the per-material totals to 1e-13.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def two_gas(nx, ny, phi, chi, L=1.0):
    cfg = wl.base_config(dim=2, nx=nx, ny=ny, n_mat=2, x0=0.0, x1=L * nx / ny, y0=0.0, y1=L,
                         gamma=[1.4, 1.6], pinf=[0.0, 0.0], bc=[wl.BC_REFLECTIVE] * 4, reinit=1)
    W = np.zeros((2, 4, ny, nx))
    W[:, 0] = [[[1.0]], [[0.5]]]
    W[:, 3] = 1.0
    return cfg, dict(phi=phi, chi=chi, W=W)


def line_field(n, theta, c0=0.513):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    nx_, ny_ = math.cos(theta), math.sin(theta)
    s = (X - 0.5) * nx_ + (Y - c0) * ny_  # signed distance to the line
    chi = (s > 0).astype(np.int32)
    return np.minimum(np.abs(s), 8 * h), chi, s, h


@pytest.mark.parametrize("theta", [0.0, 0.3, math.pi / 4, 1.1, math.pi / 2])
def test_straight_interface(theta):
    """Interface cells with crossings on both axes get the exact distance;
    a crossing on one axis only gives the distance along that axis (at most
    1/cos of the angle between normal and axis too long); the band beyond
    stays within the 8-neighbour path bias (1/cos 22.5 deg = 1.0824)."""
    n = 64
    phi, chi, s, h = line_field(n, theta)
    cfg, st = two_gas(n, n, phi, chi)
    o = oracle.Oracle(cfg)
    assert o.init(st["phi"], st["chi"], st["W"]) == 0
    o.reinit()
    g = o.get()
    new = g["phi"]
    assert np.array_equal(g["chi"], chi)
    cx = np.zeros_like(chi, bool)
    cy = np.zeros_like(chi, bool)
    cx[:, 1:] |= chi[:, 1:] != chi[:, :-1]
    cx[:, :-1] |= chi[:, :-1] != chi[:, 1:]
    cy[1:, :] |= chi[1:, :] != chi[:-1, :]
    cy[:-1, :] |= chi[:-1, :] != chi[1:, :]
    both = cx & cy
    if both.any():
        assert np.abs(new[both] - phi[both]).max() <= 1e-12
    ax = min(abs(math.cos(theta)), abs(math.sin(theta)))
    f = max(1.0824, 1.0 / max(ax, 1e-300)) if 0 < ax < 1 - 1e-12 else 1.0824
    band = phi < 8 * h
    assert np.all(new[band] >= phi[band] - 1e-12)
    assert np.all(new[band] <= np.minimum(phi[band] * f + 1e-12, 8 * h)), theta
    if ax < 1e-12 or ax > 1 - 1e-12:  # axis-aligned: exact everywhere in the band
        assert np.abs(new[band] - phi[band]).max() <= 1e-12


def test_degenerate_band_restored():
    """A vertical interface between columns 9 and 10 with phi = 0 in every
    band cell: the crossing is taken at the face (h/2 each side) and the
    distances h/2 + m h come back along the rows."""
    nx, ny = 24, 8
    h = 1.0 / ny
    chi = np.zeros((ny, nx), np.int32)
    chi[:, 10:] = 1
    phi = np.full((ny, nx), 8 * h)
    phi[:, 3:17] = 0.0
    cfg, st = two_gas(nx, ny, phi, chi)
    o = oracle.Oracle(cfg)
    assert o.init(st["phi"], st["chi"], st["W"]) == 0
    o.reinit()
    new = o.get()["phi"]
    want = np.abs(np.arange(nx) - 9.5) * h
    for j in range(ny):
        assert np.allclose(new[j, 3:17], want[3:17], rtol=0, atol=1e-15)
        assert np.all(new[j, :3] == 8 * h) and np.all(new[j, 17:] == 8 * h)
    # the volume fractions follow: the interface on the face between columns
    al = o.get()["alpha"]
    assert np.all(al[0, :, :10] == 1.0) and np.all(al[0, :, 10:] == 0.0)


def test_state_untouched_and_geometry_follows():
    n = 48
    phi, chi, s, h = line_field(n, 0.7)
    cfg, st = two_gas(n, n, phi * 0.3, chi)  # a squeezed field: crossings kept
    o = oracle.Oracle(cfg)
    assert o.init(st["phi"], st["chi"], st["W"]) == 0
    Q0 = o.get()["Q"].copy()
    o.reinit()
    g = o.get()
    assert np.array_equal(g["Q"], Q0)
    assert np.array_equal(g["chi"], chi)
    # the field is a distance again near the interface: the interface cells
    # take their distance from the crossings, which the scaling does not move
    ref = oracle.Oracle(cfg)
    assert ref.init(phi, chi, st["W"]) == 0
    ref.reinit()
    r = ref.get()
    assert np.abs(g["phi"] - r["phi"])[phi < 3 * h].max() <= 1e-12
    assert np.abs(g["alpha"] - r["alpha"]).max() <= 1e-12


def test_step_conserves_with_reinit():
    w = wl.triple_point(nx=112, ny=48)
    w["cfg"]["reinit"] = 1
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    q0 = o.get()["Q"]
    assert o.step(60) == 0
    q1 = o.get()["Q"]
    for m in range(3):
        m0, m1 = math.fsum(q0[m, 0].ravel()), math.fsum(q1[m, 0].ravel())
        xf = o.diag()["xfer"][m, 0]
        assert abs(m1 - m0 - xf) <= 1e-13 * m0, m
