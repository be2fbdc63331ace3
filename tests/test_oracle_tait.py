"""Pins of the oracle's Tait material (Sec. 2.1: p = B (rho/rho0)^gamma - B +
p0 for water-like fluids; Table 2's water, gamma = 7.15, rho0 = 1000):

* the exact Riemann problem between compressed air and water at rest, with
  the water barotropic (tests/exact_riemann.py, TaitSide): contact position,
  star pressure, water-shock position, and L1 errors that fall under grid
  refinement;
* the speed of a small acoustic pulse in water, c0 = sqrt(gamma B / rho0);
* a static air-water configuration at uniform pressure (1D and a 2D water
  column) stays at rest.
"""
import math

import numpy as np
import pytest

import exact_riemann as er
import oracle
import workloads as wl

WATER = wl.WATER


def run_to(w, T):
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    while o.diag()["t"] < T:
        assert o.step(1) == 0
    return o


def profiles(o):
    g = o.get()
    Q, chi = g["Q"][:, :, 0, :], g["chi"][0]
    al = g["alpha"][:, 0, :]
    n = chi.size
    rho, u = np.zeros(n), np.zeros(n)
    for i in range(n):
        m = chi[i]
        rho[i] = Q[m, 0, i] / al[m, i]
        u[i] = Q[m, 1, i] / Q[m, 0, i]
    return rho, u, chi


def exact(t, x, x0, air):
    L = er.Side(air[0], air[1], air[2], 1.4)
    R = er.TaitSide(1000.0, 0.0, None, WATER["gamma"], WATER["B"], WATER["rho0"], WATER["p0"])
    rho, u, p = er.sample(L, R, (x - x0) / t)
    return rho, u, p, er.wave_speeds(L, R)


def test_air_water_riemann_problem_exact():
    air = (50.0, 0.0, 1000.0)
    errs = []
    for n in (200, 400, 800):
        w = wl.air_water_tube_1d(n=n, air=air)
        x0 = 0.5 + 0.3 / n
        o = run_to(w, 0.05)
        t = o.diag()["t"]
        x = (np.arange(n) + 0.5) / n
        rho, u, chi = profiles(o)
        rho_e, u_e, p_e, (ps, us, waves) = exact(t, x, x0, air)
        dx = 1.0 / n
        # the interface (last cell of air) moves with the contact speed
        xi = x[np.nonzero(chi == 1)[0][0]] - 0.5 * dx
        assert abs(xi - (x0 + us * t)) <= 1.0 * dx, (n, xi, x0 + us * t)
        # star pressure in the water between contact and shock (Tait pressure
        # of the computed density) within 1 %
        sh = x0 + waves["right"][0] * t
        mid = (x > x0 + us * t + 8 * dx) & (x < sh - 8 * dx)
        p_w = WATER["B"] * (rho[mid] / WATER["rho0"]) ** WATER["gamma"] - WATER["B"] + WATER["p0"]
        assert np.all(np.abs(p_w - ps) <= 0.01 * ps), (n, p_w.min(), p_w.max(), ps)
        # the water shock: density half-way between the two sides within 2 cells
        half = 0.5 * (rho_e[mid][0] + 1000.0)
        water = np.nonzero((chi == 1) & (x > x0 + us * t))[0]
        above = water[rho[water] > half]
        xs = x[above[-1]] + 0.5 * dx
        assert abs(xs - sh) <= 2.0 * dx, (n, xs, sh)
        errs.append((np.mean(np.abs(rho - rho_e) / np.where(chi == 1, 1000.0, air[0])),
                     np.mean(np.abs(u - u_e))))
    print(errs)
    for a, b in zip(errs, errs[1:]):
        assert b[0] < a[0] and b[1] < a[1]


def test_acoustic_pulse_speed_in_water():
    """A small symmetric density pulse in water at rest splits into two
    halves travelling at -+ c0 = sqrt(gamma B / rho0)."""
    n, L = 800, 2.0
    x = (np.arange(n) + 0.5) * (L / n)
    dx = L / n
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=1, x1=L, gamma=[1.4], pinf=[0.0])
    wl.tait_config(cfg, [0])
    rho = WATER["rho0"] * (1.0 + 1e-5 * np.exp(-((x - 1.0) / 0.05) ** 2))
    W = np.stack([rho, np.zeros(n), wl.tait_pressure(rho)])[None, :, None, :]
    w = dict(cfg=cfg, phi=np.full((1, n), 8 * dx), chi=np.zeros((1, n), np.int32), W=W)
    o = run_to(w, 0.1)
    t = o.diag()["t"]
    d = o.get()["Q"][0, 0, 0] - WATER["rho0"]
    c0 = math.sqrt(WATER["gamma"] * WATER["B"] / WATER["rho0"])
    for side in (x > 1.0, x < 1.0):
        k = np.nonzero(side)[0][np.argmax(d[side])]
        # parabola through the maximum and its neighbours
        a, b, c = d[k - 1], d[k], d[k + 1]
        xp = x[k] + 0.5 * dx * (a - c) / (a - 2 * b + c)
        dist = abs(xp - 1.0)
        assert abs(dist - c0 * t) <= 0.25 * dx, (dist, c0 * t)


@pytest.mark.parametrize("dim", [1, 2])
def test_air_water_uniform_pressure_stays_at_rest(dim):
    if dim == 1:
        w = wl.air_water_tube_1d(n=120, air=(1.0, 0.0, 1.0))
        w["cfg"]["bc"] = [wl.BC_REFLECTIVE] * 4
    else:
        nx, ny = 48, 40
        x = (np.arange(nx) + 0.5) / 40.0
        y = (np.arange(ny) + 0.5) / 40.0
        X, Y = np.meshgrid(x, y)
        d = np.sqrt((X - 0.6) ** 2 + (Y - 0.5) ** 2) - 0.27
        cfg = wl.base_config(dim=2, nx=nx, ny=ny, n_mat=2, x1=1.2, y1=1.0, gamma=[1.4, 1.4],
                             pinf=[0.0, 0.0], bc=[wl.BC_REFLECTIVE] * 4)
        wl.tait_config(cfg, [1])
        W = np.zeros((2, 4, ny, nx))
        W[0, 0], W[0, 3] = 1.0, 1.0
        W[1, 0], W[1, 3] = 1000.0, 1.0
        w = dict(cfg=cfg, phi=np.minimum(np.abs(d), 8.0 / 40.0), chi=(d <= 0).astype(np.int32),
                 W=W)
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    assert o.step(100) == 0
    g = o.get()
    Q, al = g["Q"], g["alpha"]
    nv = Q.shape[1]
    for m, rho0 in ((0, 1.0), (1, 1000.0)):
        a = al[m]
        on = a > 1e-3
        r = Q[m, 0][on] / a[on]
        assert np.all(np.abs(r - rho0) <= 1e-12 * rho0), (m, np.abs(r - rho0).max())
        for v in range(1, nv - 1):
            assert np.all(np.abs(Q[m, v][on]) <= 1e-12 * rho0)
