"""Pins of the oracle's second face-flux variant: Roe's approximate Riemann
solver on states from characteristic-wise WENO5 (the projection of the
stencil's conserved states onto the characteristic fields of the face's Roe
average; Sec. 3 names WENO5 as the scheme's reconstruction).

* Roe flux identities: consistency F(U, U) = F(U); a contact at rest passes
  only its pressure; a stationary Rankine-Hugoniot shock passes its exact
  flux (Roe's linearisation resolves both exactly).
* The step with this flux: exact Sod solution with L1 errors that fall
  under refinement; fifth-order convergence on a smooth density wave; the
  three-material stiffened-gas tube against its two exact Riemann problems;
  uniform pressure across interfaces stays at rest.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from exact_riemann import Side, sample


def flux(W, g, pinf=0.0):
    r, u, v, p = W
    E = (p + g * pinf) / (g - 1) + 0.5 * r * (u * u + v * v)
    return np.array([r * u, r * u * u + p, r * u * v, u * (E + p)])


@pytest.fixture(scope="module")
def o1():
    cfg = wl.shock_tube_1d()["cfg"]
    cfg["flux"] = 1
    return oracle.Oracle(cfg)


def test_roe_consistency(o1):
    for m, W in ((0, [1.0, 0.3, -0.2, 1.0]), (2, [1.0, -0.4, 0.1, 2.0])):
        g, pinf = (1.4, 0.0) if m == 0 else (4.4, 6.0)
        assert np.allclose(o1.roe(m, W, W), flux(np.array(W), g, pinf), rtol=1e-14, atol=1e-14)


def test_roe_contact_at_rest(o1):
    F = o1.roe(0, [1.0, 0.0, 0.3, 1.0], [0.125, 0.0, -0.2, 1.0])
    assert np.allclose(F, [0.0, 1.0, 0.0, 0.0], atol=1e-14)


def test_roe_stationary_shock_exact(o1):
    g = 1.4
    M = 2.0
    rL, uL, pL = 1.0, M * math.sqrt(g), 1.0
    rR = rL * (g + 1) * M * M / ((g - 1) * M * M + 2)
    uR = rL * uL / rR
    pR = pL * (2 * g * M * M - (g - 1)) / (g + 1)
    WL, WR = np.array([rL, uL, 0.0, pL]), np.array([rR, uR, 0.0, pR])
    F = o1.roe(0, WL, WR)
    assert np.allclose(F, flux(WL, g), rtol=1e-13)
    assert np.allclose(flux(WL, g), flux(WR, g), rtol=1e-13)


def single_1d(n, left, right, flux_kind=1, x_if=0.5, gamma=1.4, bc=wl.BC_TRANSMISSIVE):
    x = (np.arange(n) + 0.5) / n
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=1, gamma=[gamma], pinf=[0.0], bc=[bc] * 4)
    cfg["flux"] = flux_kind
    W = np.where(x < x_if, np.array(left)[:, None], np.array(right)[:, None])
    return cfg, np.full((1, n), 8.0 / n), np.zeros((1, n), np.int32), W[None, :, None, :]


def test_roe_sod_exact_and_converges():
    errs = []
    for n in (100, 200, 400):
        cfg, phi, chi, W = single_1d(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
        o = oracle.Oracle(cfg)
        assert o.init(phi, chi, W) == 0
        while o.diag()["t"] < 0.15:
            assert o.step(1) == 0
        t = o.diag()["t"]
        x = (np.arange(n) + 0.5) / n
        re, _, _ = sample(Side(1.0, 0.0, 1.0, 1.4), Side(0.125, 0.0, 0.1, 1.4), (x - 0.5) / t)
        errs.append(np.abs(o.get()["Q"][0, 0, 0] - re).mean())
    print(errs)
    assert errs[0] < 0.01
    assert errs[0] > errs[1] > errs[2]


def test_roe_smooth_density_wave_converges_at_high_order():
    """A smooth density bump (u = 1, p = 1: a pure contact wave) advected
    for t = 0.1; L1 error of the density against the exact translated cell
    averages falls at about fifth order."""
    from scipy.integrate import quad
    bump = lambda s: 1.0 + 0.2 * np.exp(-((s - 0.4) / 0.08) ** 2)
    errs = []
    for n in (40, 80, 160):
        x = (np.arange(n) + 0.5) / n
        cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=1, gamma=[1.4], pinf=[0.0],
                             bc=[wl.BC_TRANSMISSIVE] * 4)
        cfg["flux"] = 1
        cfg["cfl"] = 0.2
        rho = np.array([quad(bump, xi - 0.5 / n, xi + 0.5 / n)[0] * n for xi in x])
        W = np.stack([rho, np.ones(n), np.ones(n)])[None, :, None, :]
        o = oracle.Oracle(cfg)
        assert o.init(np.full((1, n), 8.0 / n), np.zeros((1, n), np.int32), W) == 0
        while o.diag()["t"] < 0.1:
            assert o.step(1) == 0
        t = o.diag()["t"]
        ex = np.array([quad(lambda s: bump(s - t), xi - 0.5 / n, xi + 0.5 / n)[0] * n for xi in x])
        errs.append(np.abs(o.get()["Q"][0, 0, 0] - ex).mean())
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    print(errs, orders)
    assert orders[-1] > 4.0


def test_roe_three_material_tube_against_exact_riemann_problems():
    w = wl.shock_tube_1d()
    w["cfg"]["flux"] = 1
    o = oracle.run(w)
    t = o.diag()["t"]
    g = o.get()
    n = w["cfg"]["nx"]
    x = (np.arange(n) + 0.5) / n
    chi = g["chi"][0]
    # interfaces follow the exact contacts within one cell
    A = Side(1.0, 0.0, 1.0, 1.4)
    B = Side(0.125, 0.0, 0.1, 1.667)
    C = Side(1.0, 0.0, 1.0, 4.4, 6.0)
    from exact_riemann import star_state
    _, u1 = star_state(A, B)
    _, u2 = star_state(B, C)
    i1 = x[np.nonzero(chi == 1)[0][0]] - 0.5 / n
    i2 = x[np.nonzero(chi == 2)[0][0]] - 0.5 / n
    assert abs(i1 - (0.3 + u1 * t)) <= 1.0 / n
    assert abs(i2 - (0.6 + u2 * t)) <= 1.0 / n
    # densities against the superposition of the two exact solutions
    re = np.where(x < 0.45, sample(A, B, (x - 0.3) / t)[0], sample(B, C, (x - 0.6) / t)[0])
    rho = np.array([g["Q"][chi[i], 0, 0, i] / g["alpha"][chi[i], 0, i] for i in range(n)])
    err = np.abs(rho - re).mean()
    print("L1 density", err)
    assert err < 0.02


def test_roe_uniform_pressure_stays_at_rest():
    w = wl.uniform_pressure_2d(shape="circle", steps=60)
    w["cfg"]["flux"] = 1
    o = oracle.run(w)
    g = o.get()
    Q, al = g["Q"], g["alpha"]
    for m in range(3):
        on = al[m] > 1e-3
        for v in (1, 2):
            assert np.abs(Q[m, v][on]).max() <= 1e-12


def test_roe_sonic_rarefaction_no_expansion_shock():
    """Toro's test 1 (a left rarefaction containing a sonic point): with the
    entropy fix the fan is smooth and matches the exact solution; Roe's flux
    without it leaves an expansion shock at the sonic point."""
    n = 200
    cfg, phi, chi, W = single_1d(n, (1.0, 0.75, 1.0), (0.125, 0.0, 0.1), x_if=0.3)
    o = oracle.Oracle(cfg)
    assert o.init(phi, chi, W) == 0
    while o.diag()["t"] < 0.2:
        assert o.step(1) == 0
    t = o.diag()["t"]
    x = (np.arange(n) + 0.5) / n
    re, _, _ = sample(Side(1.0, 0.75, 1.0, 1.4), Side(0.125, 0.0, 0.1, 1.4), (x - 0.3) / t)
    rho = o.get()["Q"][0, 0, 0]
    # inside the fan (exact density between its head and tail values) the
    # largest jump between neighbouring cells stays small
    fan = (re < 0.999) & (re > 0.43) & (x < 0.5)
    jumps = np.abs(np.diff(rho[fan]))
    assert jumps.max() < 0.03, jumps.max()
    assert np.abs(rho - re).mean() < 0.01


def test_roe_tangential_velocity_galilean():
    """A 2D Sod problem varying in x only: adding a uniform tangential
    velocity leaves the density field unchanged (the Roe sound speed
    c^2 = (gamma-1)(H - |u|^2/2) does not see it), to rounding."""
    nx, ny = 64, 4
    out = []
    for vt in (0.0, 0.5):
        cfg = wl.base_config(dim=2, nx=nx, ny=ny, n_mat=1, x1=1.0, y1=ny / nx, gamma=[1.4],
                             pinf=[0.0], bc=[wl.BC_TRANSMISSIVE] * 4)
        cfg["flux"] = 1
        x = (np.arange(nx) + 0.5) / nx
        r = np.where(x < 0.5, 1.0, 0.125)
        p = np.where(x < 0.5, 1.0, 0.1)
        W = np.zeros((1, 4, ny, nx))
        W[0, 0], W[0, 2], W[0, 3] = r, vt, p
        o = oracle.Oracle(cfg)
        assert o.init(np.full((ny, nx), 8.0 / nx), np.zeros((ny, nx), np.int32), W) == 0
        o.set_dt(0.6 / nx / 2.5)
        assert o.step(40) == 0
        out.append(o.get()["Q"][0, 0])
    assert np.allclose(out[0], out[1], rtol=1e-12, atol=1e-13)
