"""Seeded synthetic initial conditions for the cut-cell multi-material solver.

This module only builds inputs: grids, the regional level set (unsigned
distance phi >= 0 plus integer indicator chi, Sec. 2.2) and per-material
primitive fields W = (rho, u, [v], p).  It contains none of the solver's
arithmetic, so both the CPU oracle and the HIP library can consume the same
arrays.

Workloads (all FP64, three materials, stiffened-gas EOS):

* ``shock_tube_1d``   -- 400-cell three-material tube on [0, 1], interfaces at
  0.3 and 0.6, transmissive ends.
* ``triple_point``    -- Case III of Sec. 3 (7 x 3 domain, reflective walls);
  the region [1,7]x[0,1.5] is the paper's garbled "[1,1]x[0,1.5]".
* ``shock_bubble``    -- Mach 1.22 planar shock (post-shock state from the
  Rankine-Hugoniot relations) hitting a nested two-material bubble in a 4 x 1
  domain; inflow left, outflow right, symmetric (reflective) top/bottom as in
  Case V of Sec. 3.
* ``batched_tubes``   -- 256 ragged 1D three-material tubes drawn from a
  seeded generator.

The level set is the exact unsigned distance to the interface network,
clamped to the narrow band ``band_ls * dx``.
"""
from __future__ import annotations

import math

import numpy as np

BC_TRANSMISSIVE = 0
BC_REFLECTIVE = 1
BC_INFLOW = 2
BC_OUTFLOW = 3


def base_config(**kw):
    cfg = dict(dim=1, nx=1, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, n_mat=3,
               gamma=[1.4] * 3, pinf=[0.0] * 3,
               bc=[BC_TRANSMISSIVE] * 4, inflow_W=[0.0] * 4, inflow_mat=0,
               cfl=0.6, rk_order=3, alpha_mix=0.5, k_ext=8, band_ls=8)
    cfg.update(kw)
    return cfg


def rankine_hugoniot(mach, gamma, rho0, p0, u0=0.0):
    """Post-shock state behind a right-moving shock of Mach ``mach`` running
    into gas (rho0, u0, p0).  Closed-form normal-shock relations for an ideal
    gas.  Returns (rho1, u1, p1, shock_speed)."""
    g = gamma
    c0 = math.sqrt(g * p0 / rho0)
    m2 = mach * mach
    p1 = p0 * (2.0 * g * m2 - (g - 1.0)) / (g + 1.0)
    rho1 = rho0 * (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    s = u0 + mach * c0
    u1 = s - (s - u0) * rho0 / rho1
    return rho1, u1, p1, s


def _centres(n, a, b):
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx, dx


def _fill_W(n_mat, dim, shape, states):
    nv = dim + 2
    W = np.zeros((n_mat, nv) + shape, dtype=np.float64)
    for m in range(n_mat):
        for k in range(nv):
            W[m, k] = states[m][k]
    return W


def shock_tube_1d(n=400, x_if=(0.3, 0.6), gammas=(1.4, 1.667, 4.4),
                  pinfs=(0.0, 0.0, 6.0), rhos=(1.0, 0.125, 1.0),
                  ps=(1.0, 0.1, 1.0), us=(0.0, 0.0, 0.0), bc=BC_TRANSMISSIVE,
                  steps=200):
    """Three-material stiffened-gas shock tube on [0, 1]."""
    x, dx = _centres(n, 0.0, 1.0)
    cfg = base_config(dim=1, nx=n, ny=1, gamma=list(gammas), pinf=list(pinfs),
                      bc=[bc, bc, bc, bc])
    a, b = x_if
    phi = np.minimum(np.abs(x - a), np.abs(x - b))
    phi = np.minimum(phi, cfg["band_ls"] * dx)
    chi = np.where(x < a, 0, np.where(x < b, 1, 2)).astype(np.int32)
    W = _fill_W(3, 1, (n,), [(rhos[m], us[m], ps[m]) for m in range(3)])
    return dict(cfg=cfg, phi=phi.reshape(1, n), chi=chi.reshape(1, n),
                W=W.reshape(3, 3, 1, n), steps=steps, name="shock_tube_1d")


def _dist_segment(px, py, ax, ay, bx, by):
    vx, vy = bx - ax, by - ay
    L2 = vx * vx + vy * vy
    t = np.clip(((px - ax) * vx + (py - ay) * vy) / L2, 0.0, 1.0)
    qx, qy = ax + t * vx, ay + t * vy
    return np.sqrt((px - qx) ** 2 + (py - qy) ** 2)


def triple_point(nx=896, ny=384, steps=2000, scale_sep=0, reinit=1):
    """Case III: 7 x 3 box, reflective walls, triple point at (1, 1.5);
    the level set redistanced after every step (reinit)."""
    x, dx = _centres(nx, 0.0, 7.0)
    y, dy = _centres(ny, 0.0, 3.0)
    X, Y = np.meshgrid(x, y)
    cfg = base_config(dim=2, nx=nx, ny=ny, x0=0.0, x1=7.0, y0=0.0, y1=3.0,
                      gamma=[1.5, 1.4, 1.5], pinf=[0.0, 0.0, 0.0],
                      bc=[BC_REFLECTIVE] * 4, scale_sep=scale_sep, reinit=reinit)
    # interfaces are axis-aligned: distances are exact differences
    d1 = np.where((Y >= 0.0) & (Y <= 3.0), np.abs(X - 1.0),
                  _dist_segment(X, Y, 1.0, 0.0, 1.0, 3.0))
    d2 = np.where(X >= 1.0, np.abs(Y - 1.5),
                  _dist_segment(X, Y, 1.0, 1.5, 7.0, 1.5))
    phi = np.minimum(np.minimum(d1, d2), cfg["band_ls"] * min(dx, dy))
    chi = np.where(X < 1.0, 0, np.where(Y < 1.5, 1, 2)).astype(np.int32)
    W = _fill_W(3, 2, (ny, nx), [(1.0, 0.0, 0.0, 1.0), (1.0, 0.0, 0.0, 0.1),
                                 (0.125, 0.0, 0.0, 0.1)])
    return dict(cfg=cfg, phi=phi, chi=chi, W=W, steps=steps,
                name="triple_point")


def shock_bubble(nx=2048, ny=512, mach=1.22, rho_outer=0.138, rho_inner=3.15,
                 steps=3000, x_shock=0.5, centre=(1.2, 0.5), r_out=0.25,
                 r_in=0.1, scale_sep=1, reinit=1):
    """Planar Mach ``mach`` shock in ambient gas hitting a nested bubble:
    outer shell (gamma 1.648, rho_outer) and inner core (gamma 1.249,
    rho_inner), both at p = 1, on a 4 x 1 domain; scale separation and the
    redistancing of the level set after every step."""
    x, dx = _centres(nx, 0.0, 4.0)
    y, dy = _centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    g0 = 1.4
    rho1, u1, p1, _ = rankine_hugoniot(mach, g0, 1.0, 1.0)
    cfg = base_config(dim=2, nx=nx, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0,
                      gamma=[g0, 1.648, 1.249], pinf=[0.0, 0.0, 0.0],
                      bc=[BC_INFLOW, BC_OUTFLOW, BC_REFLECTIVE, BC_REFLECTIVE],
                      inflow_W=[rho1, u1, 0.0, p1], inflow_mat=0, scale_sep=scale_sep,
                      reinit=reinit)
    d = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2)
    phi = np.minimum(np.abs(d - r_out), np.abs(d - r_in))
    phi = np.minimum(phi, cfg["band_ls"] * min(dx, dy))
    chi = np.where(d <= r_in, 2, np.where(d <= r_out, 1, 0)).astype(np.int32)
    W = _fill_W(3, 2, (ny, nx), [(1.0, 0.0, 0.0, 1.0),
                                 (rho_outer, 0.0, 0.0, 1.0),
                                 (rho_inner, 0.0, 0.0, 1.0)])
    post = X < x_shock
    W[0, 0][post] = rho1
    W[0, 1][post] = u1
    W[0, 3][post] = p1
    return dict(cfg=cfg, phi=phi, chi=chi, W=W, steps=steps,
                name="shock_bubble")


def rankine_hugoniot_dmach(mach, gamma, rho0, p0):
    """Derivatives with respect to the Mach number of the post-shock state
    of ``rankine_hugoniot`` (gas at rest ahead of the shock): returns
    (drho1, du1, dp1), from differentiating the closed forms."""
    g = gamma
    c0 = math.sqrt(g * p0 / rho0)
    m2 = mach * mach
    den = (g - 1.0) * m2 + 2.0
    rho1 = rho0 * (g + 1.0) * m2 / den
    drho1 = rho0 * (g + 1.0) * 4.0 * mach / (den * den)
    dp1 = p0 * 4.0 * g * mach / (g + 1.0)
    s = mach * c0
    # u1 = s (1 - rho0 / rho1)
    du1 = c0 * (1.0 - rho0 / rho1) + s * rho0 * drho1 / (rho1 * rho1)
    return drho1, du1, dp1


def shock_bubble_tangent(w, q, mach=1.22, x_shock=0.5):
    """Derivative of the primitive fields and inflow state of a
    ``shock_bubble`` workload ``w`` with respect to parameter q of
    (rho_outer, rho_inner, mach): returns (dW, dinflow)."""
    cfg = w["cfg"]
    nx, ny = cfg["nx"], cfg["ny"]
    dW = np.zeros_like(w["W"])
    dinf = np.zeros(4)
    if q == 0:
        dW[1, 0] = 1.0
    elif q == 1:
        dW[2, 0] = 1.0
    else:
        x, _ = _centres(nx, cfg["x0"], cfg["x1"])
        post = np.broadcast_to(x < x_shock, (ny, nx))
        dr, du, dp = rankine_hugoniot_dmach(mach, cfg["gamma"][0], 1.0, 1.0)
        dW[0, 0][post] = dr
        dW[0, 1][post] = du
        dW[0, 3][post] = dp
        dinf[:] = [dr, du, 0.0, dp]
    return dW, dinf


# Water of Case VI (Table 2: rho0 = 1000, gamma = 7.15, p = 1 with the
# ambient air at rho = 1, p = 1).  The paper gives no value of B; B = 3310
# is the usual Tait constant of water (3.31e8 Pa) in units of an ambient
# pressure of 1e5 Pa.
WATER = dict(gamma=7.15, rho0=1000.0, B=3310.0, p0=1.0)


def tait_config(cfg, mats, water=WATER):
    """Mark the materials ``mats`` of a configuration as Tait water."""
    M = cfg["n_mat"]
    cfg["eos"] = [1 if m in mats else 0 for m in range(M)]
    cfg["rho0"] = [water["rho0"] if m in mats else 0.0 for m in range(M)]
    cfg["tait_B"] = [water["B"] if m in mats else 0.0 for m in range(M)]
    cfg["p0"] = [water["p0"] if m in mats else 0.0 for m in range(M)]
    for m in mats:
        cfg["gamma"][m] = water["gamma"]
        cfg["pinf"][m] = 0.0
    return cfg


def tait_pressure(rho, water=WATER):
    """Pressure of Tait water at density rho (for building consistent inputs)."""
    return water["B"] * (np.asarray(rho) / water["rho0"]) ** water["gamma"] - water["B"] + water["p0"]


def air_water_tube_1d(n=400, x_if=None, air=(50.0, 0.0, 1000.0), water_rho=1000.0,
                      steps=100):
    """Two-material tube on [0, 1]: compressed air (gamma 1.4) left of x_if,
    Tait water at rest right of it; transmissive ends.  The interface sits
    inside a cell (0.3 cell past the middle face) by default."""
    x, dx = _centres(n, 0.0, 1.0)
    if x_if is None:
        x_if = 0.5 + 0.3 * dx
    cfg = base_config(dim=1, nx=n, ny=1, n_mat=2, gamma=[1.4, 1.4], pinf=[0.0, 0.0],
                      bc=[BC_TRANSMISSIVE] * 4)
    tait_config(cfg, [1])
    phi = np.minimum(np.abs(x - x_if), cfg["band_ls"] * dx)
    chi = (x >= x_if).astype(np.int32)
    pw = float(tait_pressure(water_rho))
    W = _fill_W(2, 1, (n,), [air, (water_rho, 0.0, pw)])
    return dict(cfg=cfg, phi=phi.reshape(1, n), chi=chi.reshape(1, n),
                W=W.reshape(2, 3, 1, n), steps=steps, name="air_water_tube_1d")


def shock_helium_water(nx=512, ny=128, steps=200, x_shock=0.5, bubble=(1.1, 0.5, 0.25),
                       column=(2.0, 0.5, 0.2), scale_sep=1, reinit=1):
    """Case VI set-up (Table 2): a Mach 6 shock in air (post-shock state from
    the normal-shock relations; Table 2 prints (5.268, 5.752, 41.83)) hits a
    helium bubble (gamma 1.667, rho 0.138) that then meets a water column
    (Tait water, rho0 = 1000).  The figure with the geometry is not in the
    text: bubble of radius 0.25 at (1.1, 0.5), circular water column of
    radius 0.2 at (2.0, 0.5), 4 x 1 domain, inflow left, outflow right,
    reflective top and bottom (as Case V)."""
    x, dx = _centres(nx, 0.0, 4.0)
    y, dy = _centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    rho1, u1, p1, _ = rankine_hugoniot(6.0, 1.4, 1.0, 1.0)
    cfg = base_config(dim=2, nx=nx, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0,
                      gamma=[1.4, 1.667, 1.4], pinf=[0.0, 0.0, 0.0],
                      bc=[BC_INFLOW, BC_OUTFLOW, BC_REFLECTIVE, BC_REFLECTIVE],
                      inflow_W=[rho1, u1, 0.0, p1], inflow_mat=0, scale_sep=scale_sep,
                      reinit=reinit)
    tait_config(cfg, [2])
    db = np.sqrt((X - bubble[0]) ** 2 + (Y - bubble[1]) ** 2) - bubble[2]
    dc = np.sqrt((X - column[0]) ** 2 + (Y - column[1]) ** 2) - column[2]
    phi = np.minimum(np.minimum(np.abs(db), np.abs(dc)), cfg["band_ls"] * min(dx, dy))
    chi = np.where(db <= 0.0, 1, np.where(dc <= 0.0, 2, 0)).astype(np.int32)
    W = _fill_W(3, 2, (ny, nx), [(1.0, 0.0, 0.0, 1.0), (0.138, 0.0, 0.0, 1.0),
                                 (1000.0, 0.0, 0.0, float(tait_pressure(1000.0)))])
    post = X < x_shock
    W[0, 0][post] = rho1
    W[0, 1][post] = u1
    W[0, 3][post] = p1
    return dict(cfg=cfg, phi=phi, chi=chi, W=W, steps=steps, name="shock_helium_water")


BATCH_SEED = 1704005190


def batched_tubes(n_inst=256, seed=BATCH_SEED, nmin=200, nmax=4000, steps=500):
    """Ragged batch of 1D three-material tubes on [0, 1] (ideal gases,
    transmissive ends).  Per instance, in this order: N ~ U{nmin..nmax},
    gamma_{A,B,C} ~ U(1.2, 1.7), rho ~ U(0.1, 3), p ~ U(0.1, 10), the two
    interface positions ~ U(0.2, 0.8) sorted and redrawn while closer than
    8 cells."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        n = int(rng.integers(nmin, nmax + 1))
        g = rng.uniform(1.2, 1.7, 3)
        rho = rng.uniform(0.1, 3.0, 3)
        p = rng.uniform(0.1, 10.0, 3)
        dx = 1.0 / n
        while True:
            a, b = np.sort(rng.uniform(0.2, 0.8, 2))
            if b - a >= 8 * dx:
                break
        inst = shock_tube_1d(n=n, x_if=(float(a), float(b)),
                             gammas=tuple(float(v) for v in g),
                             pinfs=(0.0, 0.0, 0.0),
                             rhos=tuple(float(v) for v in rho),
                             ps=tuple(float(v) for v in p), steps=steps)
        inst["name"] = "batched_tube"
        out.append(inst)
    return out


def uniform_pressure_2d(nx=48, ny=40, shape="circle", p0=1.0, steps=100):
    """Static uniform pressure with three materials of very different
    (gamma, pinf, rho), used to check that a pressure/velocity equilibrium is
    preserved across interfaces."""
    x, dx = _centres(nx, 0.0, 1.2)
    y, dy = _centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    cfg = base_config(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.2, y0=0.0, y1=1.0,
                      gamma=[1.4, 4.4, 1.667], pinf=[0.0, 6.0, 0.0],
                      bc=[BC_REFLECTIVE] * 4)
    if shape == "circle":
        d = np.sqrt((X - 0.55) ** 2 + (Y - 0.45) ** 2)
        phi = np.minimum(np.abs(d - 0.3), np.abs(d - 0.15))
        chi = np.where(d <= 0.15, 2, np.where(d <= 0.3, 1, 0))
    else:  # two slanted parallel lines at 30 degrees
        s = (X * math.cos(math.pi / 6) + Y * math.sin(math.pi / 6))
        phi = np.minimum(np.abs(s - 0.45), np.abs(s - 0.8))
        chi = np.where(s < 0.45, 0, np.where(s < 0.8, 1, 2))
    phi = np.minimum(phi, cfg["band_ls"] * min(dx, dy))
    W = _fill_W(3, 2, (ny, nx), [(1.0, 0.0, 0.0, p0), (5.0, 0.0, 0.0, p0),
                                 (0.1, 0.0, 0.0, p0)])
    return dict(cfg=cfg, phi=phi, chi=chi.astype(np.int32), W=W, steps=steps,
                name="uniform_pressure_" + shape)


# Case II's free-surface pressure law: 13 up to t = 0.04, then linear to 0.5
# at t = 0.125, then 0.5; the ambient (not solved) has density 0.1
ICF_PRESSURE = (13.0, 0.5, 0.04, 0.125, 0.1)


def icf_1d(n=320, r_in=1.0, r_out=1.2, gammas=(1.667, 1.667, 1.667), steps=None, t_end=0.3):
    """Case II: 1D cylindrical implosion on r in [0, 1.5] (Table 1): light
    core (rho 0.05, p 0.1) for r < r_in, dense shell (rho 1, p 0.1) up to
    r_out, ambient (rho 0.1, p 13) outside, all at rest; the ambient is not
    solved and the shell's outer interface is a free surface under the
    pressure law of ICF_PRESSURE.  Reflective axis."""
    x, dx = _centres(n, 0.0, 1.5)
    cfg = base_config(dim=1, nx=n, ny=1, x0=0.0, x1=1.5, gamma=list(gammas),
                      pinf=[0.0, 0.0, 0.0], bc=[BC_REFLECTIVE, BC_TRANSMISSIVE] * 2,
                      coord=1, fs_on=1, fs_mat=2, fs_p=list(ICF_PRESSURE))
    chi = np.where(x < r_in, 0, np.where(x < r_out, 1, 2)).astype(np.int32)
    phi = np.minimum(np.abs(x - r_in), np.abs(x - r_out))
    phi = np.minimum(phi, cfg["band_ls"] * dx)
    W = _fill_W(3, 1, (1, n), [(0.05, 0.0, 0.1), (1.0, 0.0, 0.1), (0.1, 0.0, 13.0)])
    return dict(cfg=cfg, phi=phi[None], chi=chi[None], W=W, steps=steps, t_end=t_end,
                name="icf_1d")


def workload(name, **kw):
    """Named workloads with their full sizes and step counts."""
    if name == "shock_tube_1d":
        return shock_tube_1d(**kw)
    if name == "triple_point":
        return triple_point(**kw)
    if name == "shock_bubble":
        return shock_bubble(**kw)
    raise KeyError(name)
