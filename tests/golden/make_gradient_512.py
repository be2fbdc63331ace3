"""Write the oracle's tangent gradient of the nested-bubble centroid at the
size of the gradient study (512 x 128, 300 steps).

Runs the CPU oracle only (no GPU code): the plain build records the step
sizes of the nominal run (CFL, parameters rho_shell = 0.138, rho_core =
3.15, Mach 1.22); the tangent build is then seeded, once per parameter, with
the derivative of the initial primitive fields and of the inflow state (from
``workloads.shock_bubble_tangent``) and replays those step sizes.  Stored:
the step sizes, J (the x-coordinate of the volume centroid of shell + core
after the last step) and dJ/d(rho_shell, rho_core, mach).

Usage: python tests/golden/make_gradient_512.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

NX, NY, STEPS = 512, 128, 300
PARAMS = (0.138, 3.15, 1.22)


def centroid(alpha, x):
    a = alpha[1] + alpha[2]
    S = a.sum()
    J = float((a * x).sum() / S)
    return J, (x - J) / S


def main():
    w = wl.shock_bubble(nx=NX, ny=NY, rho_outer=PARAMS[0], rho_inner=PARAMS[1],
                        mach=PARAMS[2], reinit=0)  # the adjoint is built without it
    cfg = w["cfg"]
    dx = (cfg["x1"] - cfg["x0"]) / NX
    x = np.broadcast_to(cfg["x0"] + (np.arange(NX) + 0.5) * dx, (NY, NX))
    t0 = time.time()
    o = oracle.Oracle(cfg)
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    dts = np.zeros(STEPS)
    for n in range(STEPS):
        assert o.step(1) == 0
        dts[n] = o.diag()["dt"]
    J, gJ = centroid(o.get()["alpha"], x)
    n_upd = o.diag()["n_updates"]
    print(f"nominal run: J = {J!r}, t = {o.diag()['t']}, {time.time() - t0:.0f}s", flush=True)
    grad = np.zeros(3)
    for q in range(3):
        dW, dinf = wl.shock_bubble_tangent(w, q, mach=PARAMS[2])
        ot = oracle.Oracle(cfg, tangent=True)
        assert ot.init_tangent(w["phi"], w["chi"], w["W"], dW) == 0
        ot.set_inflow_tangent(dinf)
        for n in range(STEPS):
            ot.set_dt(float(dts[n]))
            assert ot.step(1) == 0
        Jt, _ = centroid(ot.get()["alpha"], x)
        assert Jt == J, (Jt, J)
        grad[q] = float(np.sum(gJ * ot.get_tangent()["alpha"][1:].sum(axis=0)))
        print(f"parameter {q}: dJ = {grad[q]!r}, {time.time() - t0:.0f}s", flush=True)
    path = os.path.join(HERE, "gradient_nested_bubble_512.npz")
    np.savez_compressed(path, params=np.array(PARAMS), steps=STEPS, dts=dts, J=J, grad=grad,
                        n_updates=n_upd)
    print(f"wrote {path}: J = {J}, grad = {grad}", flush=True)


if __name__ == "__main__":
    main()
