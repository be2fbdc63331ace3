"""Pins of the oracle's tangent build (forward-mode derivative of the
discrete step, dt held fixed): against central finite differences of the
plain oracle, and against its own linearity.  The tangent build evaluates
the very same source with a value+derivative scalar; these checks would fail
on a wrong derivative rule or a derivative dropped on the way (e.g. through
the geometry, the level set or the mixing)."""
import numpy as np
import pytest

import oracle
import workloads as wl


def run_plain(w, steps, dt, W=None, inflow=None, state=None):
    cfg = dict(w["cfg"])
    if inflow is not None:
        cfg["inflow_W"] = list(inflow)
    o = oracle.Oracle(cfg)
    assert o.init(w["phi"], w["chi"], w["W"] if W is None else W) == 0
    o.set_dt(dt)
    return o


def fd_rel_err(tan, plus, minus, h):
    fd = (plus - minus) / (2.0 * h)
    den = np.linalg.norm(fd.ravel())
    assert den > 0.0
    return np.linalg.norm((tan - fd).ravel()) / den


@pytest.mark.parametrize("case", ["tube", "tube_face_aligned"])
def test_tangent_of_initial_densities_1d(case):
    if case == "tube":
        w = wl.shock_tube_1d(n=120)
    else:
        w = wl.shock_tube_1d(n=160, x_if=(0.3, 0.6))
    dt, steps = 4e-4, 25
    # direction: the density of material B inside its own region, scaled
    dW = np.zeros_like(w["W"])
    dW[1, 0] = w["W"][1, 0] * (w["chi"][None] == 1)[0]
    t = oracle.Oracle(w["cfg"], tangent=True)
    assert t.init_tangent(w["phi"], w["chi"], w["W"], dW) == 0
    t.set_dt(dt)
    assert t.step(steps) == 0
    tan = t.get_tangent()
    h = 1e-6
    res = []
    for sgn in (1, -1):
        o = run_plain(w, steps, dt, W=w["W"] + sgn * h * dW)
        assert o.step(steps) == 0
        res.append(o.get())
    assert fd_rel_err(tan["Q"], res[0]["Q"], res[1]["Q"], h) < 1e-6
    # the interfaces move with the densities: the level set carries a
    # derivative, and so do the volume fractions
    assert np.abs(tan["phi"]).max() > 0.0
    assert fd_rel_err(tan["phi"], res[0]["phi"], res[1]["phi"], h) < 1e-6
    assert fd_rel_err(tan["alpha"], res[0]["alpha"], res[1]["alpha"], h) < 1e-6


def drifting_bubble(nx=128, ny=32):
    """The nested shock-bubble set-up with a uniform drift (0.3, 0.1) added
    to every material and transmissive sides: no velocity is exactly zero,
    so the upwind choices of the level set are not at their switch point
    (where the step has a kink and central differences average two one-sided
    slopes)."""
    w = wl.shock_bubble(nx=nx, ny=ny)
    w["W"] = w["W"].copy()
    w["W"][:, 1] += 0.3
    w["W"][:, 2] += 0.1
    w["cfg"]["bc"] = [wl.BC_TRANSMISSIVE] * 4
    return w


def test_tangent_of_a_state_perturbation_2d():
    # random perturbation of (Q, phi) of a developed 2D three-material state.
    # (Interfaces lying exactly on cell faces, as in the triple-point set-up,
    # are kinks of the volume fraction and unsuitable for this check.)
    w, dt, n0 = drifting_bubble(), 2e-3, 40
    rng = np.random.default_rng(7)
    base = oracle.Oracle(w["cfg"])
    assert base.init(w["phi"], w["chi"], w["W"]) == 0
    base.set_dt(dt)
    assert base.step(n0) == 0
    g = base.get()
    h_cell = (w["cfg"]["x1"] - w["cfg"]["x0"]) / w["cfg"]["nx"]
    dQ = rng.standard_normal(g["Q"].shape) * np.abs(g["Q"]) * 1e-2
    dphi = rng.standard_normal(g["phi"].shape) * 1e-2 * h_cell * (g["phi"] < 6 * h_cell)
    t = oracle.Oracle(w["cfg"], tangent=True)
    assert t.init(w["phi"], w["chi"], w["W"]) == 0
    t.set_dt(dt)
    assert t.set_state(g["Q"], g["phi"], g["chi"]) == 0
    t.seed_state(dQ, dphi)
    assert t.step(2) == 0
    tan = t.get_tangent()
    h = 1e-6
    res = []
    for sgn in (1.0, -1.0):
        o = oracle.Oracle(w["cfg"])
        assert o.init(w["phi"], w["chi"], w["W"]) == 0
        o.set_dt(dt)
        assert o.set_state(g["Q"] + sgn * h * dQ, g["phi"] + sgn * h * dphi, g["chi"]) == 0
        assert o.step(2) == 0
        res.append(o.get())
    # the shifted runs keep the branch pattern of the base run
    assert np.array_equal(res[0]["chi"], res[1]["chi"])
    assert fd_rel_err(tan["Q"], res[0]["Q"], res[1]["Q"], h) < 1e-5
    assert fd_rel_err(tan["phi"], res[0]["phi"], res[1]["phi"], h) < 1e-5


def test_tangent_is_linear_in_the_seed():
    w = wl.shock_tube_1d(n=80)
    dW = np.zeros_like(w["W"])
    dW[0, 2] = 1.0
    out = []
    for scale in (1.0, 3.0):
        t = oracle.Oracle(w["cfg"], tangent=True)
        assert t.init_tangent(w["phi"], w["chi"], w["W"], scale * dW) == 0
        t.set_dt(5e-4)
        assert t.step(10) == 0
        out.append(t.get_tangent()["Q"])
    np.testing.assert_allclose(out[1], 3.0 * out[0], rtol=1e-12, atol=1e-15)


def test_tangent_of_the_inflow_state():
    # the shock-bubble inflow state enters every step through the frame
    w = wl.shock_bubble(nx=96, ny=24)
    dt, steps = 2e-3, 12
    d = np.array([1.0, 0.5, 0.0, 2.0])
    t = oracle.Oracle(w["cfg"], tangent=True)
    assert t.init(w["phi"], w["chi"], w["W"]) == 0
    t.set_dt(dt)
    t.set_inflow_tangent(d)
    assert t.step(steps) == 0
    tan = t.get_tangent()
    h = 1e-6
    res = []
    for sgn in (1, -1):
        o = run_plain(w, steps, dt, inflow=np.array(w["cfg"]["inflow_W"]) + sgn * h * d)
        assert o.step(steps) == 0
        res.append(o.get())
    assert np.abs(tan["Q"]).max() > 0.0
    assert fd_rel_err(tan["Q"], res[0]["Q"], res[1]["Q"], h) < 1e-6
