"""GPU adjoint (mm_adjoint_step) against the oracle's tangent build.

Both sides differentiate the same discrete step about the same trajectory
(the forward states are bit-identical), with the step size held fixed and
the branch pattern of the forward run.  Checks:

* dot products <lambda, J delta> (oracle tangent of delta) against
  <J^T lambda, delta> (library adjoint of lambda) for random delta in (Q,
  phi) and random lambda in (Q, phi, alpha) over one and several steps;
* the gradient of the nested-bubble centroid with respect to (shell
  density, core density, shock Mach number) against three tangent runs, and
  against central differences of the library with the recorded step sizes.

Exact ties of the branch tests at the base point (interfaces lying on
cell faces, as in the triple-point set-up) are resolved alike on both sides:
the first step of the triple point agrees at the same 1e-10.  Later steps of
the triple point carry sliver volume fractions (1e-12 down to 1e-34) that
the roundoff of the level set leaves along its face-aligned interface; the
linearisation there is ill-conditioned, and the oracle's own tangent is not
linear to better than about 1e-3 (its rounding).  Those steps are checked
against that floor: the tangent-adjoint difference stays within a small
multiple of the tangent's own linearity defect.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

DOT_REL = 1e-10


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


def single2d(nx=40, ny=24):
    rng = np.random.default_rng(3)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / nx
    X, Y = np.meshgrid(x, y)
    r = 1.0 + 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.25) ** 2) / 0.02)
    p = 1.0 + 0.5 * np.exp(-((X - 0.6) ** 2 + (Y - 0.3) ** 2) / 0.01) + 0.01 * rng.random((ny, nx))
    cfg = wl.base_config(dim=2, nx=nx, ny=ny, x1=1.0, y1=ny / nx, n_mat=1, gamma=[1.4],
                         pinf=[0.0], bc=[wl.BC_REFLECTIVE, wl.BC_TRANSMISSIVE,
                                         wl.BC_REFLECTIVE, wl.BC_OUTFLOW])
    return dict(cfg=cfg, phi=np.full((ny, nx), 1.0), chi=np.zeros((ny, nx), np.int32),
                W=np.array([r, 0.1 * np.sin(6 * Y), 0.05 * np.cos(3 * X), p])[None])


def drifting_bubble(nx=96, ny=32):
    w = wl.shock_bubble(nx=nx, ny=ny, reinit=0)
    w["W"] = w["W"].copy()
    w["W"][:, 1] += 0.3
    w["W"][:, 2] += 0.1
    w["cfg"]["bc"] = [wl.BC_TRANSMISSIVE] * 4
    return w


CASES = {
    "single2d": (single2d, 3, 1),
    "tube_1step": (lambda: wl.shock_tube_1d(n=120), 20, 1),
    "tube_4steps": (lambda: wl.shock_tube_1d(n=120), 20, 4),
    "drifting_bubble": (drifting_bubble, 15, 1),
    "bubble_at_rest_2steps": (lambda: wl.shock_bubble(nx=128, ny=32, reinit=0), 20, 2),
    "bubble_hit_3steps": (lambda: wl.shock_bubble(nx=128, ny=32, reinit=0), 60, 3),
    # face-aligned interfaces and the triple junction, before any sliver
    "triple_point_first_step": (lambda: wl.triple_point(nx=112, ny=48, reinit=0), 0, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_dot_product_against_tangent(pk, name):
    make, n0, nsteps = CASES[name]
    w = make()
    o = oracle.Oracle(w["cfg"], tangent=True)
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    assert o.step(n0) == 0
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    s.step(n0)
    g0 = o.get()
    h0 = s.get()
    for k in ("Q", "alpha", "phi", "chi"):
        assert np.array_equal(g0[k], h0[k]), k
    rng = np.random.default_rng(11)
    dQ = rng.standard_normal(g0["Q"].shape) * np.abs(g0["Q"])
    hc = (w["cfg"]["x1"] - w["cfg"]["x0"]) / w["cfg"]["nx"]
    dphi = rng.standard_normal(g0["phi"].shape) * hc * (g0["phi"] < 7 * hc)
    o.seed_state(dQ, dphi)
    assert o.step(nsteps) == 0
    tan = o.get_tangent()
    s.step(nsteps, record=2)
    g1 = o.get()
    lQ = rng.standard_normal(g1["Q"].shape)
    lphi = rng.standard_normal(g1["phi"].shape)
    la = rng.standard_normal(g1["alpha"].shape)
    lhs = np.sum(lQ * tan["Q"]) + np.sum(lphi * tan["phi"]) + np.sum(la * tan["alpha"])
    if nsteps == 1:
        aQ, aphi = s.adjoint_step(lQ, lphi, la)
    else:
        s.adjoint_step(lQ, lphi, la, out=False)
        for _ in range(nsteps - 2):
            s.adjoint_step(out=False)
        aQ, aphi = s.adjoint_step()
    rhs = np.sum(aQ * dQ) + np.sum(aphi * dphi)
    rel = abs(lhs - rhs) / max(abs(lhs), 1e-300)
    print(name, lhs, rhs, rel)
    assert rel <= DOT_REL
    # the reverse steps leave the forward state of the recorded run in place
    h1 = s.get()
    for k in ("Q", "alpha", "phi", "chi"):
        assert np.array_equal(g1[k], h1[k]), k


def tangent_q(w, n0, dq, dp):
    o = oracle.Oracle(w["cfg"], tangent=True)
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    assert o.step(n0) == 0
    o.seed_state(dq, dp)
    assert o.step(1) == 0
    return o.get_tangent()["Q"]


@pytest.mark.parametrize("n0", [3, 20])
def test_dot_product_triple_point_rounding_floor(pk, n0):
    """Triple point after n0 steps, one step, Q outputs against phi and Q
    seeds.  The floor is the tangent's own linearity defect
    |<l, T(a + b)> - <l, T(a)> - <l, T(b)>| for a random split of the seed,
    which in exact arithmetic is zero."""
    w = wl.triple_point(nx=112, ny=48, reinit=0)
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    assert o.step(n0) == 0
    g0 = o.get()
    # the sliver fractions this test is about
    al = g0["alpha"]
    assert np.any((al > 0.0) & (al < 1e-10))
    rng = np.random.default_rng(5)
    hc = 7.0 / 112
    dQ = rng.standard_normal(g0["Q"].shape) * np.abs(g0["Q"])
    dphi = rng.standard_normal(g0["phi"].shape) * hc * (g0["phi"] < 7 * hc)
    lQ = rng.standard_normal(g0["Q"].shape)
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    s.step(n0)
    s.step(1, record=1)
    z = np.zeros(g0["phi"].shape)
    aQ, aphi = s.adjoint_step(lQ, z, np.zeros((3,) + z.shape))
    s.close()
    for dq, dp in ((0 * dQ, dphi), (dQ, 0 * dphi)):
        t = tangent_q(w, n0, dq, dp)
        mq = rng.random(dq.shape) < 0.5
        mp = rng.random(dp.shape) < 0.5
        t1 = tangent_q(w, n0, dq * mq, dp * mp)
        t2 = tangent_q(w, n0, dq * ~mq, dp * ~mp)
        lhs = np.sum(lQ * t)
        defect = abs(lhs - (np.sum(lQ * t1) + np.sum(lQ * t2)))
        rhs = np.sum(aQ * dq) + np.sum(aphi * dp)
        print("n0", n0, "lhs", lhs, "rhs", rhs, "diff", abs(lhs - rhs), "tangent defect", defect)
        assert abs(lhs - rhs) <= 10.0 * defect + DOT_REL * abs(lhs)


def test_tape_state_errors(pk):
    w = wl.shock_tube_1d(n=80)
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    with pytest.raises(pk.MMError) as e:
        s.adjoint_step(np.zeros((3, 3, 1, 80)), np.zeros((1, 80)))
    assert e.value.status == 5
    s.step(2, record=1)
    n, rem, dt = s.tape()
    assert (n, rem) == (2, 2) and np.all(dt > 0)
    s.adjoint_step(out=False)
    s.adjoint_step(out=False)
    with pytest.raises(pk.MMError) as e:
        s.adjoint_step()
    assert e.value.status == 5
    # a plain step ends the tape
    s.step(1, record=1)
    s.step(1)
    assert s.tape()[0] == 0


def tangent_gradient(prob, params, steps):
    from paper_1704_00519_amd import adjoint as ad
    w = prob.w
    W, inflow = prob.fields(torch.tensor(params))
    cfg = dict(w["cfg"])
    cfg["inflow_W"] = [float(v) for v in inflow]
    g = np.zeros(3)
    for q in range(3):
        e = torch.zeros(3, dtype=torch.float64)
        e[q] = 1.0
        _, (dW, dinf) = torch.autograd.functional.jvp(prob.fields, (torch.tensor(params),), (e,))
        o = oracle.Oracle(cfg, tangent=True)
        assert o.init_tangent(w["phi"], w["chi"], W.numpy(), dW.numpy()) == 0
        o.set_inflow_tangent(dinf.numpy())
        assert o.step(steps) == 0
        _, gJ = ad.centroid(o.get()["alpha"], prob.x)
        g[q] = np.sum(gJ * o.get_tangent()["alpha"])
    return g


def branch_signature(s):
    """Counters and indicator field of a run: a change between the runs of
    a central difference means a branch of the step switched."""
    d = s.diag()
    return (d["n_mixsrc"], d["n_stranded"], d["n_posfix"], d["n_ifskip"], d["n_updates"],
            s.get()["chi"].tobytes())


def central_differences(prob, params, steps, K, dts, g):
    """Central differences of CentroidGradient.apply itself (same fixed
    schedule), h = 1e-6 |p_q|; a parameter whose +-h runs take another
    branch pattern than the nominal run is reported and not compared."""
    from paper_1704_00519_amd import adjoint as ad
    base = branch_signature(prob.run(params, steps, dts=dts)[1])
    fds = []
    for q in range(3):
        h = 1e-6 * abs(params[q])
        Js, same = [], True
        for sgn in (1.0, -1.0):
            pq = torch.tensor(params + sgn * h * np.eye(3)[q])
            Js.append(float(ad.CentroidGradient.apply(pq, prob, steps, K, dts)))
            same &= branch_signature(prob.run(params + sgn * h * np.eye(3)[q], steps,
                                              dts=dts)[1]) == base
        fd = (Js[0] - Js[1]) / (2 * h)
        print("param", q, "fd", fd, "adjoint", g[q], "same branches", same)
        fds.append((fd, same))
    return fds


def test_centroid_gradient_against_tangent_and_differences(pk):
    from paper_1704_00519_amd import adjoint as ad
    prob = ad.NestedBubble(wl.shock_bubble(nx=128, ny=32, reinit=0))
    params = np.array([0.138, 3.15, 1.22])
    steps, K = 70, 16  # past the first contact of the shock with the shell
    dts = ad.nominal_schedule(prob, params, steps)
    p = torch.tensor(params, requires_grad=True)
    J = ad.CentroidGradient.apply(p, prob, steps, K, dts)
    J.backward()
    g = p.grad.numpy()
    gt = tangent_gradient(prob, params, steps)
    print("adjoint", g, "tangent", gt)
    assert np.all(np.abs(g - gt) <= 1e-8 * np.abs(gt).max())
    for q, (fd, same) in enumerate(central_differences(prob, params, steps, K, dts, g)):
        if same:
            assert abs(fd - g[q]) <= 1e-4 * max(abs(g[q]), 1e-3 * np.abs(g).max())


def test_gradient_study_size_against_stored_tangent(pk):
    """The gradient study at its own size (512 x 128, 300 steps, checkpoint
    every 30): step sizes, J and update count against the oracle's nominal
    run, the gradient against the oracle's tangent build (stored by
    tests/golden/make_gradient_512.py, 1e-8), and against central
    differences of the function itself (1e-4)."""
    import os
    from paper_1704_00519_amd import adjoint as ad
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden",
                                "gradient_nested_bubble_512.npz"))
    params = gold["params"]
    steps, K = int(gold["steps"]), 30
    prob = ad.NestedBubble(wl.shock_bubble(nx=512, ny=128, reinit=0))
    _, s, _ = prob.run(params, steps, record=1)
    assert np.array_equal(s.tape()[2], gold["dts"])
    assert s.diag()["n_updates"] == int(gold["n_updates"])
    s.close()
    dts = gold["dts"]
    p = torch.tensor(params, requires_grad=True)
    J = ad.CentroidGradient.apply(p, prob, steps, K, dts)
    J.backward()
    g = p.grad.numpy()
    Jv = float(J.detach())
    print("J", Jv, gold["J"], "adjoint", g, "tangent", gold["grad"])
    assert abs(Jv - float(gold["J"])) <= 1e-14 * abs(float(gold["J"]))
    assert np.all(np.abs(g - gold["grad"]) <= 1e-8 * np.abs(gold["grad"]).max())
    for q, (fd, same) in enumerate(central_differences(prob, params, steps, K, dts, g)):
        if same:
            assert abs(fd - g[q]) <= 1e-4 * max(abs(g[q]), 1e-3 * np.abs(g).max())


@pytest.mark.skip(reason="capturing the reverse calls as graphs (executable graph updated "
                  "in place between calls) faulted the GPU twice, also with every update "
                  "waiting for the graph's previous launch; that path is switched off and "
                  "reverse calls launch their kernels directly")
def test_reverse_graph_matches_direct(pk):
    """Reverse calls without inputs or outputs on a stream are captured as
    graphs (the executable graph updated in place from call to call, and
    rebuilt where a segment of another length is recomputed); the gradient
    equals that of direct launches on the null stream up to the order of the
    atomic sums."""
    from paper_1704_00519_amd import adjoint as ad
    prob = ad.NestedBubble(wl.shock_bubble(nx=128, ny=32, reinit=0))
    params = np.array([0.138, 3.15, 1.22])
    steps, K = 40, 16  # segments of 16, 16 and 8 steps
    grads = []
    for stream in (None, torch.cuda.Stream()):
        kw = {} if stream is None else {"stream": stream.cuda_stream}
        s = prob.solver(params, **kw)
        alpha0 = s.get()["alpha"]
        s.step(steps, record=K)
        grads.append(ad.reverse_gradient(prob, s, alpha0, steps, params))
        torch.cuda.synchronize()
    g0, g1 = grads
    print("direct", g0, "graph", g1)
    assert np.all(np.isfinite(g1))
    assert np.all(np.abs(g1 - g0) <= 1e-10 * np.abs(g0).max())


def test_forward_after_reverse_steps(pk):
    """Reverse calls leave the forward run as it was: steps taken after some
    reverse calls give, bit for bit, what the same steps give without them
    (the forward tile list is rebuilt on the next step)."""
    w = wl.shock_bubble(nx=128, ny=32, reinit=0)
    out = []
    for reverse in (False, True):
        s = pk.Solver(w["cfg"])
        s.init(w["phi"], w["chi"], w["W"])
        s.step(12, record=5)
        if reverse:
            g = s.get()
            s.adjoint_step(np.ones_like(g["Q"]), np.zeros_like(g["phi"]), out=False)
            s.adjoint_step(out=False)
            s.adjoint_step(out=False)
            assert s.diag()["n_tiles"] > 0
        s.step(3)
        out.append(s.get())
    for k in ("Q", "alpha", "phi", "chi"):
        assert np.array_equal(out[0][k], out[1][k]), k
