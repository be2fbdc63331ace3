"""GPU parity of Case II of Sec. 3 (the 1D cylindrical implosion driven by a
pressure on the shell's outer surface) with the oracle: radial geometry
(face areas, cell volumes, the geometric source of the radial momentum, the
interface area of a cut cell, content-weighted mixing), the ambient that is
not solved and its free surface under p(t), the step size that counts the
surface's wave, and the r-weighted book-keeping; on the library path at the
resolutions the paper runs (160 to 1280 cells, to t = 0.3), on smaller
pieces of the physics, and on the batched path over the paper's parameter
study (shell thickness and gamma_2 / gamma_1).

The bar is that of the other parity tests (1e-9 relative L1 per conserved
field, the indicator field exactly, the time to 1e-12): the rarefaction
branch of the surface's wave takes a power, whose last bit the device's pow
gives otherwise than the host's for some arguments.  At 1280 cells the two
sides agree bit for bit up to step 178 (t = 0.021); in step 179 the step
size differs by one ulp, and an analysis of that state on the host shows
why: the largest wave speed is the surface's in the rarefaction branch, and
the quotient CFL h / s_max lies 0.24 ulp from the host's (correctly rounded)
result, so the final division is not the cause, the power is.  Over the 5350
steps to t = 0.3 the differences grow to 4e-10 in Q and 5e-11 in the volume
fractions (the flow converges on the axis), so the long runs hold the volume
fractions and distances to 1e-9 rather than 1e-12.  Also: a free
surface or cylindrical geometry in 2D, a free surface with the Roe flux, and
tape recording (the adjoint) are rejected."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_parity import assert_parity, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


def centres(n, L):
    dx = L / n
    return (np.arange(n) + 0.5) * dx, dx


def rest(fs_on):
    n = 120
    r, dx = centres(n, 1.5)
    cfg = wl.base_config(dim=1, nx=n, ny=1, x0=0.0, x1=1.5, gamma=[1.4, 1.667, 4.4],
                         pinf=[0.0, 0.0, 6.0], bc=[wl.BC_REFLECTIVE] * 4, coord=1,
                         fs_on=fs_on, fs_mat=2, fs_p=[1.0, 1.0, 0.0, 1.0, 0.1])
    chi = np.where(r < 0.7, 0, np.where(r < 1.13, 1, 2)).astype(np.int32)
    phi = np.minimum(np.minimum(np.abs(r - 0.7), np.abs(r - 1.13)), 8 * dx)
    W = np.zeros((3, 3, 1, n))
    W[:, 0] = np.array([0.2, 1.0, 3.0])[:, None, None]
    W[:, 2] = 1.0
    return dict(cfg=cfg, phi=phi[None], chi=chi[None], W=W)


def blast():
    n = 200
    r, dx = centres(n, 1.0)
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=1, x0=0.0, x1=1.0, gamma=[1.4], pinf=[0.0],
                         bc=[wl.BC_REFLECTIVE, wl.BC_TRANSMISSIVE] * 2, coord=1)
    W = np.stack([np.where(r < 0.3, 1.0, 0.125), 0 * r, np.where(r < 0.3, 1.0, 0.1)])[None, :, None, :]
    return dict(cfg=cfg, phi=np.full((1, n), 8 * dx), chi=np.zeros((1, n), np.int32), W=W)


def planar_fs():
    n = 400
    x, dx = centres(n, 1.0)
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=2, x0=0.0, x1=1.0, gamma=[1.4, 1.4],
                         pinf=[0.0, 0.0], bc=[wl.BC_REFLECTIVE, wl.BC_TRANSMISSIVE] * 2,
                         fs_on=1, fs_mat=1, fs_p=[13.0, 13.0, 0.0, 1.0, 0.1])
    xs0 = 0.6 + 0.3 * dx
    chi = (x >= xs0).astype(np.int32)
    phi = np.minimum(np.abs(x - xs0), 8 * dx)
    W = np.zeros((2, 3, 1, n))
    W[0, 0], W[0, 2] = 1.0, 0.1
    W[1, 0], W[1, 2] = 0.1, 13.0
    return dict(cfg=cfg, phi=phi[None], chi=chi[None], W=W)


def cylinder_two_gases():
    """Two solved gases in radial geometry (no free surface): a dense ring at
    high pressure inside a light gas, reflective axis, open outer end."""
    n = 240
    r, dx = centres(n, 1.2)
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=2, x0=0.0, x1=1.2, gamma=[1.4, 1.667],
                         pinf=[0.0, 0.0], bc=[wl.BC_REFLECTIVE, wl.BC_TRANSMISSIVE] * 2, coord=1)
    ring = (r > 0.3 + 0.37 * dx) & (r < 0.55 + 0.61 * dx)
    chi = ring.astype(np.int32)
    phi = np.minimum(np.minimum(np.abs(r - 0.3 - 0.37 * dx), np.abs(r - 0.55 - 0.61 * dx)), 8 * dx)
    W = np.zeros((2, 3, 1, n))
    W[0, 0], W[0, 2] = 0.125, 0.1
    W[1, 0], W[1, 2] = 1.0, 2.0
    return dict(cfg=cfg, phi=phi[None], chi=chi[None], W=W)


CASES = {
    "rest_fs": (lambda: rest(1), 60),
    "rest_all_solved": (lambda: rest(0), 60),
    "blast": (blast, 150),
    "planar_fs": (planar_fs, 250),
    "cylinder_two_gases": (cylinder_two_gases, 200),
    "icf_160": (lambda: wl.icf_1d(n=160), 200),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_icf_pieces_match_oracle(pk, name):
    make, steps = CASES[name]
    print("icf case", name, steps, flush=True)
    o, s = run_both(pk, make(), steps)
    info = assert_parity(o, s, label=name)
    do, dg = o.diag(), s.diag()
    assert dg["n_updates"] == do["n_updates"], (name, dg["n_updates"], do["n_updates"])
    print(name, info, "t", dg["t"], flush=True)


def run_to(o, s, t_end):
    """Step both in lockstep to t_end (the oracle decides when to stop)."""
    n = 0
    while o.diag()["t"] < t_end:
        assert o.step(1) == 0
        s.step(1)
        n += 1
    return n


def radii(alpha, dx):
    rin = alpha[0].sum() * dx
    return rin, rin + alpha[1].sum() * dx


@pytest.mark.parametrize("n,dr,ratio", [(160, 0.2, 1.0), (320, 0.2, 1.0), (640, 0.2, 1.0),
                                         (1280, 0.2, 1.0), (320, 0.1, 1.0), (640, 0.05, 2.8)])
def test_case_ii_resolutions_to_t03(pk, n, dr, ratio):
    """The paper's resolutions, to t = 0.3 (past stagnation), in one run of
    each side; the interface radii (volumes of core and shell) agree too.
    The last two are thin shells of the parameter study that reach t = 0.3
    only with new-cell filling of own-material parts without mass."""
    w = wl.icf_1d(n=n, r_out=1.0 + dr, gammas=(1.667, 1.667 * ratio, 1.667))
    print("icf resolution", n, dr, ratio, flush=True)
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    k = 0
    while o.diag()["t"] < 0.3:
        assert o.step(1) == 0
        k += 1
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    s.step(k)
    g, h = o.get(), s.get()
    assert np.array_equal(g["chi"], h["chi"])
    for m in range(3):
        for v in range(3):
            ref = math.fsum(np.abs(g["Q"][m, v]).ravel())
            err = math.fsum(np.abs(h["Q"][m, v] - g["Q"][m, v]).ravel())
            assert err <= 1e-9 * ref, (n, m, v, err / ref)
    da = float(np.abs(g["alpha"] - h["alpha"]).max())
    dp = float(np.abs(g["phi"] - h["phi"]).max())
    assert da <= 1e-9 and dp <= 1e-9, (da, dp)
    assert s.diag()["t"] == pytest.approx(o.diag()["t"], rel=1e-12)
    dx = 1.5 / n
    ro = radii(g["alpha"][:, 0], dx)
    rg = radii(h["alpha"][:, 0], dx)
    assert np.allclose(ro, rg, rtol=0, atol=1e-9), (ro, rg)
    print(n, k, "steps; bitwise", bool(np.array_equal(g["Q"], h["Q"])), "max |dQ|",
          float(np.abs(g["Q"] - h["Q"]).max()), "max |dalpha|", da, "radii", rg, flush=True)


def rsums(Q, x0, dx):
    """r-weighted sums of Q per material and component (rho, rho u, 0,
    rho E), exactly rounded, and of |r Q|."""
    M, nv, _, n = Q.shape
    r = x0 + (np.arange(n) + 0.5) * dx
    s, a = np.zeros((M, 4)), np.zeros((M, 4))
    for m in range(M):
        for c, v in enumerate((0, 1, 3)):
            s[m, v] = math.fsum(Q[m, c, 0] * r)
            a[m, v] = math.fsum(np.abs(Q[m, c, 0] * r))
    return s, a


def test_case_ii_bookkeeping(pk):
    """r-weighted sums of Q, boundary and exchange totals (with the geometric
    source) against the oracle's, and the balance of every solved material
    closed; the ambient books nothing."""
    w = wl.icf_1d(n=320)
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    dg0 = s.diag()
    assert o.step(400) == 0
    s.step(400)
    dg, do = s.diag(), o.diag()
    dx = 1.5 / 320
    ref, absref = rsums(o.get()["Q"], 0.0, dx)
    assert np.all(np.abs(dg["sum_Q"][:3] - ref) <= 1e-13 * np.maximum(absref, 1e-300))
    scale = np.maximum(absref.max(axis=1, keepdims=True), 1e-300)
    assert np.all(np.abs(dg["bnd_in"][:3] - do["bnd"]) <= 1e-13 * scale)
    assert np.all(np.abs(dg["exch"][:3] - do["xsum"]) <= 1e-13 * scale)
    bal = (dg["sum_Q"] - dg0["sum_Q"] - dg["bnd_in"] - dg["exch"])[:2] - do["xfer"][:2]
    assert np.all(np.abs(bal) <= 1e-13 * scale[:2]), bal
    assert np.all(dg["bnd_in"][2] == 0.0) and np.all(dg["exch"][2] == 0.0)
    # core and shell masses: constant (nothing crosses the axis or the surface)
    assert np.all(np.abs(dg["sum_Q"][:2, 0] - dg0["sum_Q"][:2, 0]) <= 1e-13 * dg0["sum_Q"][:2, 0])


def sweep():
    """The paper's parameter study: shell thickness r_2 - r_1 from 0.05 to
    0.3 and gamma_2 / gamma_1 from 1 to 10 (gamma_1 = 1.667), 320 cells."""
    out = []
    for dr in (0.05, 0.1, 0.2, 0.3):
        out.append(wl.icf_1d(n=320, r_out=1.0 + dr))
    for ratio in (2.0, 5.0, 10.0):
        out.append(wl.icf_1d(n=320, gammas=(1.667, 1.667 * ratio, 1.667)))
    return out


def test_case_ii_parameter_sweep_batched(pk):
    insts = sweep()
    steps = 600
    print("icf sweep", len(insts), steps, flush=True)
    b = pk.Batch(insts)
    b.init(insts)
    b.step(steps)
    got = b.get()
    for q, w in enumerate(insts):
        o = oracle.run(w, steps=steps)
        g = o.get()
        assert np.array_equal(g["chi"], got[q]["chi"]), q
        Q0, Q1 = g["Q"], got[q]["Q"]
        for m in range(Q0.shape[0]):
            for v in range(Q0.shape[1]):
                ref = math.fsum(np.abs(Q0[m, v]).ravel())
                err = math.fsum(np.abs(Q1[m, v] - Q0[m, v]).ravel())
                assert err <= 1e-9 * ref, (q, m, v, err / max(ref, 1e-300))
        assert np.abs(g["alpha"] - got[q]["alpha"]).max() <= 1e-12, q
        print(q, "bitwise", bool(np.array_equal(Q0, Q1)), flush=True)


def test_case_ii_batched_bookkeeping(pk):
    insts = sweep()[:3]
    steps = 200
    b = pk.Batch(insts)
    b.init(insts)
    d0 = b.diag()
    b.step(steps)
    d1 = b.diag()
    for q, w in enumerate(insts):
        o = oracle.run(w, steps=steps)
        do = o.diag()
        ref, absref = rsums(o.get()["Q"], 0.0, 1.5 / 320)
        scale = np.maximum(absref.max(axis=1, keepdims=True), 1e-300)
        assert np.all(np.abs(d1[q]["sum_Q"][:3] - ref) <= 1e-13 * np.maximum(absref, 1e-300)), q
        assert np.all(np.abs(d1[q]["exch"][:3] - do["xsum"]) <= 1e-13 * scale), q
        bal = (d1[q]["sum_Q"] - d0[q]["sum_Q"] - d1[q]["bnd_in"] - d1[q]["exch"])[:2] - do["xfer"][:2]
        assert np.all(np.abs(bal) <= 1e-13 * scale[:2]), (q, bal)


def test_case_ii_rejections(pk):
    w = wl.triple_point(nx=28, ny=12)
    for extra in ({"coord": 1}, {"fs_on": 1, "fs_mat": 2, "fs_p": [1.0, 1.0, 0.0, 1.0, 0.1]}):
        cfg = dict(w["cfg"], **extra)
        with pytest.raises(pk.MMError) as e:
            pk.Solver(cfg)
        assert e.value.status == 1, extra
    w = wl.icf_1d(n=80)
    with pytest.raises(pk.MMError) as e:
        pk.Solver(dict(w["cfg"], flux=1))
    assert e.value.status == 1
    with pytest.raises(pk.MMError) as e:
        pk.Solver(dict(w["cfg"], fs_p=[13.0, 0.5, 0.1, 0.1, 0.1]))
    assert e.value.status == 1
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    with pytest.raises(pk.MMError) as e:
        s.step(2, record=2)
    assert e.value.status == 6
