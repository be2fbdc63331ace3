"""GPU parity of the multiresolution analysis (Sec. 2.4) with the oracle:
the detail flags of every level, the interface identifiers, the leaf level
of every block, the per-level counts and the fields' largest magnitudes,
exactly (every decision is a comparison of FP64 values that both sides form
in the same order).  States: both sides stepped from the same initial data
(the solvers agree bit for bit on these), the paper's block layouts (the
triple point with 7 x 3 blocks at the coarsest level, the shock bubble with
4 x 1), a smooth single-material field over a range of thresholds, and the
full 2048 x 512 bubble with five levels.  Also the rejected arguments."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import mr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


def smooth_field(n=128):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    cfg = wl.base_config(dim=2, nx=n, ny=n, n_mat=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                         gamma=[1.4], pinf=[0.0], bc=[wl.BC_TRANSMISSIVE] * 4)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) + 0.5 * (X > 0.62)
    W = np.stack([rho, 0.1 + 0 * X, 0 * X, 1.0 + 0.1 * np.cos(4 * np.pi * X)])[None]
    return dict(cfg=cfg, phi=np.full((n, n), 8.0 / n), chi=np.zeros((n, n), np.int32), W=W)


CASES = {
    # name: (workload, steps, [(block, levels, eps), ...])
    "triple_point_896x384_t0": (lambda: wl.triple_point(), 0, [(16, 3, 1e-3), (8, 3, 1e-4)]),
    "triple_point_448x192_s40": (lambda: wl.triple_point(nx=448, ny=192), 40, [(16, 2, 1e-3)]),
    "bubble_512x128_s100": (lambda: wl.shock_bubble(nx=512, ny=128), 100,
                            [(16, 3, 1e-3), (8, 4, 1e-4), (4, 5, 1e-2)]),
    "smooth_128": (smooth_field, 0, [(16, 3, 1e-2), (16, 3, 1e-4), (4, 5, 1e-6), (8, 4, 3e-3)]),
}


def band_of(cfg):
    return cfg["band_ls"] * min((cfg["x1"] - cfg["x0"]) / cfg["nx"],
                                (cfg["y1"] - cfg["y0"]) / cfg["ny"])


def compare(o, s, cfg, block, levels, eps, label):
    g = o.get()
    band = band_of(cfg)
    ref = mr.analyse(g["Q"], g["phi"], band, B=block, L=levels, eps=eps)
    got = s.mr_analyse(block=block, levels=levels, eps=eps, band=band)
    assert got["scale"] == ref["scale"], label
    for l in range(levels):
        assert np.array_equal(got["detail"][l], ref["detail"][l]), (label, "detail", l)
    for l in range(levels + 1):
        assert np.array_equal(got["iface"][l], ref["iface"][l]), (label, "iface", l)
    assert np.array_equal(got["leaf"], ref["leaf"]), label
    assert got["counts"] == ref["counts"], label
    assert got["compression"] == pytest.approx(ref["compression"], rel=1e-15)
    return got


@pytest.mark.parametrize("name", sorted(CASES))
def test_mr_matches_oracle(pk, name):
    make, steps, settings = CASES[name]
    w = make()
    print("mr case", name, steps, flush=True)
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    if steps:
        assert o.step(steps) == 0
        s.step(steps)
    before = s.get()["Q"]
    for block, levels, eps in settings:
        got = compare(o, s, w["cfg"], block, levels, eps, f"{name} {block} {levels} {eps}")
        print(name, block, levels, eps, "counts", got["counts"],
              "compression %.4f" % got["compression"], flush=True)
    # the analysis leaves the state alone
    assert np.array_equal(before, s.get()["Q"])


def test_mr_full_size_bubble(pk):
    """2048 x 512 with 16 x 16 blocks and five levels (4 x 1 blocks at the
    coarsest level, as the paper's Case V), at t = 0 and after 3 steps."""
    w = wl.shock_bubble()
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    compare(o, s, w["cfg"], 16, 5, 1e-3, "bubble_t0")
    assert o.step(3) == 0
    s.step(3)
    got = compare(o, s, w["cfg"], 16, 5, 1e-3, "bubble_s3")
    assert got["counts"][0][0] == 4  # 4 x 1 blocks at level 0
    print("bubble 2048x512 counts", got["counts"], "compression", got["compression"])


def test_mr_rejections(pk):
    w = wl.triple_point(nx=112, ny=48)
    s = pk.Solver(w["cfg"])
    with pytest.raises(pk.MMError) as e:
        s.mr_analyse(block=16, levels=1)
    assert e.value.status == 5  # before mm_init_state
    s.init(w["phi"], w["chi"], w["W"])
    for kw in (dict(block=16, levels=1), dict(block=1, levels=1), dict(block=8, levels=0),
               dict(block=8, levels=1, eps=0.0), dict(block=8, levels=11)):
        with pytest.raises(pk.MMError) as e:
            s.mr_analyse(**kw)
        assert e.value.status == 1, kw
    got = s.mr_analyse(block=8, levels=1)  # 112 = 8 x 14, 48 = 8 x 6
    assert got["leaf"].shape == (6, 14)
    w1 = wl.shock_tube_1d()
    s1 = pk.Solver(w1["cfg"])
    s1.init(w1["phi"], w1["chi"], w1["W"])
    with pytest.raises(pk.MMError) as e:
        s1.mr_analyse(block=8, levels=1)
    assert e.value.status == 1
