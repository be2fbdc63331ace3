"""GPU parity where conserved quantities move between the materials of a
cell: mixing sources without an eligible target (their state joins the
cell's material; a fragment of the cell's own material first gives the cell
to the material of largest other volume fraction) and the interface
scale-separation model after every step (Sec. 2.3.3).  The library against
the oracle on the oracle's own pin cases (a filament removed by the model,
one removed by the mixing reading, a droplet below the grid scale), 1D thin
layers (plain and batched), and the triple point at two sizes; every
counter of moves must equal the oracle's, the state meet the 1e-9 bar.
A tape recorded over such a step cannot be reversed (MM_ENOTIMPL)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_parity import assert_parity
from test_oracle_scale_sep import droplet, layered

pytestmark = pytest.mark.gpu
N = 20
MOVES = ("n_absorb", "n_relabel", "n_oddball", "n_stranded")


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


def thin1d(n, a, b):
    x = (np.arange(n) + 0.5) / n
    chi = np.where(x < a, 0, np.where(x < b, 1, 2)).astype(np.int32)
    phi = np.where(x < a, a - x, np.where(x < b, np.minimum(x - a, b - x), x - b))
    cfg = wl.base_config(dim=1, nx=n, ny=1, n_mat=3, gamma=[1.4, 1.667, 1.4],
                         pinf=[0.0] * 3, bc=[wl.BC_REFLECTIVE] * 4, scale_sep=1)
    W = np.zeros((3, 3, 1, n))
    W[:, 0] = np.array([1.0, 1.5, 2.0])[:, None, None]
    W[:, 2] = 1.0
    return dict(cfg=cfg, phi=np.minimum(phi, 8.0 / n)[None], chi=chi[None], W=W)


def run_pair(pk, w, steps, dt=None):
    cfg = dict(w["cfg"], scale_sep=w["cfg"].get("scale_sep", 1))
    o = oracle.Oracle(cfg)
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    s = pk.Solver(cfg)
    s.init(w["phi"], w["chi"], w["W"])
    if dt:
        o.set_dt(dt)
        s.set_dt(dt)
    assert o.step(steps) == 0
    s.step(steps)
    return o, s


CASES = {
    "filament_model": lambda: layered([0.0, 0.5 - 0.8 / N, 0.5 + 0.8 / N, 1.0], [0, 1, 2]),
    "filament_mixing": lambda: layered([0.0, 0.5 - 0.6 / N, 0.5 + 0.6 / N, 1.0], [0, 1, 2]),
    "droplet_small": lambda: droplet(0.5 / N),
    "thin1d_a": lambda: thin1d(100, 0.5 - 0.3 / 100, 0.5 + 0.9 / 100),
    "thin1d_b": lambda: thin1d(137, 0.5 - 0.4 / 137, 0.5 + 1.0 / 137),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_moves_match_oracle_at_rest(pk, name):
    print("moves case", name, flush=True)
    o, s = run_pair(pk, CASES[name](), 3, dt=1e-4)
    d, do = s.diag(), o.diag()
    print(name, {k: (d[k], do[k]) for k in MOVES})
    assert sum(do[k] for k in MOVES[:3]) > 0
    for k in MOVES:
        assert d[k] == do[k], k
    info = assert_parity(o, s, label=name)
    assert info["bitwise"], info


@pytest.mark.parametrize("nx,ny,steps", [(112, 48, 60), (224, 96, 150)])
def test_triple_point_moves(pk, nx, ny, steps):
    print("triple point", nx, ny, steps, flush=True)
    # without the redistancing, so that many moves happen in these few steps
    o, s = run_pair(pk, wl.triple_point(nx=nx, ny=ny, scale_sep=1, reinit=0), steps)
    d, do = s.diag(), o.diag()
    print({k: (d[k], do[k]) for k in MOVES})
    for k in MOVES:
        assert d[k] == do[k], k
    assert do["n_oddball"] > 0 and do["n_absorb"] > 0
    print(assert_parity(o, s, label=f"triple_{nx}x{ny}"))


def test_batched_thin_layers(pk):
    insts = [thin1d(n, 0.5 - 0.3 / n, 0.5 + 0.9 / n) for n in (100, 160, 241)]
    insts += [thin1d(137, 0.5 - 0.4 / 137, 0.5 + 1.0 / 137)]
    print("batched thin layers", len(insts), flush=True)
    b = pk.Batch(insts)
    b.init(insts)
    b.step(4)
    got, diags = b.get(), b.diag()
    total = 0
    for q, w in enumerate(insts):
        o = oracle.run(w, steps=4)
        g = o.get()
        for k in ("Q", "alpha", "phi", "chi"):
            assert np.array_equal(g[k], got[q][k]), (q, k)
        for k in MOVES:
            assert diags[q][k] == o.diag()[k], (q, k)
        total += o.diag()["n_oddball"] + o.diag()["n_absorb"]
    assert total > 0


def test_tape_over_a_move_is_refused(pk):
    w = CASES["filament_mixing"]()
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    s.set_dt(1e-4)
    s.step(1, record=1)
    assert s.diag()["n_relabel"] > 0
    lamQ = np.zeros_like(s.get()["Q"])
    with pytest.raises(pk.MMError) as e:
        s.adjoint_step(lamQ, np.zeros((N, N)))
    assert e.value.status == 6
