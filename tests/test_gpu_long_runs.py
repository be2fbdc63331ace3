"""Long runs at full size against stored oracle results.

tests/golden/make_long_runs.py ran the oracle (and only the oracle) for the
workloads' full step counts and stored, per workload, the step reached (a
run that meets a non-physical state stops there, with status 4 and the
cell), the full indicator field, per (material, component) sums of Q and,
at a fixed sample of cells (every cell next to an interface at the end plus
a seeded random sample), the complete state.  Here the library repeats each
run on the GPU and is compared element by element on the sample, and in
its failure step and cell where the oracle failed.
"""
import math
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REL_L1 = 1e-9

RUNS = {
    "shock_tube_1d": lambda: wl.shock_tube_1d(),
    "shock_bubble_512": lambda: wl.shock_bubble(nx=512, ny=128, steps=300),
    "triple_point": lambda: wl.triple_point(),
    "shock_bubble": lambda: wl.shock_bubble(),
}


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


@pytest.mark.parametrize("name", sorted(RUNS))
def test_long_run_matches_stored_oracle_run(pk, name):
    path = os.path.join(HERE, "golden", f"long_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle run for {name}: tests/golden/make_long_runs.py writes it")
    ref = np.load(path)
    w = RUNS[name]()
    steps, status = int(ref["steps"]), int(ref["status"])
    s = pk.Solver(w["cfg"])
    s.init(w["phi"], w["chi"], w["W"])
    done = 0
    while done < steps:
        n = min(500, steps - done)
        s.step(n)
        done += n
        print(f"{name}: {done}/{steps} steps", flush=True)
    g = s.get()
    assert s.diag()["t"] == pytest.approx(float(ref["t"]), rel=1e-12)
    assert np.array_equal(g["chi"].astype(np.int8), ref["chi"])
    cells = ref["cells"]
    M, nv = g["Q"].shape[:2]
    Q = g["Q"].reshape(M, nv, -1)[:, :, cells]
    for m in range(M):
        for v in range(nv):
            r = ref["Q"][m, v]
            den = math.fsum(np.abs(r))
            err = math.fsum(np.abs(Q[m, v] - r))
            assert (err == 0.0) if den == 0.0 else (err / den <= REL_L1), (m, v, err, den)
    assert np.abs(g["alpha"].reshape(M, -1)[:, cells] - ref["alpha"]).max() <= 1e-12
    assert np.abs(g["phi"].ravel()[cells] - ref["phi"]).max() <= 1e-12
    full = g["Q"].reshape(M, nv, -1)
    for m in range(M):
        for v in range(nv):
            tot = math.fsum(full[m, v])
            assert abs(tot - ref["sum_Q"][m, v]) <= 1e-12 * max(ref["sum_absQ"][m, v], 1e-300)
    if status:
        # the oracle met a non-physical state in the next step: so must the
        # library, in the same cell
        with pytest.raises(pk.MMError) as e:
            s.step(1)
        assert e.value.status == status
        assert s.diag()["err_cell"] == int(ref["err_cell"])
