"""Write the oracle's results at the full step counts of the workloads.

Runs the CPU oracle only (no GPU code) and stores, per workload, an .npz
with: the time reached and step count (a run that meets a non-physical state
stops; the stored state is then the one after the last complete step, and
the status and cell of the failing step are kept), the full indicator field
chi, per
(material, component) sums of Q and |Q|, and the complete state (Q, alpha,
phi) at a fixed sample of cells: every cell within one cell of an interface
at the end, plus a seeded random sample.  The GPU parity test recomputes the
same run and compares element by element on the sample.

Usage: python tests/golden/make_long_runs.py <name> [steps]
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

WORKLOADS = {
    "shock_tube_1d": lambda: wl.shock_tube_1d(),
    "triple_point": lambda: wl.triple_point(),
    "shock_bubble": lambda: wl.shock_bubble(),
    "shock_bubble_512": lambda: wl.shock_bubble(nx=512, ny=128, steps=300),
}


def sample_cells(chi, n_random=8192, seed=20170403):
    ny, nx = chi.shape
    pad = np.pad(chi, 1, mode="edge")
    mixed = np.zeros_like(chi, dtype=bool)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            mixed |= pad[1 + dj:1 + dj + ny, 1 + di:1 + di + nx] != chi
    rng = np.random.default_rng(seed)
    rand = rng.choice(ny * nx, size=min(n_random, ny * nx), replace=False)
    sel = np.zeros(ny * nx, dtype=bool)
    sel[rand] = True
    sel |= mixed.ravel()
    return np.nonzero(sel)[0]


def main():
    name = sys.argv[1]
    w = WORKLOADS[name]()
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else w["steps"]
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    t0 = time.time()
    done, status, chunk = 0, 0, 50
    # a step that meets a non-physical state stops part-way; the stored state
    # is the one after the last complete step
    g, d = o.get(), o.diag()
    while done < steps:
        n = min(chunk, steps - done)
        for _ in range(n):
            status = o.step(1)
            if status:
                break
            done += 1
            g, d = o.get(), o.diag()
        print(f"{name}: {done}/{steps} steps, {time.time() - t0:.0f}s", flush=True)
        if status:
            break
    Q = g["Q"]
    cells = sample_cells(g["chi"])
    M, nv = Q.shape[:2]
    flatQ = Q.reshape(M, nv, -1)
    out = dict(
        name=name, steps=done, requested=steps, status=status,
        err_cell=o.err_cell() if status else -1, t=d["t"],
        chi=g["chi"].astype(np.int8),
        sum_Q=np.array([[math.fsum(flatQ[m, v]) for v in range(nv)] for m in range(M)]),
        sum_absQ=np.array([[math.fsum(np.abs(flatQ[m, v])) for v in range(nv)] for m in range(M)]),
        cells=cells.astype(np.int64),
        Q=flatQ[:, :, cells],
        alpha=g["alpha"].reshape(M, -1)[:, cells],
        phi=g["phi"].ravel()[cells],
    )
    path = os.path.join(HERE, f"long_{name}.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}: {done} steps, status {status}, t = {d['t']:.6f}, "
          f"{len(cells)} sampled cells", flush=True)


if __name__ == "__main__":
    main()
