"""Write the oracle's results for the ragged batch of 256 1D tubes after 500
steps each (``workloads.batched_tubes``).

Runs the CPU oracle only (no GPU code), one instance at a time, in a pool
of worker processes.  Stored per instance: the SHA-256 of the final state
(Q [3][3][nx], alpha [3][nx], phi [nx] as little-endian float64 bytes, chi
[nx] as int32 bytes, in that order), the time reached, the update count,
the sums of Q per (material, component), and the full state of a fixed
sample of cells (every cell within one cell of an interface at the end,
plus 8 seeded random cells).  A GPU run that reproduces the oracle bit for
bit reproduces the hashes; the sampled cells and sums give the error when
it does not.

Usage: python tests/golden/make_batched_500.py [workers]
"""
import hashlib
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

STEPS = 500


def state_hash(Q, alpha, phi, chi):
    h = hashlib.sha256()
    for a, dt in ((Q, "<f8"), (alpha, "<f8"), (phi, "<f8"), (chi, "<i4")):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def sample(chi, q):
    n = chi.size
    c = chi.ravel()
    near = np.zeros(n, bool)
    near[1:] |= c[1:] != c[:-1]
    near[:-1] |= c[1:] != c[:-1]
    rng = np.random.default_rng(1000 + q)
    near[rng.choice(n, size=8, replace=False)] = True
    return np.nonzero(near)[0]


def run_one(q):
    w = wl.batched_tubes(steps=STEPS)[q]
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    st = o.step(STEPS)
    g, d = o.get(), o.diag()
    cells = sample(g["chi"], q)
    Q = g["Q"].reshape(3, 3, -1)
    return dict(q=q, status=st, hash=state_hash(g["Q"], g["alpha"], g["phi"], g["chi"]),
                t=d["t"], n_updates=d["n_updates"],
                sums=np.array([[math.fsum(Q[m, v]) for v in range(3)] for m in range(3)]),
                cells=cells, Qs=Q[:, :, cells], alphas=g["alpha"].reshape(3, -1)[:, cells],
                phis=g["phi"].ravel()[cells], chis=g["chi"].ravel()[cells])


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    n = len(wl.batched_tubes(steps=STEPS))
    t0 = time.time()
    with Pool(workers) as pool:
        res = []
        for r in pool.imap(run_one, range(n)):
            res.append(r)
            if len(res) % 32 == 0:
                print(f"{len(res)}/{n} instances, {time.time() - t0:.0f}s", flush=True)
    assert all(r["status"] == 0 for r in res)
    ncell = np.array([r["cells"].size for r in res])
    off = np.concatenate([[0], np.cumsum(ncell)])
    out = dict(steps=STEPS, hashes=np.array([r["hash"] for r in res]),
               t=np.array([r["t"] for r in res]),
               n_updates=np.array([r["n_updates"] for r in res], np.int64),
               sums=np.stack([r["sums"] for r in res]), cell_off=off,
               cells=np.concatenate([r["cells"] for r in res]).astype(np.int32),
               Q=np.concatenate([r["Qs"] for r in res], axis=2),
               alpha=np.concatenate([r["alphas"] for r in res], axis=1),
               phi=np.concatenate([r["phis"] for r in res]),
               chi=np.concatenate([r["chis"] for r in res]).astype(np.int8))
    path = os.path.join(HERE, "batched_tubes_500.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}: {n} instances, {off[-1]} sampled cells, {time.time() - t0:.0f}s",
          flush=True)


if __name__ == "__main__":
    main()
