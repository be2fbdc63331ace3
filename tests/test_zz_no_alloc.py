"""The batched run without device allocation (mm_batch_run_noalloc) against
the allocating batched entry points: bitwise equal results, on two calls in
a row (the second with fewer, smaller instances, so the shared work array
holds the first call's contents when the second starts)."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _packed(insts):
    phi = np.concatenate([np.asarray(w["phi"], np.float64).ravel() for w in insts])
    chi = np.concatenate([np.asarray(w["chi"], np.int32).ravel() for w in insts])
    W = np.concatenate([np.asarray(w["W"], np.float64).ravel() for w in insts])
    return phi, chi, W


def _reference(pk, insts, steps, threads):
    b = pk.Batch(insts)
    b.init(insts)
    b.set_threads(threads)
    b.step(steps)
    out = b.get()
    b.close()
    return out


@pytest.mark.parametrize("threads", [256])
def test_noalloc_matches_batched_twice(threads):
    import torch
    import paper_1704_00519_amd as pk
    dev = torch.device("cuda:0")
    cases = [(wl.batched_tubes(n_inst=12, nmin=200, nmax=1200, steps=40), 40),
             (wl.batched_tubes(n_inst=5, seed=7, nmin=150, nmax=600, steps=25), 25)]
    for call, (insts, steps) in enumerate(cases):
        print(f"noalloc call {call}: {len(insts)} instances, {steps} steps", flush=True)
        phi, chi, W = _packed(insts)
        M = 3
        N = phi.size
        tphi = torch.from_numpy(phi).to(dev)
        tchi = torch.from_numpy(chi).to(dev)
        tW = torch.from_numpy(W).to(dev)
        Q = torch.full((M * 3 * N,), float("nan"), dtype=torch.float64, device=dev)
        al = torch.full((M * N,), float("nan"), dtype=torch.float64, device=dev)
        po = torch.full((N,), float("nan"), dtype=torch.float64, device=dev)
        co = torch.full((N,), -1, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        pk.batch_run_noalloc([w["cfg"] for w in insts], tphi, tchi, tW, steps, threads,
                             Q, al, po, co)
        Qh, ah, ph, ch = (Q.cpu().numpy(), al.cpu().numpy(), po.cpu().numpy(),
                          co.cpu().numpy())
        ref = _reference(pk, insts, steps, threads)
        o = 0
        for q, w in enumerate(insts):
            nx = int(w["cfg"]["nx"])
            r = ref[q]
            assert np.array_equal(Qh[M * 3 * o:M * 3 * (o + nx)], r["Q"].ravel()), (call, q)
            assert np.array_equal(ah[M * o:M * (o + nx)], r["alpha"].ravel()), (call, q)
            assert np.array_equal(ph[o:o + nx], r["phi"].ravel()), (call, q)
            assert np.array_equal(ch[o:o + nx], r["chi"].ravel()), (call, q)
            o += nx
        print(f"noalloc call {call}: bitwise equal", flush=True)


def test_noalloc_rejects_oversized():
    import torch
    import paper_1704_00519_amd as pk
    insts = wl.batched_tubes(n_inst=65, nmin=200, nmax=210, steps=1)
    N = sum(int(w["cfg"]["nx"]) for w in insts)
    dev = torch.device("cuda:0")
    z = torch.zeros(3 * 3 * N, dtype=torch.float64, device=dev)
    with pytest.raises(pk.MMError, match="MM_EINVAL"):
        pk.batch_run_noalloc([w["cfg"] for w in insts], z[:N], torch.zeros(N, dtype=torch.int32,
                             device=dev), z, 1, 256, z)
    big = wl.batched_tubes(n_inst=40, nmin=3900, nmax=4000, steps=1)
    N = sum(int(w["cfg"]["nx"]) for w in big)
    z = torch.zeros(3 * 3 * N, dtype=torch.float64, device=dev)
    with pytest.raises(pk.MMError, match="MM_EINVAL"):
        pk.batch_run_noalloc([w["cfg"] for w in big], z[:N], torch.zeros(N, dtype=torch.int32,
                             device=dev), z, 1, 256, z)
