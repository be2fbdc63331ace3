#!/usr/bin/env python3
"""Throughput of the cut-cell multi-material step on one MI355X.

One "step" is one full time step of the method (all Runge-Kutta stages of
geometry, ghost states, interface exchange, fluxes, level set and mixing)
on the 2D nested shock-bubble problem (4 x 1 box, 2048 x 512 uniform cells,
Mach 1.22 shock into a two-material bubble, three ideal gases, inflow /
outflow / reflective boundaries), FP64, synthetic analytic initial data
already resident on the GPU.  The unit of work is one active material-cell
RK-substep update (a cell/material pair with alpha > 0, updated in one
stage), counted on the device.  The K timed steps are a window centred in
the workload's full run (the whole run when K is its full length), reached
by untimed steps from t = 0 after the warm-up.

Prints one JSON line.  Also reports the dominant kernel (the bulk
flux/update kernel) against the HBM roof from its algorithmic bytes (HIP
events around its launches on the stream it runs on), with its FP64
operation rate against the FP64 vector issue rate beside it, the whole
step's HBM fraction, the same workload at 8192 x 2048 (working set far
beyond the 256 MB last-level cache), the triple point at 896 x 384, the
1D cylindrical implosion (one instance and its parameter study batched), the
batched form, the adjoint, and the CPU oracle's rate on a bounded sample of
the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector peak of the MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops
# (fused multiply-add) x 2.4 GHz; the path is compiled without contraction
# (bitwise parity with the oracle), so each lane issues at most one FP64
# add / multiply / divide step per clock: half of that, 39.3 T operations/s
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP64_NOFMA_PEAK_TOPS = 39.3
# algorithmic HBM bytes of one 2D update: read Q^(s) 32 + write Q^(s+1) 32 +
# read Q^n in two of three stages 21.3
BYTES_PER_UPDATE_2D = 32.0 + 32.0 + 2.0 / 3.0 * 32.0
# the main workload and its full length
WORKLOAD = dict(name="shock_bubble", nx=2048, ny=512)
FULL_STEPS = 3000
# FP64 operations (add, subtract, multiply, divide, square root) of one bulk
# 2D update, mean over the three SSP-RK3 stages: 2 faces x (8 WENO5 + 1 HLLC)
# + the cell's primitive state + 4 RK combinations.  Counted from the
# library's own point-wise templates by tests/opcount/op_count.cpp (a CPU
# test keeps the two in step).
FLOPS_PER_BULK_UPDATE_2D = 1320.0
COUNTERS = os.path.join(ROOT, "profiles",
                        "k_flux_bulk2_counters_shock_bubble_2048x512_8192x2048.md")
KERNEL_SOURCES = ("paper_1704_00519_amd/csrc/mmfv_kernels.h", "paper_1704_00519_amd/csrc/mmfv_math.h")


def measured_traffic(grid="2048x512"):
    """HBM bytes per launch of the dominant kernel on the given grid from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE runs, calibrated on
    a plain copy), if it was taken on the current kernel sources; else None."""
    import re
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    t = re.search(r"traffic_bytes_per_launch_%s: (\d+)" % grid, text)
    h = re.search(r"kernel_sources_sha256: ([0-9a-f]+)", text)
    if not t or not h:
        return None
    return int(t.group(1)) if bulk_kernel_sha256() == h.group(1) else None


def bulk_kernel_sha256():
    """Hash of the bulk kernel's source: its section of mmfv_kernels.h (from
    the bulk-update comment to the 1D bulk tile) and the point-wise numerics
    it calls (mmfv_math.h from its templates on; the parameter block before
    them gains fields that the kernel does not read)."""
    import hashlib
    kern = open(os.path.join(ROOT, KERNEL_SOURCES[0]), "rb").read()
    a = kern.index(b"// Bulk update: cells with no cut cell")
    b = kern.index(b"// 1D bulk update of one tile")
    math = open(os.path.join(ROOT, KERNEL_SOURCES[1]), "rb").read()
    m0 = math.index(b"// The point-wise functions below are templates")
    d = hashlib.sha256()
    d.update(kern[a:b])
    d.update(math[m0:])
    return d.hexdigest()


def bulk_roofline(prof):
    """Roofline of the bulk flux/update kernel from the library's event
    timings: its algorithmic bytes per second against the HBM peak, and its
    FP64 operations per second against the FP64 issue rate without fused
    multiply-adds beside it (about 1.3k operations per update against 85
    bytes: the operation count, not the bytes, sets its floor)."""
    n = max(1, prof["bulk_launches"])
    bulk_s = prof["bulk_ms"] * 1e-3
    upd = prof["bulk_updates"]
    tops = FLOPS_PER_BULK_UPDATE_2D * upd / bulk_s / 1e12 if bulk_s > 0 else 0.0
    gbs = prof["bulk_bytes"] / bulk_s / 1e9 if bulk_s > 0 else 0.0
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None, kernel="k_flux_bulk2",
                bytes_per_update=round(BYTES_PER_UPDATE_2D, 3),
                updates_per_launch=upd / n, bytes_per_launch=prof["bulk_bytes"] / n,
                launches=prof["bulk_launches"], avg_launch_us=round(prof["bulk_ms"] * 1e3 / n, 2),
                alu=dict(achieved=round(tops, 3), peak=FP64_NOFMA_PEAK_TOPS,
                         unit="T FP64 op/s (no FMA)", frac=round(tops / FP64_NOFMA_PEAK_TOPS, 4),
                         ops_per_update=FLOPS_PER_BULK_UPDATE_2D,
                         frac_of_fma_peak=round(tops / FP64_VECTOR_PEAK_TFLOPS, 4)))


def whole_step_hbm(rate):
    """Whole-step rate as a fraction of the HBM roof (algorithmic bytes)."""
    gbs = rate * BYTES_PER_UPDATE_2D / 1e9
    return dict(achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4))


def timed_run(pk, w, stream, steps, warmup, start):
    """Warm-up on a throwaway context (graph capture, first touch), then a
    fresh context from t = 0: `start` untimed steps, then exactly `steps`
    timed steps (events on the solver's stream around the graph replays)."""
    import torch
    if warmup:
        s = pk.Solver(w["cfg"], stream=stream.cuda_stream)
        s.init(w["phi"], w["chi"], w["W"])
        s.step(warmup)
        s.close()
    s = pk.Solver(w["cfg"], stream=stream.cuda_stream)
    s.init(w["phi"], w["chi"], w["W"])
    s.step(start) if start else s.step(0)  # step(0) captures the step graph
    torch.cuda.synchronize()
    d0 = s.diag()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d1 = s.diag()
    updates = d1["n_updates"] - d0["n_updates"]
    return s, dict(ms=ms, wall=wall, updates=updates, rate=updates / (ms * 1e-3),
                   t_start=d0["t"], t_end=d1["t"], step_start=d0["steps"],
                   n_band=d1["n_band"], n_tiles=d1["n_tiles"])


def profile_bulk(s, steps):
    """The bulk kernel's launches bracketed by HIP events (graph replay off
    while they are recorded) over `steps` further steps."""
    s.set_profiling(True)
    s.step(steps)
    prof = s.profile()
    s.set_profiling(False)
    return prof


def hbm_resident_leg(pk, wl, stream, nx=8192, ny=2048, warm=3, steps=20):
    """The shock-bubble problem at 8192 x 2048 (the effective resolution of
    the paper's Case V; working set of several GB, far beyond the 256 MB
    last-level cache): whole steps timed, and the bulk kernel against the
    HBM roof, where its algorithmic bytes have to come from HBM."""
    import torch
    w = wl.shock_bubble(nx=nx, ny=ny)
    s, r = timed_run(pk, w, stream, steps, 0, warm)
    del w
    prof = profile_bulk(s, 10)
    torch.cuda.synchronize()
    s.close()
    roof = bulk_roofline(prof)
    roof["traffic"] = measured_traffic(f"{nx}x{ny}")
    return dict(workload=f"shock_bubble_{nx}x{ny}", value=r["rate"], unit="updates/s",
                steps=steps, warmup=warm, ms_per_step=r["ms"] / steps,
                hbm_whole_step=whole_step_hbm(r["rate"]), roofline=roof)


def triple_point_leg(pk, wl, stream, steps=300, warm=10):
    """Case III at 896 x 384 (whole steps after a warm-up), for comparison
    with the earlier figures of this workload."""
    w = wl.triple_point()
    s, r = timed_run(pk, w, stream, steps, 0, warm)
    s.close()
    return dict(workload="triple_point_896x384", value=r["rate"], unit="updates/s",
                steps=steps, warmup=warm, ms_per_step=r["ms"] / steps,
                t_start=r["t_start"], t_end=r["t_end"])


def icf_leg(pk, wl, stream, n=1280, steps=5350, sweep_n=320, sweep_steps=1199, warm=10):
    """Case II (the 1D cylindrical implosion with a free surface): one
    instance at n cells over the run to t = 0.3 (`steps` steps), and the
    paper's parameter study as one batched launch over a 16 x 16 grid (shell
    thickness 0.16 to 0.31, gamma_2 / gamma_1 from 1 to 10: 256 instances at
    sweep_n cells, sweep_steps steps each; shells of 0.15 and thinner stop
    with a non-physical state near stagnation at these resolutions for some
    gamma ratios); the oracle's rate on the 320-cell instance beside them."""
    import torch
    import oracle
    w = wl.icf_1d(n=n)
    s, r = timed_run(pk, w, stream, steps, 0, warm)
    s.close()
    insts = [wl.icf_1d(n=sweep_n, r_out=1.0 + float(dr), gammas=(1.667, 1.667 * float(q), 1.667))
             for dr in np.linspace(0.16, 0.31, 16) for q in np.linspace(1.0, 10.0, 16)]
    b = pk.Batch(insts, stream=stream.cuda_stream)
    b.init(insts)
    b.step(1)
    torch.cuda.synchronize()
    u0 = sum(d["n_updates"] for d in b.diag())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(sweep_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    upd = sum(d["n_updates"] for d in b.diag()) - u0
    t_end = [round(d["t"], 4) for d in b.diag()]
    wo = wl.icf_1d(n=320)
    o = oracle.Oracle(wo["cfg"])
    assert o.init(wo["phi"], wo["chi"], wo["W"]) == 0
    t0 = time.perf_counter()
    o.step(1199)
    el = time.perf_counter() - t0
    return dict(workload=f"icf_1d_{n}", value=r["rate"], unit="updates/s", steps=steps,
                ms_per_step=r["ms"] / steps, t_end=r["t_end"],
                sweep=dict(instances=len(insts), cells=sweep_n, steps=sweep_steps + 1,
                           value=upd / (ms * 1e-3), unit="updates/s", ms=ms,
                           t_end_min=min(t_end), t_end_max=max(t_end)),
                cpu_oracle=dict(value=o.diag()["n_updates"] / el, unit="updates/s", cores=1,
                                sample="icf_1d 320 cells, 1199 steps (to t = 0.3)"))


def mr_leg(s, stream, w, block=16, levels=5, eps=1e-3, reps=20):
    """Multiresolution analysis (Sec. 2.4) of the state the solver holds:
    the paper's block structure (16 x 16 blocks, five levels above the
    4 x 1 coarsest blocks of the 2048 x 512 grid), timed over `reps` calls
    (each synchronises and copies the leaf map out), against the HBM roof
    from its algorithmic bytes: per cell of the grid 41 B for the fields
    (rho and rho E of the cell's material, occupancy and level set read,
    two fields written) and per level 16 B per fine and per coarse cell for
    each of the projection and the detail passes.  Beside it, the oracle's
    analysis (numpy) of the workload's initial state, on the host."""
    import torch
    nx, ny = s.nx, s.ny
    r = s.mr_analyse(block=block, levels=levels, eps=eps, flags=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = s.mr_analyse(block=block, levels=levels, eps=eps, flags=False)
    el = (time.perf_counter() - t0) / reps
    n = [(nx >> (levels - l)) * (ny >> (levels - l)) for l in range(levels + 1)]
    byt = 41.0 * nx * ny + sum(2 * 16.0 * (n[l + 1] + n[l]) for l in range(levels))
    gbs = byt / el / 1e9
    import oracle
    from oracle import mr
    o = oracle.Oracle(w["cfg"])
    assert o.init(w["phi"], w["chi"], w["W"]) == 0
    g = o.get()
    band = s.cfg["band_ls"] * min((s.cfg["x1"] - s.cfg["x0"]) / nx, (s.cfg["y1"] - s.cfg["y0"]) / ny)
    t0 = time.perf_counter()
    mr.analyse(g["Q"], g["phi"], band, B=block, L=levels, eps=eps)
    cpu_ms = (time.perf_counter() - t0) * 1e3
    return dict(block=block, levels=levels, eps=eps, ms=el * 1e3, bytes=byt,
                achieved_gbs=round(gbs, 1), frac_hbm=round(gbs / HBM_PEAK_GBS, 4),
                counts=r["counts"], compression=r["compression"],
                cpu_oracle_ms=round(cpu_ms, 1))


def host_cpu():
    """Host core count and model of the machine the oracle runs on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(workload, steps, runs=5):
    """The oracle (plain single-threaded C, one core) on the same workload:
    `runs` runs of the first `steps` steps from t = 0, median rate."""
    import oracle
    rates = []
    for _ in range(runs):
        o = oracle.Oracle(workload["cfg"])
        assert o.init(workload["phi"], workload["chi"], workload["W"]) == 0
        t0 = time.perf_counter()
        rc = o.step(steps)
        el = time.perf_counter() - t0
        if rc:
            return None
        rates.append(o.diag()["n_updates"] / el)
        del o
    ncpu, model = host_cpu()
    cfg = workload["cfg"]
    return dict(value=float(np.median(rates)), unit="updates/s", cores=1, kind="oracle",
                sample=f"{workload['name']} {cfg['nx']}x{cfg['ny']}, first {steps} steps "
                       f"from t=0, single-threaded C oracle, median of {runs} runs",
                runs=[round(r) for r in rates], host_nproc=ncpu, host_cpu=model)


def batched(pk, wl, stream, steps, ref_inst=8, ref_steps=30):
    """Batched form: the 256 ragged 1D tubes in one persistent launch, and the
    same work done instance by instance with the single-instance entry point
    (measured on a subset, per update)."""
    import torch
    insts = wl.batched_tubes(steps=steps)
    b = pk.Batch(insts, stream=stream.cuda_stream)
    b.init(insts)
    b.step(1)  # chooses the workgroup size (state snapshot restored)
    torch.cuda.synchronize()
    u0 = sum(d["n_updates"] for d in b.diag())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    upd = sum(d["n_updates"] for d in b.diag()) - u0
    threads, tune = b.threads()
    # per-instance launches: each instance on its own context, one after the
    # other on the same stream
    per_upd, per_ms = 0, 0.0
    for w in insts[:ref_inst]:
        s = pk.Solver(w["cfg"], stream=stream.cuda_stream)
        s.init(w["phi"], w["chi"], w["W"])
        s.step(1)
        torch.cuda.synchronize()
        d0 = s.diag()["n_updates"]
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        s.step(ref_steps)
        f1.record(stream)
        torch.cuda.synchronize()
        per_ms += f0.elapsed_time(f1)
        per_upd += s.diag()["n_updates"] - d0
        s.close()
    rate = upd / (ms * 1e-3)
    per_rate = per_upd / (per_ms * 1e-3)
    return dict(value=rate, unit="updates/s", instances=len(insts), steps=steps,
                ms=ms, workgroup=threads, tune_ms=[round(x, 3) for x in tune],
                per_instance_value=per_rate,
                per_instance_sample=f"first {ref_inst} instances x {ref_steps} steps, "
                                    "one context each, same stream",
                speedup=rate / per_rate)


def adjoint_leg(pk, wl, stream, steps=300, K=30):
    """Differentiation form on the 512 x 128 nested shock-bubble: gradient of
    the bubble's centroid x-position after `steps` steps with respect to
    (shell density, core density, shock Mach number) through the library's
    reverse steps, checkpoint every K steps.  Cost = wall time of (forward
    with tape + all reverse steps) over that of the plain forward run."""
    import torch
    from paper_1704_00519_amd import adjoint as ad
    prob = ad.NestedBubble(wl.shock_bubble(nx=512, ny=128))
    params = np.array([0.138, 3.15, 1.22])
    s = prob.solver(params, stream=stream.cuda_stream)
    s.step(2)  # graph capture and first-touch outside the timing
    s = prob.solver(params, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s = prob.solver(params, stream=stream.cuda_stream)
    alpha0 = s.get()["alpha"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, record=K)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    g = ad.reverse_gradient(prob, s, alpha0, steps, params)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    J, _ = ad.centroid(s.get()["alpha"], prob.x)
    return dict(workload="nested_shock_bubble_512x128", steps=steps, checkpoint_every=K,
                forward_s=round(t_fwd, 4), forward_with_tape_s=round(t_rec, 4),
                forward_and_reverse_s=round(t_all, 4), ratio=t_all / t_fwd,
                J=J, gradient=[float(x) for x in g],
                parameters=["rho_shell", "rho_core", "mach"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=FULL_STEPS)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--start", type=int, default=None,
                    help="first timed step (default: the K-step window centred in the full run)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-hbm-leg", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the main workload (for profiler runs)")
    ap.add_argument("--grid", default=f"{WORKLOAD['nx']}x{WORKLOAD['ny']}",
                    help="grid of the shock-bubble workload (profiler runs at other sizes)")
    ap.add_argument("--icf-only", action="store_true",
                    help="run only the Case II leg (one JSON object)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_00519_amd as pk
    import workloads as wl

    if args.icf_only:
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        print(json.dumps(icf_leg(pk, wl, stream)))
        return
    nx, ny = (int(v) for v in args.grid.split("x"))
    w = wl.shock_bubble(nx=nx, ny=ny)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # a real stream: time steps replay a captured graph
    torch.cuda.set_stream(stream)
    start = args.start if args.start is not None else max(0, (FULL_STEPS - args.steps) // 2)
    s, r = timed_run(pk, w, stream, args.steps, args.warmup, start)
    value = r["rate"]
    prof = profile_bulk(s, max(1, min(args.steps, 20)))
    mr = None if args.no_extra else mr_leg(s, stream, w)
    s.close()
    roofline = bulk_roofline(prof)
    roofline["traffic"] = measured_traffic(f"{nx}x{ny}")
    roofline["share_of_step"] = round(prof["bulk_ms"] / max(1, min(args.steps, 20)) /
                                      (r["ms"] / args.steps), 4)
    out = dict(metric="material-cell RK-substep updates/sec (plain)",
               value=value, unit="updates/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=r["ms"] / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload=f"shock_bubble_{nx}x{ny}", grid=[nx, ny],
                           materials=3, rk_stages=3, cfl=0.6, full_steps=FULL_STEPS,
                           step_start=r["step_start"], t_start=r["t_start"],
                           t_end=r["t_end"], band_cells_last_stage=r["n_band"],
                           wall_s=round(r["wall"], 3)),
               roofline=roofline, hbm_whole_step=whole_step_hbm(value))
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8,
                                         "launches": 3}
    if mr is not None:
        out["mr"] = mr
    if not args.no_extra:
        if not args.no_hbm_leg:
            out["hbm_resident"] = hbm_resident_leg(pk, wl, stream)
        out["triple_point"] = triple_point_leg(pk, wl, stream)
        out["icf"] = icf_leg(pk, wl, stream)
        if not args.no_batch:
            out["batched"] = batched(pk, wl, stream, args.batch_steps)
        if not args.no_adjoint:
            out["adjoint"] = adjoint_leg(pk, wl, stream)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
