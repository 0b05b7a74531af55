#!/usr/bin/env python
"""Benchmark: finite-difference cell-updates/s of one FWI iteration's
propagation on one MI355X.

One step = the propagation work of one network-preconditioned FWI iteration
on the 600x200 layered model (64 shots, 600 receivers, 4000 steps, dt 0.8 ms,
15 Hz): the FWI gradient and the Born demigration-remigration pair of that
gradient, in one library call (fwi_gradient_pair): a forward sweep storing
the imaging history, the adjoint with imaging, the scattered field driven by
the stored history, and the second adjoint: four wavefield passes over all
shots. Inputs are resident in HBM before the timed region; every step is
timed with HIP events and ms_per_step is the median. Beside the headline:
the same step with checkpointed wavefields (`checkpointed`), the HBM-bound
fractions of the stencil kernels on a grid far beyond the last-level cache
(`spill_probe`, also carried in `roofline.hbm_bound`), the operator variants,
the network's training and inference, the FWI time to model error and the
FP64 oracle on the host's cores (`cpu_baseline`). Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0      # dense bf16 matrix-core peak of MI355X

# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from a plain 1 GiB copy;
# see profiles/stencil_kernels_layered_600x200_hbm_counters.md). Valid only
# for the kernel source it was measured on: reported as null otherwise.
MEASURED_TRAFFIC = {
    # FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 per launch, by the tiling the
    # class runs with: "columns per lane, rows per wave, levels per launch,
    # rows prefetched" (two-level launches advance two time levels)
    "kernels_sha1": "22d3d4607b1407e9646db99b75bf0fb415125ee6",
    "stencil_adj": {"1,8,1,1": 258.1e6, "1,8,1,2": 253.1e6, "1,16,1,1": 273.0e6, "1,16,1,2": 272.8e6,
        "1,16,2,1": 434.2e6, "1,16,2,2": 438.5e6, "1,24,1,1": 264.5e6, "1,24,1,2": 265.7e6,
        "1,24,2,1": 413.5e6, "1,24,2,2": 414.6e6, "1,32,1,1": 260.3e6, "1,32,1,2": 261.7e6,
        "1,32,2,2": 405.8e6, "1,48,1,1": 249.7e6, "1,48,1,2": 250.9e6, "1,48,2,1": 374.2e6,
        "1,48,2,2": 378.5e6, "1,96,2,2": 358.4e6, "2,8,1,1": 266.6e6, "2,8,1,2": 262.7e6, "2,16,1,1": 271.3e6,
        "2,16,1,2": 272.9e6, "2,16,2,2": 426.6e6, "2,24,1,1": 262.1e6, "2,24,1,2": 264.3e6,
        "2,24,2,1": 398.1e6, "2,24,2,2": 396.9e6, "2,32,1,1": 257.0e6, "2,32,1,2": 258.3e6,
        "2,32,2,2": 384.9e6, "2,48,2,1": 361.9e6, "2,48,2,2": 364.0e6, "2,96,2,2": 350.5e6},
    "stencil_fwd": {"1,8,1,1": 170.8e6, "1,8,1,2": 167.3e6, "1,16,1,1": 189.3e6, "1,16,1,2": 187.4e6,
        "1,16,2,1": 324.8e6, "1,16,2,2": 325.6e6, "1,24,1,1": 179.3e6, "1,24,1,2": 180.8e6,
        "1,24,2,1": 304.7e6, "1,24,2,2": 306.0e6, "1,32,1,1": 175.2e6, "1,32,1,2": 175.9e6,
        "1,32,2,2": 296.9e6, "1,48,1,1": 170.3e6, "1,48,1,2": 170.4e6, "1,48,2,1": 276.8e6,
        "1,48,2,2": 278.7e6, "1,96,2,2": 270.3e6, "2,8,1,1": 183.7e6, "2,8,1,2": 177.2e6, "2,16,1,1": 187.1e6,
        "2,16,1,2": 187.8e6, "2,16,2,2": 320.3e6, "2,24,1,1": 177.7e6, "2,24,1,2": 178.1e6,
        "2,24,2,1": 297.6e6, "2,24,2,2": 297.4e6, "2,32,1,1": 174.4e6, "2,32,1,2": 174.7e6,
        "2,32,2,2": 286.4e6, "2,48,2,1": 271.7e6, "2,48,2,2": 271.6e6, "2,96,2,2": 263.2e6},
    "stencil_born": {"1,8,1,1": 169.3e6, "1,8,1,2": 166.7e6, "1,16,1,1": 186.9e6, "1,16,1,2": 185.8e6,
        "1,16,2,1": 356.9e6, "1,16,2,2": 352.3e6, "1,24,1,1": 180.2e6, "1,24,1,2": 181.4e6,
        "1,24,2,1": 329.0e6, "1,24,2,2": 324.7e6, "1,32,1,1": 175.3e6, "1,32,1,2": 176.6e6,
        "1,32,2,2": 314.2e6, "1,48,1,1": 170.4e6, "1,48,1,2": 170.5e6, "1,48,2,1": 289.4e6,
        "1,48,2,2": 297.1e6, "1,96,2,2": 271.0e6, "2,8,1,1": 176.1e6, "2,8,1,2": 172.0e6, "2,16,1,1": 186.4e6,
        "2,16,1,2": 186.3e6, "2,16,2,2": 352.6e6, "2,24,1,1": 178.8e6, "2,24,1,2": 179.8e6,
        "2,24,2,1": 325.3e6, "2,24,2,2": 319.1e6, "2,32,1,1": 175.5e6, "2,32,1,2": 176.2e6,
        "2,32,2,2": 307.3e6, "2,48,2,1": 282.9e6, "2,48,2,2": 281.7e6, "2,96,2,2": 267.4e6},
}


# Algorithmic bytes per cell-update of each pass: forward with the D^n
# emission 20 B; adjoint with imaging 28 B less 8 (1 - 1/k) when k time
# levels share one read-modify-write of the image; joint Born 16 B per field
# update; the scattered field driven by the stored history 24 B. The
# library's byte counters hold each kernel's own minimal traffic instead,
# which a two-level launch lowers further (the field levels are read and
# written once per two updates): 14 B per forward and 18 B per adjoint
# update. Per-update figures by class and levels per launch: (table, own).
def bytes_per_update(cls: str, levels: int):
    if cls == "fwd":
        return 20.0, (20.0 if levels == 1 else 14.0)
    if cls == "adj":
        return 28.0 - 8.0 * (1.0 - 1.0 / levels), (28.0 if levels == 1 else 18.0)
    return 1.0, 1.0   # Born classes: one level per launch, table = own


def kernels_sha1() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2403_17518_amd", "csrc", "fwi_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-shots", type=int, default=0, help="0: one per usable host thread (at most 64)")
    ap.add_argument("--cpu-nt", type=int, default=600)
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-checkpointed", action="store_true",
                    help="skip the timing of the same step with checkpointed wavefields")
    ap.add_argument("--ckpt-budget-gb", type=float, default=16.0)
    ap.add_argument("--mem-budget-gb", type=float, default=0.0)
    ap.add_argument("--tiling", default="",
                    help="force the forward/adjoint tiling 'cols,rows,levels[,prefetch]' (default: autotuned)")
    ap.add_argument("--no-deblur", action="store_true", help="skip the network timing")
    ap.add_argument("--deblur-only", action="store_true",
                    help="run only the network timing (for profiling its kernels)")
    ap.add_argument("--deblur-paper-only", action="store_true",
                    help="only time the paper-scale deblurring network (widths 128-2048, depth 4)")
    ap.add_argument("--no-spill-probe", action="store_true",
                    help="skip the full-width salt-grid measurement of the stencil kernels")
    ap.add_argument("--spill-nt", type=int, default=60)
    ap.add_argument("--spill-only", action="store_true",
                    help="run only the full-width salt-grid measurement (for profiling its kernels)")
    ap.add_argument("--no-fwi", action="store_true",
                    help="skip the plain vs network-preconditioned FWI time-to-error run")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the off-grid / free-surface / relative-perturbation step timings")
    ap.add_argument("--variant-steps", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain 1 GiB device-to-device copy, three times: the reference for
    scaling the FETCH_SIZE / WRITE_SIZE counters of the stencil kernels."""
    import torch
    n = 1 << 28
    x = torch.ones(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "copies": 3}), flush=True)


def host_cpu() -> dict:
    """The host's CPU as this process sees it: logical CPUs of the machine,
    CPUs this process may run on, the cgroup quota, the thread cap from
    OMP_NUM_THREADS and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
            if q != "max":
                quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    usable = aff
    if quota:
        usable = min(usable, max(1, int(quota)))
    if omp and omp.isdigit():
        usable = min(usable, int(omp))
    return {"nproc": os.cpu_count(), "affinity": aff, "cgroup_quota": quota,
            "omp_num_threads": omp, "usable": usable, "model": model}


def cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the same step: the FWI
    gradient and the Born pair of its negative on `cpu_shots` shots (default:
    one per usable host thread, at most 64) and the first `cpu_nt` steps,
    run `cpu_runs` times; the rate is the step's four counted passes over the
    median run time. The oracle executes more than it is credited with: its
    adjoint recomputes the background forward of every shot and the pair's
    Born sweep advances two fields (7 wavefield passes run, 4 counted)."""
    import numpy as np
    import oracle
    from synth import configs
    from synth.problem import cell_updates
    hc = host_cpu()
    nshots = args.cpu_shots or min(64, hc["usable"])
    wl = configs.layered_600x200(nshots=64, nt=args.cpu_nt)
    pick = np.linspace(0, 63, nshots).round().astype(int)
    acq = wl.acq.subset(pick)
    cores = oracle.set_threads(min(hc["usable"], nshots))
    v0 = wl.v0.astype(np.float32).astype(np.float64)
    d_obs = oracle.forward(wl.grid, acq, wl.v_true.astype(np.float32).astype(np.float64))
    times = []
    for _ in range(args.cpu_runs):
        t0 = time.perf_counter()
        g, _, _ = oracle.gradient(wl.grid, acq, v0, d_obs)
        oracle.born_pair(wl.grid, acq, v0, -g)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    upd = 4 * cell_updates(wl.grid, acq)      # the same step's work count as the GPU value
    return {"value": upd / dt, "unit": "cell-updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"gradient + Born pair, {len(pick)} of 64 shots, {args.cpu_nt} of 4000 steps, FP64, "
                      f"OpenMP over shots; median of {len(times)} runs "
                      f"({', '.join(f'{t:.1f}' for t in times)} s); rate = the 4 counted passes / time "
                      f"(the oracle runs 7: its adjoint recomputes each shot's forward, the Born sweep "
                      f"advances two fields)",
            "host": hc}


def spill_probe(nt: int):
    """The stencil kernels on the 1700 x 350 salt grid with full-width
    windows (300 shots x 390 x 1740 padded cells, 0.8 GB per wavefield): one
    FWI gradient and one Born demigration of ``nt`` steps, first with the
    autotuned tilings, then with one time level per launch forced. Its working
    set is far beyond the 256 MB last-level cache, so the fractions measure
    HBM. A two-level launch moves fewer algorithmic bytes per cell-update, so
    its fraction is lower at a higher update rate; both are reported."""
    import numpy as np
    import torch
    from paper_2403_17518_amd import ops
    from synth import configs
    from synth.problem import cell_updates

    wl = configs.salt_full_width(nshots=300, nt=nt)
    grid, acq = wl.grid, wl.acq
    acq.wavelet = acq.wavelet.astype(np.float32)
    cells = cell_updates(grid, acq) // nt
    ctx = ops.FwiContext(0)
    try:
        v0 = torch.from_numpy(wl.v0.astype(np.float32)).cuda()
        d_obs = torch.zeros(acq.data_size(grid), device="cuda")
        dv = torch.from_numpy((wl.v_true - wl.v0).astype(np.float32)).cuda()

        def measure():
            ctx.fwi_gradient(grid, acq, v0, d_obs, want_misfit=False)   # plan, tuning, buffers
            ctx.born_demig(grid, acq, v0, dv)
            torch.cuda.synchronize()
            ctx.set_profiling(True)
            acc, tiles = {}, None
            for call in (lambda: ctx.fwi_gradient(grid, acq, v0, d_obs, want_misfit=False),
                         lambda: ctx.born_demig(grid, acq, v0, dv)):
                call()
                torch.cuda.synchronize()
                st = ctx.stats()
                tiles = tiles or st
                for k in ("ms_fwd", "ms_adj", "ms_born", "bytes_fwd", "bytes_adj", "bytes_born",
                          "n_fwd", "n_adj", "n_born"):
                    acc[k] = acc.get(k, 0.0) + st[k]
            ctx.set_profiling(False)
            res = {}
            for i, cls in enumerate(("fwd", "adj", "born")):
                ms, b, n = acc["ms_" + cls], acc["bytes_" + cls], acc["n_" + cls]
                if ms <= 0:
                    continue
                levels = tiles["tile_levels"][i] or 1
                gbs = b / (ms * 1e-3) / 1e9                     # the kernel's own minimal traffic
                table, own = bytes_per_update(cls, levels)
                res[cls] = {"tiling_cols_rows_levels_prefetch": [tiles["tile_cw"][i], tiles["tile_rows"][i],
                                                                 levels, tiles["tile_prefetch"][i]],
                            "us_per_level": ms / (n * levels) * 1e3,
                            "cell_updates_per_s": cells * (2 if cls == "born" else 1) / (ms / (n * levels) * 1e-3),
                            "achieved_GBs": gbs * table / own, "frac": gbs * table / own / HBM_PEAK_GBS,
                            "bytes_per_update": table if cls != "born" else 16.0,
                            "min_traffic": {"achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                                            "bytes_per_update": own if cls != "born" else 16.0}}
            return res

        out = {"workload": f"salt_full_width: 300 shots x 390 x 1740 padded cells (pitch 1760), {nt} steps, "
                           f"gradient + Born demigration", "cells_per_step": cells,
               "autotuned": measure()}
        ctx.set_tiling(0, 1, 32, 1, 1)
        ctx.set_tiling(1, 1, 32, 1, 1)
        out["one_level"] = measure()
        return out
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def variants(ctx, wl, v_true, v0, steps: int, base_ms: float):
    """The timed step (fused gradient + Born pair) of the same workload with
    each operator variant: sources and receivers off the grid (bilinear
    spreading and sampling, seeded fractions), a pressure-free top surface,
    the relative-perturbation Born operator, and a perfectly matched layer
    instead of the sponge. Per variant: observed data
    in that setting, one untimed step (plan, autotuning, graph capture),
    then `steps` steps timed with events."""
    import copy
    from dataclasses import replace
    import numpy as np
    import torch
    g0, a0 = wl.grid, wl.acq
    off = copy.deepcopy(a0)
    rng = np.random.default_rng(2403)
    nr = off.rec_z.shape[0]
    fz = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    fx = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    sfz = rng.uniform(0.0, 1.0, off.nshots).astype(np.float32)
    sfx = rng.uniform(0.0, 1.0, off.nshots).astype(np.float32)
    for s in range(off.nshots):       # the cell after an off-grid point stays inside
        x0, wn = off.window(s, g0)
        r0, r1 = off.rec_ptr[s], off.rec_ptr[s + 1]
        fx[r0:r1][off.rec_x[r0:r1] >= x0 + wn - 1] = 0.0
        if off.src_x[s] >= x0 + wn - 1:
            sfx[s] = 0.0
        if off.src_z[s] >= g0.nz - 1:
            sfz[s] = 0.0
    fz[off.rec_z >= g0.nz - 1] = 0.0
    off.rec_fz, off.rec_fx, off.src_fz, off.src_fx = fz, fx, sfz, sfx
    cases = {"off_grid": (g0, off), "free_surface": (replace(g0, free_surface=True), a0),
             "relative": (replace(g0, relative=True), a0), "pml": (replace(g0, pml=True), a0)}
    stream = torch.cuda.current_stream()
    out = {}
    for name, (g, a) in cases.items():
        d_obs = ctx.fwi_forward(g, a, v_true)
        ctx.gradient_pair(g, a, v0, d_obs, scale=-1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            ctx.gradient_pair(g, a, v0, d_obs, scale=-1.0)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = ctx.stats()
        out[name] = {"ms_per_step": ms, "vs_default_step": ms / base_ms,
                     "tiles_cols_rows_levels_prefetch": {k: [st["tile_cw"][i], st["tile_rows"][i],
                                                             st["tile_levels"][i], st["tile_prefetch"][i]]
                                                         for i, k in enumerate(("fwd", "adj", "born", "scat"))}}
    return out


def timed_steps(call, steps: int, stream) -> list[float]:
    """ms of each of `steps` calls, from HIP events recorded on `stream`
    between consecutive calls."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        call()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]


def checkpointed(wl, v0, d_obs, budget_gb: float, steps: int, base_ms: float) -> dict:
    """The timed step with checkpointed wavefields: the same fused gradient +
    pair call in a context whose memory budget is far below the step's
    164 GB imaging history, so each adjoint sweep recomputes segments of the
    history from snapshots of (u^{n-1}, u^n) and the pair runs its own joint
    Born sweep (background and scattered field) instead of reusing the
    forward's history. Two schedules: the one the budget gives (uniform
    checkpoints when they fit) and a binomial one with the snapshot count
    capped at 4. Per schedule: one untimed step, then `steps` timed ones."""
    import numpy as np
    import torch
    from paper_2403_17518_amd import ops
    from synth.problem import cell_updates
    grid, acq = wl.grid, wl.acq
    useful = 4 * cell_updates(grid, acq)
    ctx = ops.FwiContext(0)
    out = {"memory_budget_GB": budget_gb}
    try:
        ctx.set_mem_budget(int(budget_gb * 2**30))
        stream = torch.cuda.current_stream()
        for name, slots in (("budget", -1), ("binomial_4_snapshots", 4)):
            ctx.set_ckpt_slots(slots)
            ctx.gradient_pair(grid, acq, v0, d_obs, scale=-1.0)
            ms = timed_steps(lambda: ctx.gradient_pair(grid, acq, v0, d_obs, scale=-1.0), steps, stream)
            st = ctx.stats()
            med = float(np.median(ms))
            out[name] = {"ms_per_step": med, "ms_steps": ms, "vs_stored_history_step": med / base_ms,
                         "segments": st["n_segments"], "ckpt_every": st["ckpt_every"],
                         "snapshots": st["ckpt_slots"], "recomputed_steps": st["recomputed_steps"],
                         "executed_cell_updates_per_step": st["cell_updates"],
                         "useful_cell_updates_per_step": useful,
                         "useful_cell_updates_per_s": useful / (med * 1e-3)}
        return out
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def fwi_time_to_error() -> dict:
    """Plain gradient against network-preconditioned FWI on the 848 x 176
    salt workload (100 shots of uneven aperture and record length, bands 3 /
    8 / 15 Hz, 20 iterations each, the driver's default options): the
    iterations, solves and wall time (gradient, pair, training, line search)
    the network method needs to reach the plain method's final model error."""
    import numpy as np
    import torch
    from paper_2403_17518_amd import fwi_driver as D
    from paper_2403_17518_amd import ops
    from paper_2403_17518_amd.deblur import DeblurConfig
    from synth import configs
    wl = configs.salt_848x176(100)
    grid, acq = wl.grid, wl.acq
    fctx = ops.FwiContext(0)
    try:
        v_true = torch.from_numpy(wl.v_true.astype(np.float32)).cuda()
        H, W = D.net_grid(grid.nz, grid.nx, 3)
        res = {}
        for method in ("plain", "net"):
            target = res["plain"][-1]["model_error"] if method == "net" else None
            opts = D.FwiOptions(method=method, net=DeblurConfig(3, 32, 0.0, H, W), target_error=target)
            run = D.FwiRun(fctx, grid, acq, wl.v0, opts, v_true=wl.v_true, log=lambda line: None)
            res[method] = run.run(lambda a: fctx.fwi_forward(grid, a, v_true))
            if run.net is not None:
                run.net.close()
        out = {"workload": "salt_848x176: 100 shots, 176 x 848 cells of 20 m, records 3-5 s at 2 ms, "
                           "bands 3/8/15 Hz x 20 iterations, network widths 32-256"}
        out.update(D.time_to_error(res["plain"], res["net"]))
        out["plain_final_ssim"] = res["plain"][-1]["ssim"]
        return out
    finally:
        fctx.close()
        torch.cuda.empty_cache()


def deblur_flops(H: int, W: int, depth: int = 3, base: int = 32) -> float:
    """Flops (2 per multiply-add) of one forward pass of the deblurring UNet on
    an H x W image: 3x3 convolutions at every level, 2x2 stride-2 transposed
    convolutions, the 1x1 output convolution."""
    C = [base << l for l in range(depth + 1)]
    hw = lambda l: (H >> l) * (W >> l)
    f = 2 * hw(0) * 9 * (C[0] * 1 + C[0] * C[0]) + 2 * hw(0) * C[0]
    for l in range(1, depth + 1):
        f += 2 * hw(l) * 9 * (C[l] * C[l - 1] + C[l] * C[l])
    for l in range(depth):
        f += 2 * hw(l) * (C[l + 1] * C[l] + 9 * (C[l] * 2 * C[l] + C[l] * C[l]))
    return float(f)


def deblur_timing(train_steps: int = 40, applies: int = 10, depth: int = 3, base: int = 32,
                  slope: float = 0.0) -> dict:
    """Training (Adam steps) and inference of the deblurring network at the
    208 x 608 size of the 600 x 200 workload; a training step is counted as
    three forward passes (forward, data gradient, weight gradient)."""
    import torch
    from paper_2403_17518_amd import ops
    from paper_2403_17518_amd.deblur import DeblurConfig, DeblurNet
    ctx = ops.FwiContext(0)
    net = DeblurNet(ctx, DeblurConfig(depth, base, slope, 208, 608))
    try:
        g = torch.Generator(device="cuda").manual_seed(2403)
        x = torch.randn(200, 600, device="cuda", generator=g)
        y = torch.randn(200, 600, device="cuda", generator=g)
        net.deblur_train(x, y, 3, 1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.deblur_train(x, y, train_steps, 1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(applies):
            net.deblur_apply(x)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd = deblur_flops(208, 608, depth, base)
        tr = (t1 - t0) / train_steps
        ap = (t2 - t1) / applies
        widths = "-".join(str(base << l) for l in range(depth + 1))
        act = f"LeakyReLU {slope}" if slope else "ReLU"
        out = {"workload": f"UNet depth {depth}, widths {widths}, {act}, 208 x 608, bf16 MFMA, FP32 accumulation",
               "train_ms_per_step": tr * 1e3, "train_TFLOPs": 3 * fwd / tr / 1e12,
               "apply_ms": ap * 1e3, "apply_TFLOPs": fwd / ap / 1e12, "forward_GFLOP": fwd / 1e9,
               "peak_TFLOPs": BF16_PEAK_TFLOPS}
        out["train_frac"] = out["train_TFLOPs"] / BF16_PEAK_TFLOPS
        # per-layer GEMM timing over 3 training steps (events around each launch)
        net.set_profiling(True)
        net.deblur_train(x, y, 3, 1e-3)
        recs = net.layer_stats()
        net.set_profiling(False)
        out["layers"] = [[r["name"], r["pass"], r["M"], r["N"], r["K"],
                          round(r["flops"] / (r["ms"] * 1e-3) / 1e12, 1)] for r in recs]
        out["layers_fields"] = ["layer", "pass", "M", "N", "K", "TFLOP/s"]
        print(f"train {train_steps} steps: {tr * 1e3:.2f} ms/step, {out['train_TFLOPs']:.1f} TFLOP/s; "
              f"apply {ap * 1e3:.2f} ms, {out['apply_TFLOPs']:.1f} TFLOP/s", file=sys.stderr, flush=True)
        return out
    finally:
        net.close()
        ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the propagation path runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.deblur_only:
        print(json.dumps(deblur_timing(train_steps=100)), flush=True)
        return
    if args.deblur_paper_only:
        print(json.dumps(deblur_timing(train_steps=10, applies=5, depth=4, base=128, slope=0.2)), flush=True)
        return
    if args.spill_only:
        print(json.dumps(spill_probe(args.spill_nt)), flush=True)
        return
    import numpy as np
    import torch
    from paper_2403_17518_amd import ops
    from synth import configs
    from synth.problem import cell_updates

    spill = None if args.no_spill_probe else spill_probe(args.spill_nt)

    wl = configs.layered_600x200(nshots=args.shots, nt=args.nt)
    grid, acq = wl.grid, wl.acq
    acq.wavelet = acq.wavelet.astype(np.float32)
    dev = torch.device("cuda", 0)
    ctx = ops.FwiContext(0)
    if args.mem_budget_gb > 0:
        ctx.set_mem_budget(int(args.mem_budget_gb * 2**30))
    if args.tiling:
        t = [int(x) for x in args.tiling.split(",")] + [0]
        ctx.set_tiling(0, t[0], t[1], t[2], t[3])
        ctx.set_tiling(1, t[0], t[1], t[2], t[3])
    v_true = torch.from_numpy(wl.v_true.astype(np.float32)).to(dev)
    v0 = torch.from_numpy(wl.v0.astype(np.float32)).to(dev)
    d_obs = ctx.fwi_forward(grid, acq, v_true)        # synthetic observed data
    torch.cuda.synchronize()

    acc = {}

    st_last = {}

    def add_stats():
        s = ctx.stats()
        st_last.update(s)
        for k in ("cell_updates", "ms_fwd", "ms_adj", "ms_born", "n_fwd", "n_adj", "n_born",
                  "bytes_fwd", "bytes_adj", "bytes_born"):
            acc[k] = acc.get(k, 0.0) + s[k]
        acc["n_segments"] = s["n_segments"] or acc.get("n_segments", 0)
        acc["ckpt_every"] = s["ckpt_every"] or acc.get("ckpt_every", 0)

    def step(record):
        g, phi, dm1 = ctx.gradient_pair(grid, acq, v0, d_obs, scale=-1.0)
        if record:
            add_stats()
        return dm1

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_steps = timed_steps(lambda: step(True), args.steps, stream)
    wall = time.perf_counter() - t0
    ms = float(np.median(ms_steps))
    ctx.set_profiling(False)

    useful = 4 * cell_updates(grid, acq)          # fwd, adj, scattered field, adj
    value = useful / (ms * 1e-3)
    # the adjoint re-touches two field levels, the image accumulator and the
    # model every step (the D^n history streams through once)
    f_bytes = 4 * grid.NZ * sum(acq.window(s, grid)[1] + 2 * grid.nb for s in range(acq.nshots))
    working_set = 3 * f_bytes + 4 * grid.nz * grid.nx
    # dominant kernel by time, its algorithmic bytes per launch / average duration
    kinds = {"stencil_fwd": ("ms_fwd", "n_fwd", "bytes_fwd"),
             "stencil_adj": ("ms_adj", "n_adj", "bytes_adj"),
             "stencil_born": ("ms_born", "n_born", "bytes_born")}
    dom = max(kinds, key=lambda k: acc.get(kinds[k][0], 0.0))
    kms, kn, kb = (acc[x] for x in kinds[dom])
    achieved_own = (kb / kn) / ((kms / kn) * 1e-3) / 1e9
    st = st_last
    # the step's Born-class time is the scattered-field pass (tiling class 3)
    cls = {"stencil_fwd": 0, "stencil_adj": 1, "stencil_born": 3}[dom]
    tkey = f"{st['tile_cw'][cls]},{st['tile_rows'][cls]},{st['tile_levels'][cls]},{st['tile_prefetch'][cls]}"
    table, own = bytes_per_update({"stencil_fwd": "fwd", "stencil_adj": "adj", "stencil_born": "born"}[dom],
                                  st["tile_levels"][cls] or 1)
    achieved = achieved_own * table / own
    traffic = None
    if MEASURED_TRAFFIC["kernels_sha1"] == kernels_sha1():
        traffic = MEASURED_TRAFFIC.get(dom, {}).get(tkey)
    out = {
        "metric": "FD cell-updates/s & % HBM roofline; FWI iters+time to model error vs plain",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"layered_600x200: FWI gradient + Born demigration/migration pair (4 field passes), {acq.nshots} shots, "
                        f"{grid.nt_max} steps, padded 240x640, 600 receivers",
            "global_batch": acq.nshots,
            "seq_len": grid.nt_max,
            "parallelism": "single GPU, all shots per launch",
            "checkpoint_segments": acc.get("n_segments", 0),
            "executed_cell_updates_per_step": acc["cell_updates"] / args.steps,
            "useful_cell_updates_per_step": useful,
            "wall_s": wall,
            "tiles_cols_rows_levels_prefetch": {k: [st_last["tile_cw"][i], st_last["tile_rows"][i],
                                                    st_last["tile_levels"][i], st_last["tile_prefetch"][i]]
                                                for i, k in enumerate(("fwd", "adj", "born", "scat"))},
        },
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "bytes_per_update": table if dom != "stencil_born" else 24.0,
            # the same launches against the kernel's own minimal traffic
            "min_traffic": {"achieved": achieved_own, "frac": achieved_own / HBM_PEAK_GBS,
                            "bytes_per_update": own if dom != "stencil_born" else 24.0},
            # the timed workload's re-touched working set fits in the 256 MB
            # last-level cache, so its fraction is cache-assisted; the
            # HBM-bound fractions of the same kernel classes come from the
            # full-width salt grid (spill_probe)
            "cache_assisted": working_set < 256e6, "working_set_MB": working_set / 1e6,
            "hbm_bound": None,
            "traffic": traffic,
            "avg_launch_us": kms / kn * 1e3, "launches": int(kn),
            "bytes_per_launch": kb / kn * table / own,
            "kernel_ms": {k: acc[v[0]] / args.steps for k, v in kinds.items()},
        },
    }
    out["ms_steps"] = ms_steps
    if spill is not None:
        cls = {"stencil_fwd": "fwd", "stencil_adj": "adj", "stencil_born": "born"}[dom]
        hb = {"workload": spill["workload"], "kernel_class": cls}
        for mode in ("one_level", "autotuned"):
            r = spill.get(mode, {}).get(cls)
            if r:
                hb[mode] = {"frac": r["frac"], "achieved_GBs": r["achieved_GBs"],
                            "frac_min_traffic": r["min_traffic"]["frac"],
                            "tiling_cols_rows_levels_prefetch": r["tiling_cols_rows_levels_prefetch"]}
        out["roofline"]["hbm_bound"] = hb
    if not args.no_checkpointed:
        out["checkpointed"] = checkpointed(wl, v0, d_obs, args.ckpt_budget_gb, 2, ms)
    if not args.no_variants:
        try:
            out["variants"] = variants(ctx, wl, v_true, v0, args.variant_steps, ms)
        except Exception as e:   # reported in the line; the headline figures stand
            out["variants"] = {"error": repr(e)}
    if spill is not None:
        out["spill_probe"] = spill
    if not args.no_deblur:
        out["deblur"] = deblur_timing()
        out["deblur_paper_scale"] = deblur_timing(train_steps=10, applies=5, depth=4, base=128, slope=0.2)
    if not args.no_fwi:
        out["fwi_time_to_error"] = fwi_time_to_error()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
