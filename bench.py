"""Benchmark: Gcell-updates/s and achieved HBM GB/s of the split Euler step.

Workload: 512^3 cells, smooth periodic initial state (seeded Fourier fields),
FP32 storage and arithmetic (the headline), with the same run in FP64 for the
FP32-vs-FP64 comparison.  One step = wave speeds (fused into the previous
step's z sweep) -> dt -> x, y, z sweeps, i.e. one pass of the whole hot path.
State buffers are resident in HBM before timing starts.

Prints one JSON line.  `value` is Gcell-updates/s at FP32; `roofline` is the
dominant sweep kernel's algorithmic bytes per launch over its mean launch
duration, timed with HIP events around every launch inside the timed region;
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload on this host.  `force2d_flux_difference` reports the 2D FORCE
flux-difference benchmark (square grids of 1024^2 .. 32768^2 cells, FP32 and
FP64, strided and contiguous layouts), one computation per call;
`shock_bubble_2d` the 2D split Euler solver on the shock-bubble problem at
6400 x 4000 and 9600 x 6000 cells, 1000 steps; `particle_update` the 3D
particle update x += v dt (100 thousand to 80 million particles, FP32 and
FP64, strided, contiguous and blocked layouts).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Vector-ALU peak without packed FP32 (which this build does not use): 256 CUs
# x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The same for FP64.
PEAK_VALU_TFLOPS = 78.6
# Arithmetic of one cell update along one axis, counted from the formulas the
# kernels evaluate (add, sub, mul, min, max, median, reciprocal and square root
# 1 each, fused multiply-add 2): slopes and Hancock half step 88, HLLC face
# flux 74 (the star-state correction formed from g - 1), conservative update 15.
FLOPS_PER_CELL_AXIS = 177
CSRC = os.path.join(ROOT, "paper_2104_08571_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(f"{kernel}@{workload}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def run_gpu(n, dtype, layout, aosoa_w, steps, warmup, seed, tiling):
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream().cuda_stream
    g = R.make_grid((n, n, n), dtype=dtype, layout=layout, aosoa_w=aosoa_w,
                    bc=(R.PERIODIC,) * 3, tiling=tiling)
    a = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
    W = ist.smooth_periodic((n, n, n), seed=seed, device="cuda")
    R.ripple_fv_import(ctx, g, W.data_ptr(), R.PRIMITIVE, a.data_ptr(), stream)
    torch.cuda.synchronize()
    del W
    pa, pb = [a.data_ptr()], [b.data_ptr()]
    if warmup > 0:
        R.ripple_fv_run_batch(ctx, [g], pa, pb, warmup, 0.9, R.RUN_EAGER, stream)
    torch.cuda.synchronize()
    R.ripple_fv_profile(ctx)  # clear
    # timed region: eager launches with HIP events around each kernel
    t0 = time.perf_counter()
    R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_PROFILE, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = R.ripple_fv_profile(ctx)
    # same loop replayed as a captured hipGraph (captured by an untimed run
    # of the same step count)
    R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    status = R.ripple_fv_check(ctx)
    R.ripple_fv_destroy(ctx)
    del a, b
    torch.cuda.empty_cache()
    return {"seconds": t1 - t0, "graph_seconds": t3 - t2, "profile": prof, "status": status}


def run_batch_workload(steps, warmup):
    """64 grids with extents drawn from {32, 48, ..., 192} (FP32, periodic):
    layout and tiling chosen by the autotuner, then batched persistent
    launches replayed as hipGraphs vs one launch per grid per kernel."""
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream().cuda_stream
    ext = ist.batch_extents(64, seed=42)
    base = [R.make_grid(e, dtype=R.F32, layout=R.SOA, bc=(R.PERIODIC,) * 3) for e in ext]
    t0 = time.perf_counter()
    grids = R.ripple_fv_batch_tune(ctx, base, stream)
    tune_s = time.perf_counter() - t0
    a, b = [], []
    for i, (g, e) in enumerate(zip(grids, ext)):
        W = ist.smooth_periodic(e, seed=1000 + i, device="cuda")
        a.append(torch.empty(g.bytes, dtype=torch.uint8, device="cuda"))
        b.append(torch.empty(g.bytes, dtype=torch.uint8, device="cuda"))
        R.ripple_fv_import(ctx, g, W.data_ptr(), R.PRIMITIVE, a[-1].data_ptr(), stream)
    pa, pb = [x.data_ptr() for x in a], [x.data_ptr() for x in b]
    cells = sum(e[0] * e[1] * e[2] for e in ext)
    out = {"grids": 64, "cells": cells, "tune_seconds": round(tune_s, 2),
           "chosen": {"layout": ["aos", "soa", "aosoa"][grids[0].layout], "aosoa_w": grids[0].aosoa_w,
                      "x_block": grids[0].x_block, "yz_block": grids[0].yz_block,
                      "yz_segment": grids[0].yz_segment, "persist": grids[0].persist,
                      "yz_cols": grids[0].yz_cols, "split_xy": grids[0].split_xy}}
    for name, flags in (("batched_graph", R.RUN_GRAPH), ("batched_eager", R.RUN_EAGER),
                        ("per_grid", R.RUN_PER_GRID)):
        # warm-up of the same step count (captures the graph in graph mode)
        R.ripple_fv_run_batch(ctx, grids, pa, pb, steps if flags & R.RUN_GRAPH else warmup, 0.9,
                              flags, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.ripple_fv_run_batch(ctx, grids, pa, pb, steps, 0.9, flags, stream)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[name] = {"gcell_updates_per_s": round(cells * steps / secs / 1e9, 3),
                     "ms_per_step": round(secs / steps * 1e3, 4)}
    # per-kernel times of the batched launches (HIP events around each launch)
    R.ripple_fv_profile(ctx)
    R.ripple_fv_run_batch(ctx, grids, pa, pb, steps, 0.9, R.RUN_PROFILE, stream)
    torch.cuda.synchronize()
    out["kernel_ms"] = {k: round(ms / c, 4) for k, (ms, c) in R.ripple_fv_profile(ctx).items() if c}
    out["status"] = R.ripple_fv_check(ctx)
    R.ripple_fv_destroy(ctx)
    return out


def run_partition_workload(steps, warmup):
    """768^3 FP32 blast wave as 2 x 2 x 2 sub-blocks of 384^3 with on-device
    halo copies each sweep (one GPU's share of a partitioned run)."""
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream().cuda_stream
    n = (768, 768, 768)
    whole = R.make_grid(n, dtype=R.F32, layout=R.SOA)
    subs = R.ripple_fv_partition(whole, (2, 2, 2))
    a, b = [], []
    for i, s in enumerate(subs):
        o = ((i % 2) * 384, ((i // 2) % 2) * 384, (i // 4) * 384)
        W = ist.blast((384, 384, 384), origin=o, n_global=n, device="cuda")
        a.append(torch.empty(s.bytes, dtype=torch.uint8, device="cuda"))
        b.append(torch.empty(s.bytes, dtype=torch.uint8, device="cuda"))
        R.ripple_fv_import(ctx, s, W.data_ptr(), R.PRIMITIVE, a[-1].data_ptr(), stream)
        del W
    pa, pb = [x.data_ptr() for x in a], [x.data_ptr() for x in b]
    R.ripple_fv_run_batch(ctx, subs, pa, pb, warmup, 0.9, R.RUN_EAGER, stream)
    torch.cuda.synchronize()
    R.ripple_fv_profile(ctx)
    t0 = time.perf_counter()
    R.ripple_fv_run_batch(ctx, subs, pa, pb, steps, 0.9, R.RUN_PROFILE, stream)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    prof = R.ripple_fv_profile(ctx)
    cells = 768 ** 3
    out = {"cells": cells, "sub_blocks": 8, "gcell_updates_per_s": round(cells * steps / secs / 1e9, 3),
           "ms_per_step": round(secs / steps * 1e3, 4),
           "kernel_ms": {k: (round(ms / c, 4) if c else None) for k, (ms, c) in prof.items()},
           "halo_ms_per_step": round(prof["halo"][0] / steps, 4),
           "status": R.ripple_fv_check(ctx)}
    R.ripple_fv_destroy(ctx)
    del a, b
    torch.cuda.empty_cache()
    return out


def run_layout_workload(n, steps, warmup, layouts):
    """The 256^3 FP64 periodic smooth field (seed 2104) in each cell layout:
    `steps` steps replayed from hipGraphs with the state resident in HBM, and
    per-kernel times from a profiled eager run of a few steps.  Bytes per step
    are reported for the two passes the step makes (20 s per cell: x-y and z,
    each reading and writing the state once) and for three separate sweeps
    (30 s per cell, the accounting of a step that makes three passes)."""
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    lays = {"soa": (R.SOA, 0), "aos": (R.AOS, 0), "aosoa16": (R.AOSOA, 16),
            "aosoa32": (R.AOSOA, 32), "aosoa64": (R.AOSOA, 64)}
    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream().cuda_stream
    W = ist.smooth_periodic((n, n, n), seed=2104, device="cuda")
    cells = n ** 3
    rows = []
    try:
        for name in layouts:
            g = R.make_grid((n, n, n), dtype=R.F64, layout=lays[name][0], aosoa_w=lays[name][1],
                            bc=(R.PERIODIC,) * 3)
            a = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
            b = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
            pa, pb = [a.data_ptr()], [b.data_ptr()]
            R.ripple_fv_import(ctx, g, W.data_ptr(), R.PRIMITIVE, a.data_ptr(), stream)
            R.ripple_fv_run_batch(ctx, [g], pa, pb, warmup, 0.9, R.RUN_EAGER, stream)
            R.ripple_fv_profile(ctx)
            R.ripple_fv_run_batch(ctx, [g], pa, pb, 5, 0.9, R.RUN_PROFILE, stream)
            torch.cuda.synchronize()
            prof = R.ripple_fv_profile(ctx)
            R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)  # capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            row = {"layout": name, "steps": steps, "ms_per_step": round(secs / steps * 1e3, 4),
                   "gcell_updates_per_s": round(cells * steps / secs / 1e9, 3),
                   "GBps_two_passes": round(20 * 8 * cells * steps / secs / 1e9, 1),
                   "GBps_three_sweeps": round(30 * 8 * cells * steps / secs / 1e9, 1),
                   "kernel_ms": {k: round(ms / c, 4) for k, (ms, c) in prof.items() if c},
                   "status": R.ripple_fv_check(ctx)}
            rows.append(row)
            print(f"[bench] layouts 256^3 f64 {name}: {row}", file=sys.stderr, flush=True)
            del a, b
            torch.cuda.empty_cache()
    finally:
        R.ripple_fv_destroy(ctx)
    return {"workload": f"euler3d_smooth_periodic_{n}cubed_f64", "cells": cells, "results": rows}


def run_shock_bubble_workload(sizes, dtypes, steps, warmup):
    """The paper's 2D scaling application on one GPU: the split Euler solver
    (wave speeds -> dt -> x sweep -> y sweep per step) on a Mach 3.81 shock
    hitting a low-density bubble, transmissive faces, `steps` steps replayed
    from hipGraphs, state resident in HBM; per-sweep times from a separate
    profiled run of a few steps."""
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    try:
        for dt_name in dtypes:
            dtype = R.F32 if dt_name == "f32" else R.F64
            for nx, ny in sizes:
                g = R.make_grid((nx, ny, 1), dtype=dtype, layout=R.SOA, bc=(0, 0, 0),
                                dx=(1.0 / ny, 1.0 / ny, 1.0))
                W = ist.shock_bubble(nx, ny, device="cuda")
                a = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
                b = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
                pa, pb = [a.data_ptr()], [b.data_ptr()]

                def load():
                    R.ripple_fv_import(ctx, g, W.data_ptr(), R.PRIMITIVE, a.data_ptr(), stream)

                load()
                R.ripple_fv_run_batch(ctx, [g], pa, pb, warmup, 0.9, R.RUN_EAGER, stream)
                R.ripple_fv_profile(ctx)
                R.ripple_fv_run_batch(ctx, [g], pa, pb, 5, 0.9, R.RUN_PROFILE, stream)
                torch.cuda.synchronize()
                prof = R.ripple_fv_profile(ctx)
                # capture the graphs of this step count before timing
                load()
                R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)
                load()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                R.ripple_fv_run_batch(ctx, [g], pa, pb, steps, 0.9, R.RUN_GRAPH, stream)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
                t_end, _ = R.ripple_fv_batch_time(ctx, [g])
                cells = nx * ny
                row = {"nx": nx, "ny": ny, "dtype": dt_name, "steps": steps,
                       "seconds": round(secs, 4), "ms_per_step": round(secs / steps * 1e3, 4),
                       "gcell_updates_per_s": round(cells * steps / secs / 1e9, 3),
                       "t_reached": t_end[0],
                       "kernel_ms": {k: round(ms / c, 4) for k, (ms, c) in prof.items() if c},
                       "status": R.ripple_fv_check(ctx)}
                rows.append(row)
                print(f"[bench] shock bubble {dt_name} {nx}x{ny}: {row}", file=sys.stderr,
                      flush=True)
                del W, a, b
                torch.cuda.empty_cache()
    finally:
        R.ripple_fv_destroy(ctx)
    return {"workload": "shock_bubble_2d_mach3.81", "results": rows}


# The paper's particle-update table ("tab:particle_update", one V100, ms per
# update) for the strided and contiguous layouts -- context only.
PAPER_PARTICLE_MS = {"soa": {100_000: 0.0191, 1_000_000: 0.1036, 10_000_000: 0.8679,
                             20_000_000: 1.7146, 40_000_000: 3.4062, 80_000_000: 6.7914},
                     "aos": {100_000: 0.0259, 1_000_000: 0.1620, 10_000_000: 1.4472,
                             20_000_000: 2.8487, 40_000_000: 5.7184, 80_000_000: 11.452},
                     # shared-memory variants of the same table (strided, contiguous)
                     "soa_lds": {100_000: 0.0221, 1_000_000: 0.1343, 10_000_000: 1.1834,
                                 20_000_000: 2.3441, 40_000_000: 4.6741, 80_000_000: 9.3259},
                     "aos_lds": {100_000: 0.0379, 1_000_000: 0.2381, 10_000_000: 2.0507,
                                 20_000_000: 4.0743, 40_000_000: 8.1453, 80_000_000: 16.3081}}


def run_particle_workload(sizes, dtypes, layouts, reps, warmup):
    """Particle update x += v dt in place: mean and minimum time per update
    from HIP events around every call on the launching stream; 9 elements
    move per particle (6 read, 3 written)."""
    import torch

    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream()
    # name: (layout, aosoa_w, stage); "_lds": staged through LDS with direct
    # global-to-LDS loads
    lays = {"soa": (R.SOA, 0, 0), "aos": (R.AOS, 0, 0), "aosoa64": (R.AOSOA, 64, 0),
            "soa_lds": (R.SOA, 0, 1), "aos_lds": (R.AOS, 0, 1)}
    rows = []
    try:
        for dt_name in dtypes:
            dtype = R.F32 if dt_name == "f32" else R.F64
            s_bytes = 4 if dtype == R.F32 else 8
            for lay_name in layouts:
                for n in sizes:
                    p = R.make_particles(n, dtype=dtype, layout=lays[lay_name][0],
                                         aosoa_w=lays[lay_name][1], stage=lays[lay_name][2])
                    buf = torch.empty(p.bytes, dtype=torch.uint8, device="cuda")
                    gen = torch.Generator(device="cuda").manual_seed(n)
                    src = torch.rand((6, n), dtype=torch.float64, device="cuda", generator=gen)
                    R.ripple_particles_import(ctx, p, src.data_ptr(), buf.data_ptr(),
                                              stream.cuda_stream)
                    del src
                    for _ in range(warmup):
                        R.ripple_particles_update(ctx, p, buf.data_ptr(), 1e-3, stream.cuda_stream)
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
                    torch.cuda.synchronize()
                    ev[0].record(stream)
                    for k in range(reps):
                        R.ripple_particles_update(ctx, p, buf.data_ptr(), 1e-3, stream.cuda_stream)
                        ev[k + 1].record(stream)
                    torch.cuda.synchronize()
                    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
                    mean = sum(ms) / reps
                    row = {"n": n, "dtype": dt_name, "layout": lay_name, "ms": round(mean, 4),
                           "ms_min": round(min(ms), 4),
                           "GBps_algorithmic": round(9 * s_bytes * n / mean / 1e6, 1)}
                    if lay_name in PAPER_PARTICLE_MS and n in PAPER_PARTICLE_MS[lay_name]:
                        row["paper_v100_ms"] = PAPER_PARTICLE_MS[lay_name][n]
                    rows.append(row)
                    print(f"[bench] particles {dt_name} {lay_name} {n}: {row}", file=sys.stderr,
                          flush=True)
                    del buf
                    torch.cuda.empty_cache()
    finally:
        R.ripple_fv_destroy(ctx)
    out = {"workload": "particle_update_3d", "reps": reps, "results": rows}
    for r in rows:
        if r["layout"] == "soa" and r["n"] == max(sizes):
            key = f"particle_update_{r['n']}_{r['dtype']}_soa"
            out[f"roofline_{r['dtype']}"] = {
                "bound": "hbm", "kernel": "particles", "workload": key,
                "achieved": r["GBps_algorithmic"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(r["GBps_algorithmic"] / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("particles", key), "mean_launch_ms": r["ms"],
                "bytes_per_launch_algorithmic": 9 * (4 if r["dtype"] == "f32" else 8) * r["n"]}
    return out


# The paper's table of the 2D flux difference ("tab:flux", one V100, ms per
# computation) for the strided and contiguous layouts -- other hardware,
# reported as context only.
PAPER_FLUX_MS = {"soa": {1024: 0.0757, 2048: 0.2438, 4096: 0.9101, 8192: 3.5533,
                         16384: 14.282, 32768: 59.028},
                 "aos": {1024: 0.1065, 2048: 0.3614, 4096: 1.3971, 8192: 5.5284,
                         16384: 22.081, 32768: 86.756},
                 # strided layout in shared memory
                 "soa_lds": {1024: 0.0921, 2048: 0.2979, 4096: 1.1425, 8192: 4.4941,
                             16384: 18.090, 32768: 74.797}}
# Arithmetic of one cell of the 2D flux difference, counted like the sweeps'
# (each face flux is evaluated once and shared by its two cells): physical
# x and y fluxes of the cell 19, one x and one y FORCE face 2 x 62, the two
# differences and their sum 12.
FLOPS_PER_CELL_FORCE2D = 155


def run_force2d_workload(sizes, dtypes, layouts, reps, warmup):
    """2D FORCE flux difference (one computation = every cell's D) on square
    smooth periodic grids: mean and minimum time per computation from HIP
    events around every call on the launching stream, with the state
    resident in HBM."""
    import torch

    from paper_2104_08571_amd import initial_states as ist
    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    stream = torch.cuda.current_stream()
    # name: (layout, aosoa_w, stage); "_lds": rows staged through LDS with
    # direct global-to-LDS loads
    lays = {"soa": (R.SOA, 0, 0), "aos": (R.AOS, 0, 0), "aosoa64": (R.AOSOA, 64, 0),
            "soa_lds": (R.SOA, 0, 1), "aos_lds": (R.AOS, 0, 1)}
    lam = 0.25
    rows = []
    try:
        for dt_name in dtypes:
            dtype = R.F32 if dt_name == "f32" else R.F64
            s_bytes = 4 if dtype == R.F32 else 8
            for lay_name in layouts:
                for n in sizes:
                    g = R.make_force2d_grid((n, n), dtype=dtype, layout=lays[lay_name][0],
                                            aosoa_w=lays[lay_name][1], bc=(R.PERIODIC,) * 2,
                                            stage=lays[lay_name][2])
                    u = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
                    d = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
                    W = ist.smooth_periodic_2d((n, n), 2104, device="cuda")
                    R.ripple_force2d_import(ctx, g, W.data_ptr(), R.PRIMITIVE, u.data_ptr(),
                                            stream.cuda_stream)
                    torch.cuda.synchronize()
                    del W
                    for _ in range(warmup):
                        R.ripple_force2d_flux_difference(ctx, g, u.data_ptr(), lam, lam,
                                                         d.data_ptr(), stream.cuda_stream)
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
                    torch.cuda.synchronize()
                    ev[0].record(stream)
                    for k in range(reps):
                        R.ripple_force2d_flux_difference(ctx, g, u.data_ptr(), lam, lam,
                                                         d.data_ptr(), stream.cuda_stream)
                        ev[k + 1].record(stream)
                    torch.cuda.synchronize()
                    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
                    mean = sum(ms) / reps
                    cells = n * n
                    row = {"n": n, "dtype": dt_name, "layout": lay_name,
                           "ms": round(mean, 4), "ms_min": round(min(ms), 4),
                           "gcells_per_s": round(cells / mean / 1e6, 2),
                           "GBps_algorithmic": round(8 * s_bytes * cells / mean / 1e6, 1)}
                    if lay_name in PAPER_FLUX_MS and n in PAPER_FLUX_MS[lay_name]:
                        row["paper_v100_ms"] = PAPER_FLUX_MS[lay_name][n]
                    rows.append(row)
                    print(f"[bench] force2d {dt_name} {lay_name} {n}^2: {row}", file=sys.stderr,
                          flush=True)
                    del u, d
                    torch.cuda.empty_cache()
    finally:
        R.ripple_fv_destroy(ctx)
    out = {"workload": "flux_difference_2d_smooth_periodic", "lam": lam, "reps": reps,
           "results": rows}
    big = [r for r in rows if r["layout"] == "soa" and r["n"] == max(sizes)]
    for r in big:
        gbs = r["GBps_algorithmic"]
        key = f"flux_difference_2d_{r['n']}sq_{r['dtype']}_soa"
        out[f"roofline_{r['dtype']}"] = {
            "bound": "hbm", "kernel": "force2d", "workload": key, "achieved": gbs,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic("force2d", key), "mean_launch_ms": r["ms"],
            "bytes_per_launch_algorithmic": 8 * (4 if r["dtype"] == "f32" else 8) * r["n"] ** 2,
            "tflops_algorithmic": round(FLOPS_PER_CELL_FORCE2D * r["n"] ** 2 / r["ms"] / 1e9, 2)}
    return out


def copy_ceiling(nbytes=2 << 30, reps=20):
    """Device-to-device copy rate over `nbytes`-byte buffers, (read + write
    bytes) / time: the library's reference copy (16-byte accesses, default and
    non-temporal stores; median of `reps` copies timed one by one) and, for
    comparison, the runtime's blit copy that torch's copy_ uses.  It is the
    practical HBM ceiling the sweeps are compared with, and the known-size
    program against which rocprofv3's FETCH_SIZE / WRITE_SIZE counters are
    calibrated."""
    import torch

    from paper_2104_08571_amd import ripple_fv as R

    ctx = R.ripple_fv_create(0)
    st = torch.cuda.current_stream()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"bytes_per_copy": nbytes}
    try:
        for name, flags in (("stream_copy", 0), ("stream_copy_nontemporal", R.COPY_NONTEMPORAL)):
            for _ in range(3):
                R.ripple_fv_stream_copy(ctx, dst.data_ptr(), src.data_ptr(), nbytes, flags,
                                        st.cuda_stream)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            torch.cuda.synchronize()
            ev[0].record(st)
            for k in range(reps):
                R.ripple_fv_stream_copy(ctx, dst.data_ptr(), src.data_ptr(), nbytes, flags,
                                        st.cuda_stream)
                ev[k + 1].record(st)
            torch.cuda.synchronize()
            ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))[reps // 2]
            out[name] = {"ms_per_copy": round(ms, 4),
                         "GBps_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out["runtime_blit_copy"] = {"ms_per_copy": round(ms, 4),
                                    "GBps_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
    finally:
        R.ripple_fv_destroy(ctx)
        del src, dst
        torch.cuda.empty_cache()
    return out


def cpu_baseline(n, seed, steps):
    import numpy as np  # noqa: F401

    from oracle import Oracle
    from paper_2104_08571_amd import initial_states as ist

    o = Oracle()
    W = ist.smooth_periodic((n, n, n), seed=seed, device="cuda").cpu().numpy()
    U = o.prim_to_cons(W)
    del W
    t0 = time.perf_counter()
    o.run(U, steps, [1.0 / n] * 3, [1, 1, 1], cfl=0.9)
    t1 = time.perf_counter()
    cells = n ** 3
    return {"value": cells * steps / (t1 - t0) / 1e9, "unit": "Gcell-updates/s",
            "cores": o.num_threads(), "kind": "oracle",
            "sample": f"{steps} step(s) of the {n}^3 FP64 smooth periodic workload "
                      f"({t1 - t0:.1f} s on the host)"}


def roofline(m, traffic):
    """Roofline of the dominant kernel.  The fused x-y sweep does two sweeps'
    arithmetic per byte moved and is bound by vector-ALU issue, so it is
    reported against the ALU peak, with its HBM figures beside; a single
    sweep is reported against HBM."""
    hbm = {"achieved": round(m["dominant_achieved_GBps"], 1), "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": round(m["dominant_achieved_GBps"] / PEAK_HBM_GBS, 4),
           "traffic": traffic, "bytes_per_launch_algorithmic": m["bytes_per_launch"]}
    if m["dominant"] == "sweep_xy":
        out = {"bound": "alu", "kernel": m["dominant"], "achieved": round(m["dominant_tflops"], 2),
               "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
               "frac": round(m["dominant_tflops"] / PEAK_VALU_TFLOPS, 4), "traffic": traffic,
               "flops_per_launch_algorithmic": m["dominant_flops_per_launch"],
               "mean_launch_ms": round(m["dominant_ms"], 4), "hbm": hbm}
    else:
        out = {"bound": "hbm", "kernel": m["dominant"], **hbm,
               "mean_launch_ms": round(m["dominant_ms"], 4)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--layout", default="soa", choices=["soa", "aos", "aosoa16", "aosoa32", "aosoa64"])
    ap.add_argument("--tiling", default="0,0,0,0,0,0",
                    help="x_block,yz_block,yz_segment,persist,yz_cols,split_xy "
                         "(0 = library default; split_xy 1 = separate x and y sweeps, "
                         "2 / 3 = fused pass in the rows / wave-strip form)")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps timed for cpu_baseline (0 = skip); 3 steps of the "
                         "512^3 workload are about 12 s on 16 host threads")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and partitioned workloads and the 256^3 layout leg")
    ap.add_argument("--layouts", default="aos,soa,aosoa16,aosoa32,aosoa64",
                    help="cell layouts of the 256^3 FP64 leg (100 steps each)")
    ap.add_argument("--layout-steps", type=int, default=100)
    ap.add_argument("--layouts-only", action="store_true",
                    help="run only the 256^3 FP64 layout leg (prints its JSON)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-grid batch leg (prints its JSON)")
    ap.add_argument("--partition-only", action="store_true",
                    help="run only the 768^3 2x2x2 sub-block leg (prints its JSON)")
    ap.add_argument("--no-force2d", action="store_true",
                    help="skip the 2D FORCE flux-difference leg")
    ap.add_argument("--force2d-only", action="store_true",
                    help="run only the 2D FORCE flux-difference leg (prints its JSON)")
    ap.add_argument("--force2d-sizes", default="1024,2048,4096,8192,16384,32768")
    ap.add_argument("--force2d-layouts", default="soa,aos,soa_lds")
    ap.add_argument("--force2d-dtypes", default="f32,f64")
    ap.add_argument("--no-shock-bubble", action="store_true",
                    help="skip the 2D shock-bubble solver leg")
    ap.add_argument("--shock-bubble-only", action="store_true",
                    help="run only the 2D shock-bubble solver leg (prints its JSON)")
    ap.add_argument("--shock-bubble-steps", type=int, default=1000)
    ap.add_argument("--no-particles", action="store_true", help="skip the particle-update leg")
    ap.add_argument("--particles-sizes", default="100000,1000000,10000000,20000000,40000000,80000000")
    ap.add_argument("--particles-layouts", default="soa,aos,aosoa64,soa_lds,aos_lds")
    ap.add_argument("--particles-dtypes", default="f32,f64")
    ap.add_argument("--particles-only", action="store_true",
                    help="run only the particle-update leg (prints its JSON)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain-copy calibration (2 GiB, 20 copies) and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the partitioned path is measured as sub-blocks on one GPU)", file=sys.stderr)
        sys.exit(2)

    if args.copy_only:
        print(json.dumps({"copy_ceiling": copy_ceiling()}), flush=True)
        return
    f2_args = ([int(v) for v in args.force2d_sizes.split(",")], args.force2d_dtypes.split(","),
               args.force2d_layouts.split(","), max(args.steps, 5), args.warmup)
    sb_args = ([(6400, 4000), (9600, 6000)], ["f32", "f64"], args.shock_bubble_steps, args.warmup)
    pt_args = ([int(v) for v in args.particles_sizes.split(",")], args.particles_dtypes.split(","),
               args.particles_layouts.split(","), max(args.steps, 5), args.warmup)
    lay_args = (256, args.layout_steps, args.warmup, args.layouts.split(","))
    if args.partition_only:
        print(json.dumps({"partition_768_f32_2x2x2": run_partition_workload(args.steps, args.warmup)}),
              flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch_64_grids_f32": run_batch_workload(args.steps, args.warmup)}),
              flush=True)
        return
    if args.layouts_only:
        print(json.dumps({"layouts_256_f64": run_layout_workload(*lay_args)}), flush=True)
        return
    if args.particles_only:
        print(json.dumps({"particle_update": run_particle_workload(*pt_args)}), flush=True)
        return
    if args.shock_bubble_only:
        print(json.dumps({"shock_bubble_2d": run_shock_bubble_workload(*sb_args)}), flush=True)
        return
    if args.force2d_only:
        print(json.dumps({"force2d_flux_difference": run_force2d_workload(*f2_args)}), flush=True)
        return

    from paper_2104_08571_amd import ripple_fv as R

    lay = {"soa": (R.SOA, 0), "aos": (R.AOS, 0), "aosoa16": (R.AOSOA, 16),
           "aosoa32": (R.AOSOA, 32), "aosoa64": (R.AOSOA, 64)}[args.layout]
    tiling = tuple(int(v) for v in args.tiling.split(","))
    n = args.n
    cells = n ** 3
    seed = 8571
    workload = f"euler3d_smooth_periodic_{n}cubed"

    def measure(dtype, s_bytes):
        r = run_gpu(n, dtype, lay[0], lay[1], args.steps, args.warmup, seed, tiling)
        secs = r["seconds"]
        per_sweep = {k: (ms / cnt if cnt else None) for k, (ms, cnt) in r["profile"].items()}
        sweeps = {k: per_sweep[k] for k in ("sweep_x", "sweep_y", "sweep_z", "sweep_xy")
                  if per_sweep[k]}
        dom = max(sweeps, key=lambda k: r["profile"][k][0])
        bytes_per_launch = 10 * s_bytes * cells
        achieved = bytes_per_launch / (sweeps[dom] * 1e-3) / 1e9
        axes = 2 if dom == "sweep_xy" else 1
        tflops = FLOPS_PER_CELL_AXIS * axes * cells / (sweeps[dom] * 1e-3) / 1e12
        return {
            "gcell_updates_per_s": cells * args.steps / secs / 1e9,
            "ms_per_step": secs / args.steps * 1e3,
            "graph_ms_per_step": r["graph_seconds"] / args.steps * 1e3,
            "algorithmic_GBps_step": 30 * s_bytes * cells * args.steps / secs / 1e9,
            "kernel_ms": {k: round(v, 4) if v else v for k, v in per_sweep.items()},
            "dominant": dom, "dominant_ms": sweeps[dom], "dominant_achieved_GBps": achieved,
            "dominant_tflops": tflops, "dominant_flops_per_launch": FLOPS_PER_CELL_AXIS * axes * cells,
            "bytes_per_launch": bytes_per_launch, "status": r["status"],
        }

    f32 = measure(R.F32, 4)
    print(f"[bench] fp32 {n}^3: {f32['gcell_updates_per_s']:.2f} Gcell-updates/s, "
          f"{f32['ms_per_step']:.3f} ms/step, kernels {f32['kernel_ms']}", file=sys.stderr, flush=True)
    f64 = None
    if not args.no_f64:
        f64 = measure(R.F64, 8)
        print(f"[bench] fp64 {n}^3: {f64['gcell_updates_per_s']:.2f} Gcell-updates/s, "
              f"{f64['ms_per_step']:.3f} ms/step, kernels {f64['kernel_ms']}", file=sys.stderr,
              flush=True)

    ceiling = copy_ceiling()
    print(f"[bench] plain copy: {ceiling}", file=sys.stderr, flush=True)

    batch = part = lays = None
    if not args.no_extra:
        batch = run_batch_workload(args.steps, args.warmup)
        print(f"[bench] batch 64 grids: {batch}", file=sys.stderr, flush=True)
        part = run_partition_workload(args.steps, args.warmup)
        print(f"[bench] partition 768^3: {part}", file=sys.stderr, flush=True)
        lays = run_layout_workload(*lay_args)

    sb = None
    if not args.no_shock_bubble:
        sb = run_shock_bubble_workload(*sb_args)
    pt = None
    if not args.no_particles:
        pt = run_particle_workload(*pt_args)
    f2 = None
    if not args.no_force2d:
        f2 = run_force2d_workload(*f2_args)

    base = None
    if args.cpu_steps > 0:
        base = cpu_baseline(n, seed, args.cpu_steps)
        print(f"[bench] cpu oracle: {base['value']:.4f} Gcell-updates/s on {base['cores']} "
              "threads", file=sys.stderr, flush=True)

    traffic = measured_traffic(f32["dominant"], f"{workload}_f32_{args.layout}")
    out = {
        "metric": "Gcell-updates/s and achieved HBM GB/s, 512^3 Euler step, FP32 vs FP64",
        "value": round(f32["gcell_updates_per_s"], 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded smooth periodic Fourier fields)",
        "config": {"workload": workload, "cells": cells, "layout": args.layout,
                   "tiling": args.tiling, "cfl": 0.9, "boundary": "periodic",
                   "scheme": "split MUSCL-Hancock/minmod/HLLC, gamma 1.4"},
        "achieved_GBps_algorithmic": round(f32["algorithmic_GBps_step"], 1),
        "graph_ms_per_step": round(f32["graph_ms_per_step"], 4),
        "kernel_ms": f32["kernel_ms"],
        "roofline": roofline(f32, traffic),
        "cpu_baseline": base,
        "copy_ceiling": ceiling,
    }
    # the long per-size tables first, so that the end of the line (what a
    # log tail shows) holds the 3D results and the summary
    if f2 is not None:
        out["force2d_flux_difference"] = f2
    if pt is not None:
        out["particle_update"] = pt
    if sb is not None:
        out["shock_bubble_2d"] = sb
    if batch is not None:
        out["batch_64_grids_f32"] = batch
    if part is not None:
        out["partition_768_f32_2x2x2"] = part
    if lays is not None:
        out["layouts_256_f64"] = lays
    if f64 is not None:
        out["f64"] = {"value": round(f64["gcell_updates_per_s"], 4), "unit": "Gcell-updates/s",
                      "ms_per_step": round(f64["ms_per_step"], 4),
                      "graph_ms_per_step": round(f64["graph_ms_per_step"], 4),
                      "achieved_GBps_algorithmic": round(f64["algorithmic_GBps_step"], 1),
                      "kernel_ms": f64["kernel_ms"],
                      "roofline": roofline(f64, measured_traffic(
                          f64["dominant"], f"{workload}_f64_{args.layout}"))}
    summary = {
        f"f32_{n}": {"gcell_updates_per_s": round(f32["gcell_updates_per_s"], 2),
                     "ms_per_step": round(f32["ms_per_step"], 4),
                     "graph_ms_per_step": round(f32["graph_ms_per_step"], 4),
                     "GBps_two_passes": round(f32["algorithmic_GBps_step"] * 2 / 3, 1),
                     "kernel_ms": {k: v for k, v in f32["kernel_ms"].items() if v}},
    }
    if f64 is not None:
        summary[f"f64_{n}"] = {"gcell_updates_per_s": round(f64["gcell_updates_per_s"], 2),
                               "ms_per_step": round(f64["ms_per_step"], 4),
                               "GBps_two_passes": round(f64["algorithmic_GBps_step"] * 2 / 3, 1),
                               "kernel_ms": {k: v for k, v in f64["kernel_ms"].items() if v}}
    if batch is not None:
        summary["batch_64_grids_f32"] = {
            "graph": batch["batched_graph"]["gcell_updates_per_s"],
            "eager": batch["batched_eager"]["gcell_updates_per_s"],
            "per_grid": batch["per_grid"]["gcell_updates_per_s"], "chosen": batch["chosen"]}
    if part is not None:
        summary["partition_768_f32_2x2x2"] = {"gcell_updates_per_s": part["gcell_updates_per_s"],
                                              "halo_ms_per_step": part["halo_ms_per_step"]}
    if lays is not None:
        summary["layouts_256_f64_gcell_updates_per_s"] = {
            r["layout"]: r["gcell_updates_per_s"] for r in lays["results"]}
    out["summary"] = summary
    print("[bench] summary: " + json.dumps(summary), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
