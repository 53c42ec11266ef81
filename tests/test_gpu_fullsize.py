"""The workloads at their full sizes, in the launch configuration the
benchmark times (persistent tile lists, default tiling, eager or graph).

Where the FP64 oracle finishes in seconds on the host it is run on the whole
grid for the first steps.  For the full step counts the tests check
properties that hold at any size: conservation to round-off on periodic
grids (FP64 sums on the device), layout and launch-mode invariance, mirror
symmetry, partitioned == monolithic, and oracle parity on sampled grids of the
batch.
"""
import time

import numpy as np
import pytest
import torch

import gpu_util as G
from paper_2104_08571_amd import initial_states as ist
from paper_2104_08571_amd import ripple_fv as R

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[fullsize] {msg}", flush=True)


def sums(g, buf):
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    R.ripple_fv_conserved_sums(G.ctx(), g, buf.data_ptr(), out.data_ptr(), G.stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def abs_sums(U):
    return np.abs(U).reshape(5, -1).sum(1)


def run_keep(grids, states, nsteps, flags=R.RUN_EAGER):
    """Run and return the state buffers (the result, in place; no export)."""
    a = [G.load(g, W) for g, W in zip(grids, states)]
    b = [G.buffer(g) for g in grids]
    R.ripple_fv_run_batch(G.ctx(), grids, [x.data_ptr() for x in a], [x.data_ptr() for x in b],
                          nsteps, 0.9, flags, G.stream())
    torch.cuda.synchronize()
    assert R.ripple_fv_check(G.ctx()) == R.OK
    return a


@pytest.mark.parametrize("layout", [R.AOS, R.SOA], ids=["aos", "soa"])
def test_smooth_256_fp64(oracle, layout):
    """256^3 FP64 periodic smooth field: parity with the oracle over the
    first two steps on the full grid; 100 steps conserve all totals."""
    n = (256, 256, 256)
    W = ist.smooth_periodic(n, seed=2104, device="cuda")
    g = R.make_grid(n, dtype=R.F64, layout=layout, bc=(1, 1, 1))
    log(f"256^3 fp64 layout={layout}: oracle 2 steps")
    t0 = time.time()
    ref, t_ref, _ = oracle.run(oracle.prim_to_cons(W.cpu().numpy()), 2, G.unit_dx(n), [1, 1, 1])
    log(f"oracle done in {time.time() - t0:.1f} s")
    (gpu,), (t,) = G.run(g, W, 2)
    err = G.assert_parity(gpu, ref, 1e-12, "256^3 fp64 2 steps")
    assert abs(t - t_ref) <= 1e-13 * t_ref
    log(f"rel L1 after 2 steps {err}")
    del ref, gpu
    U0 = G.export(g, G.load(g, W))
    buf = run_keep([g], [W], 100)[0]
    s1 = sums(g, buf)
    drift = np.abs(s1 - U0.reshape(5, -1).sum(1)) / abs_sums(U0)
    log(f"100-step conservation drift {drift}")
    assert (drift < 1e-13).all(), drift


def test_smooth_256_layouts_agree_at_100_steps():
    n = (256, 256, 256)
    W = ist.smooth_periodic(n, seed=2104, device="cuda")
    outs = []
    for layout in (R.AOS, R.SOA):
        g = R.make_grid(n, dtype=R.F64, layout=layout, bc=(1, 1, 1))
        outs.append(G.export(g, run_keep([g], [W], 100)[0]))
    assert np.array_equal(outs[0], outs[1])


def test_smooth_512_fp32(oracle):
    """512^3 FP32 periodic (the benchmark's workload and launch shape): one
    step against the FP64 oracle on the whole grid; 50 steps keep the FP64
    totals to round-off of FP32 storage."""
    n = (512, 512, 512)
    W = ist.smooth_periodic(n, seed=8571, device="cuda")
    g = R.make_grid(n, dtype=R.F32, layout=R.SOA, bc=(1, 1, 1))
    log("512^3 fp32: oracle 1 step")
    t0 = time.time()
    ref, t_ref, _ = oracle.run(oracle.prim_to_cons(W.cpu().numpy()), 1, G.unit_dx(n), [1, 1, 1])
    log(f"oracle done in {time.time() - t0:.1f} s")
    (gpu,), (t,) = G.run(g, W, 1)
    err = G.assert_parity(gpu, ref, 1e-5, "512^3 fp32 1 step")
    assert abs(t - t_ref) <= 1e-6 * t_ref
    log(f"rel L1 after 1 step {err}")
    del ref, gpu
    U0 = G.export(g, G.load(g, W))
    buf = run_keep([g], [W], 50, flags=R.RUN_GRAPH)[0]
    s1 = sums(g, buf)
    drift = np.abs(s1 - U0.reshape(5, -1).sum(1)) / abs_sums(U0)
    log(f"50-step conservation drift (FP32 storage, FP64 sums) {drift}")
    assert (drift < 1e-8).all(), drift


def test_smooth_512_fp64(oracle):
    """512^3 FP64 periodic, the benchmark's FP64 comparison run (the fused
    pass in its wave-strip form): one step against the oracle on the whole
    grid; 20 steps keep the totals to FP64 round-off."""
    n = (512, 512, 512)
    W = ist.smooth_periodic(n, seed=8571, device="cuda")
    g = R.make_grid(n, dtype=R.F64, layout=R.SOA, bc=(1, 1, 1))
    log("512^3 fp64: oracle 1 step")
    t0 = time.time()
    ref, t_ref, _ = oracle.run(oracle.prim_to_cons(W.cpu().numpy()), 1, G.unit_dx(n), [1, 1, 1])
    log(f"oracle done in {time.time() - t0:.1f} s")
    (gpu,), (t,) = G.run(g, W, 1)
    err = G.assert_parity(gpu, ref, 1e-12, "512^3 fp64 1 step")
    assert abs(t - t_ref) <= 1e-14 * t_ref
    log(f"rel L1 after 1 step {err}")
    del ref, gpu
    U0 = G.export(g, G.load(g, W))
    buf = run_keep([g], [W], 20, flags=R.RUN_GRAPH)[0]
    s1 = sums(g, buf)
    drift = np.abs(s1 - U0.reshape(5, -1).sum(1)) / abs_sums(U0)
    log(f"20-step conservation drift (FP64) {drift}")
    assert (drift < 1e-13).all(), drift


def test_batch_64_grids(oracle):
    """64 grids with extents drawn from {32, 48, ..., 192}: batched graph
    replay == per-grid launches bitwise; three sampled grids match the oracle."""
    ext = ist.batch_extents(64, seed=42)
    grids = [R.make_grid(e, dtype=R.F32, layout=R.SOA, bc=(1, 1, 1)) for e in ext]
    states = [ist.smooth_periodic(e, seed=1000 + i, device="cuda") for i, e in enumerate(ext)]
    log(f"batch: {sum(e[0] * e[1] * e[2] for e in ext) / 1e6:.1f} M cells")
    batched, tb = G.run(grids, states, 2, flags=R.RUN_GRAPH)
    per_grid, tp = G.run(grids, states, 2, flags=R.RUN_PER_GRID)
    assert tb == tp
    for a, b in zip(batched, per_grid):
        assert np.array_equal(a, b)
    sizes = [e[0] * e[1] * e[2] for e in ext]
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes)), 17):
        ref, t_ref, _ = oracle.run(oracle.prim_to_cons(states[i].cpu().numpy()), 2,
                                   G.unit_dx(ext[i]), [1, 1, 1])
        G.assert_parity(batched[i], ref, 1e-5, f"batch grid {i} {ext[i]}")
        assert abs(tb[i] - t_ref) <= 1e-6 * t_ref
    del batched, per_grid
    bufs = run_keep(grids, states, 50, flags=R.RUN_GRAPH)
    for i in (0, 33):
        U0 = G.export(grids[i], G.load(grids[i], states[i]))
        drift = np.abs(sums(grids[i], bufs[i]) - U0.reshape(5, -1).sum(1)) / abs_sums(U0)
        assert (drift < 1e-8).all(), (i, drift)


def test_blast_192_fp64(oracle):
    """Blast wave at 192^3 in FP64 against the oracle (5 steps)."""
    n = (192, 192, 192)
    W = ist.blast(n, device="cuda")
    g = R.make_grid(n, dtype=R.F64, layout=R.SOA)
    ref, t_ref, _ = oracle.run(oracle.prim_to_cons(W.cpu().numpy()), 5, G.unit_dx(n), [0, 0, 0])
    (gpu,), (t,) = G.run(g, W, 5)
    err = G.assert_parity(gpu, ref, 1e-12, "blast 192^3")
    assert abs(t - t_ref) <= 1e-13 * t_ref
    log(f"blast 192^3 rel L1 {err}")


def test_partition_768_fp32():
    """768^3 FP32 blast as 2 x 2 x 2 sub-blocks of 384^3 with on-device halo
    copies == the monolithic 768^3 grid, bitwise; the result is mirror
    symmetric about the centre planes."""
    n = (768, 768, 768)
    whole = R.make_grid(n, dtype=R.F32, layout=R.SOA)
    subs = R.ripple_fv_partition(whole, (2, 2, 2))
    steps = 3
    log("768^3 monolithic")
    Wfull = ist.blast(n, device="cuda")
    mono = run_keep([whole], [Wfull], steps)[0]
    del Wfull
    torch.cuda.empty_cache()
    log("768^3 as 2x2x2 sub-blocks")
    origins = [((i % 2) * 384, ((i // 2) % 2) * 384, (i // 4) * 384) for i in range(8)]
    states = [ist.blast((384, 384, 384), origin=o, n_global=n, device="cuda") for o in origins]
    parts = run_keep(subs, states, steps)
    del states
    ref = G.export(whole, mono)
    for s, o, buf in zip(subs, origins, parts):
        U = G.export(s, buf)
        part = ref[:, o[2]:o[2] + 384, o[1]:o[1] + 384, o[0]:o[0] + 384]
        assert np.array_equal(U, part), o
    # mirror symmetry on bands through the centre (x and y mirrors on a band of
    # z planes, the z mirror on a band of y rows)
    scale = np.abs(ref[:, 380:388]).max(axis=(1, 2, 3), keepdims=True)
    band = ref[:, 372:396]
    for axis in (2, 3):
        M = np.flip(band, axis=axis).copy()
        M[4 - axis] *= -1
        assert (np.abs(M - band) <= 1e-5 * scale).all(), axis
    band = ref[:, :, 372:396]
    M = np.flip(band, axis=1).copy()
    M[3] *= -1
    assert (np.abs(M - band) <= 1e-5 * scale).all()
