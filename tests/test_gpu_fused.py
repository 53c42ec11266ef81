"""The fused x-then-y sweep gives bitwise the states of the separate x and y
sweeps, in both of its forms (whole rows per workgroup exchanging through
LDS, split_xy = 2; strips of 60 cells per wave exchanging by lane shifts,
split_xy = 3) and in the form the library picks (split_xy = 0), for every
layout, precision, boundary condition and row length, and for sub-blocks
linked along x and/or y (whose padding, corners included, the halo copies
fill before the pass); grids it does not accept (rows under 16 cells) fall
back to the separate sweeps with the same results.  Also checks the
in-place semantics of the step entry points on both paths."""
import numpy as np
import pytest
import torch

import gpu_util as G
from paper_2104_08571_amd import initial_states as ist
from paper_2104_08571_amd import ripple_fv as R

pytestmark = pytest.mark.gpu


def assert_forms_equal(shape, dtype, layout, aosoa_w, bc, nsteps, cols=0, seed=31, state=None):
    """Run the separate sweeps (split_xy = 1), the library's pick (0), the
    rows form (2) and the wave-strip form (3); all must agree bitwise."""
    W = state if state is not None else ist.smooth_periodic(shape, seed=seed)
    out = {}
    for split in (1, 0, 2, 3):
        g = R.make_grid(shape, dtype=dtype, layout=layout, aosoa_w=aosoa_w, bc=bc,
                        tiling=(0, 0, 0, 0, cols, split))
        (U,), (t,) = G.run(g, W, nsteps)
        out[split] = (U, t)
    Us, ts = out[1]
    for split in (0, 2, 3):
        U, t = out[split]
        assert t == ts, (shape, bc, split)
        assert np.array_equal(U, Us), (shape, bc, split)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("layout,w", [(R.SOA, 0), (R.AOS, 0), (R.AOSOA, 16), (R.AOSOA, 64)],
                         ids=["soa", "aos", "aosoa16", "aosoa64"])
@pytest.mark.parametrize("cols", [1, 2])
def test_fused_equals_split(dtype, layout, w, cols):
    for shape, bc in (((37, 29, 11), (1, 1, 1)), ((16, 24, 9), (0, 0, 1)), ((33, 20, 7), (0, 1, 0))):
        assert_forms_equal(shape, dtype, layout, w, bc, 3, cols)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("nx", [2, 3, 16, 17, 56, 57, 58, 59, 60, 61, 62, 119, 120, 121, 176, 192,
                                255, 300, 384, 385, 508, 509, 512, 513, 520, 1000, 1016, 1017, 1100])
def test_fused_row_lengths(dtype, nx):
    """Row lengths from 2 to 1100 cells: below, inside and above what one
    workgroup holds and around multiples of the 60-cell strip (fused where
    n0 >= 16, separate sweeps below 16), odd lengths; blast (transmissive)
    vs periodic faces; several z planes per tile."""
    shape = (nx, 9, 7)
    for bc in ((1, 1, 1), (0, 0, 0)):
        # the blast needs a few cells across it to stay physical
        state = ist.blast(shape) if bc[0] == 0 and nx >= 16 else None
        assert_forms_equal(shape, dtype, R.SOA, 0, bc, 2, 0, state=state)


def assert_partitions_match(shape, dtype, bc, seed, cases, nsteps=3):
    """Each (parts, split_xy) partition of the grid, run as linked sub-blocks,
    equals the whole grid bitwise."""
    whole = R.make_grid(shape, dtype=dtype, layout=R.SOA, bc=bc)
    W = ist.smooth_periodic(shape, seed=seed)
    (ref,), (t_ref,) = G.run(whole, W, nsteps)
    for parts, split in cases:
        subs = [R.copy_grid(sb, split_xy=split) for sb in R.ripple_fv_partition(whole, parts)]
        states, origins = [], []
        for idx, sb in enumerate(subs):
            a, b, c = idx % parts[0], (idx // parts[0]) % parts[1], idx // (parts[0] * parts[1])
            o = [k * (n // m) + min(k, n % m) for k, n, m in zip((a, b, c), shape, parts)]
            origins.append(o)
            states.append(ist.smooth_periodic(list(sb.n), seed, origin=o, n_global=shape))
        outs, ts = G.run(subs, states, nsteps)
        for sb, U, o, t in zip(subs, outs, origins, ts):
            assert t == t_ref
            part = ref[:, o[2]:o[2] + sb.n[2], o[1]:o[1] + sb.n[1], o[0]:o[0] + sb.n[0]]
            assert np.array_equal(U, part), (shape, parts, split, o)
    return whole


def test_linked_sub_blocks_match_whole_grid():
    """Sub-blocks linked along y, along x, and along both (so the fused pass
    reads corner padding), fused and split, match the whole grid bitwise; the
    single fused sweep entry point reports a linked grid unsupported."""
    shape = (40, 24, 10)   # sub-block rows of 20 or 40 cells: fused
    whole = assert_partitions_match(
        shape, R.F64, (1, 0, 1), 77,
        (((1, 2, 1), 0), ((2, 1, 1), 0), ((2, 2, 1), 0), ((2, 3, 2), 0), ((2, 2, 1), 1),
         ((1, 2, 1), 3), ((2, 1, 1), 3), ((2, 3, 2), 3), ((2, 2, 1), 2)))
    sub = R.ripple_fv_partition(whole, (1, 2, 1))[0]
    a, b = G.buffer(sub), G.buffer(sub)
    with pytest.raises(R.RippleFVError) as e:
        R.ripple_fv_sweep(G.ctx(), sub, R.AXIS_XY, a.data_ptr(), b.data_ptr(), 1e-3, G.stream())
    assert e.value.status == R.E_UNSUPPORTED


@pytest.mark.parametrize("shape,bc,cases", [
    # rows of 20 and 40 cells (several per workgroup, four ghost lanes each);
    # x periodic (both faces of every sub-block linked) and x transmissive
    # (the outer faces physical)
    ((40, 24, 10), (1, 0, 1), (((2, 1, 1), 0), ((2, 2, 1), 0), ((2, 3, 2), 0), ((2, 2, 1), 2))),
    ((40, 24, 10), (0, 1, 0), (((2, 1, 1), 0), ((2, 2, 2), 2), ((2, 1, 1), 3))),
    # rows of 384 cells (the 768^3 partition's sub-block rows): strips (0)
    # and rows of 388 lanes (2)
    ((768, 10, 6), (1, 1, 1), (((2, 1, 1), 0), ((2, 2, 1), 2))),
    ((768, 10, 6), (0, 0, 1), (((2, 1, 1), 0), ((2, 1, 1), 2))),
    # rows of 400 cells: rows of 404 lanes (2) and strips (0, 3)
    ((800, 10, 6), (1, 0, 1), (((2, 1, 1), 2), ((2, 1, 1), 0), ((2, 1, 1), 3))),
], ids=["r20p", "r20t", "r384p", "r384t", "r400"])
def test_linked_sub_blocks_f32_row_forms(shape, bc, cases):
    """FP32 sub-blocks linked along x in each form of the fused pass match
    the whole grid bitwise."""
    assert_partitions_match(shape, R.F32, bc, 91, cases)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("layout,w", [(R.SOA, 0), (R.AOS, 0), (R.AOSOA, 16)],
                         ids=["soa", "aos", "aosoa16"])
def test_shared_strip_tails(dtype, layout, w):
    """Wave strips whose short tails share one wave across three
    consecutive z rows: several groups of rows and a ragged last group, in
    every layout (the rows' cells then lie up to two planes apart within
    one wave)."""
    for shape, bc in (((61, 5, 25), (1, 0, 1)), ((64, 6, 13), (0, 1, 0)),
                      ((75, 4, 5), (1, 1, 1)), ((130, 5, 11), (0, 0, 1)), ((16, 3, 10), (1, 1, 0))):
        assert_forms_equal(shape, dtype, layout, w, bc, 2)


def test_shared_strip_tails_linked_sub_blocks():
    """Sub-blocks of 61 cells along x (tails of one cell, three rows to a
    wave) linked along x, in the strip form and the library's pick, match
    the whole grid bitwise."""
    assert_partitions_match((122, 8, 25), R.F64, (1, 0, 1), 5,
                            (((2, 1, 1), 3), ((2, 1, 1), 0), ((2, 2, 2), 3)))


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_wide_rows_linked_sub_blocks_match_whole_grid(dtype):
    """Rows longer than a workgroup (wave strips), on a whole grid and on
    sub-blocks whose linked x faces fall inside a strip or at its edge:
    bitwise the whole grid."""
    shape = (1100, 20, 6)
    whole = R.make_grid(shape, dtype=dtype, layout=R.SOA, bc=(1, 0, 1))
    W = ist.smooth_periodic(shape, seed=88)
    (ref,), (t_ref,) = G.run(whole, W, 3)
    split = R.copy_grid(whole, split_xy=1)
    (ref_s,), _ = G.run(split, W, 3)
    assert np.array_equal(ref, ref_s)
    for parts in ((2, 1, 1), (2, 2, 1), (3, 1, 2)):
        subs = R.ripple_fv_partition(whole, parts)
        states, origins = [], []
        for idx, sb in enumerate(subs):
            a, b, c = idx % parts[0], (idx // parts[0]) % parts[1], idx // (parts[0] * parts[1])
            o = [k * (n // m) + min(k, n % m) for k, n, m in zip((a, b, c), shape, parts)]
            origins.append(o)
            states.append(ist.smooth_periodic(list(sb.n), 88, origin=o, n_global=shape))
        outs, ts = G.run(subs, states, 3)
        for sb, U, o, t in zip(subs, outs, origins, ts):
            assert t == t_ref
            part = ref[:, o[2]:o[2] + sb.n[2], o[1]:o[1] + sb.n[1], o[0]:o[0] + sb.n[0]]
            assert np.array_equal(U, part), (parts, o)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_sweep_axis_xy_equals_x_then_y(dtype):
    shape = (48, 40, 13)
    W = ist.smooth_periodic(shape, seed=41)
    g = R.make_grid(shape, dtype=dtype, layout=R.SOA, bc=(1, 0, 1))
    dt = 2e-3
    a, b = G.load(g, W), G.buffer(g)
    R.ripple_fv_sweep(G.ctx(), g, R.AXIS_XY, a.data_ptr(), b.data_ptr(), dt, G.stream())
    fused = G.export(g, b)
    x, y, z = G.load(g, W), G.buffer(g), G.buffer(g)
    R.ripple_fv_sweep(G.ctx(), g, 0, x.data_ptr(), y.data_ptr(), dt, G.stream())
    R.ripple_fv_sweep(G.ctx(), g, 1, y.data_ptr(), z.data_ptr(), dt, G.stream())
    assert np.array_equal(fused, G.export(g, z))
    # the input is not modified
    assert np.array_equal(G.export(g, a), G.export(g, G.load(g, W)))


@pytest.mark.parametrize("split", [0, 1])
def test_step_is_in_place(split):
    """After 1, 2 and 3 steps the state is in the first buffer on both paths."""
    shape = (30, 26, 14)
    W = ist.smooth_periodic(shape, seed=51)
    g = R.make_grid(shape, dtype=R.F64, layout=R.SOA, bc=(1, 1, 1),
                    tiling=(0, 0, 0, 0, 0, split))
    ref = R.make_grid(shape, dtype=R.F64, layout=R.SOA, bc=(1, 1, 1),
                      tiling=(0, 0, 0, 0, 0, 1 - split))
    for n in (1, 2, 3):
        (U,), _ = G.run(g, W, n)
        (V,), _ = G.run(ref, W, n)
        assert np.array_equal(U, V), n
    a, b = G.load(g, W), G.buffer(g)
    R.ripple_fv_step(G.ctx(), g, a.data_ptr(), b.data_ptr(), 0.9, 0.0, None, G.stream())
    torch.cuda.synchronize()
    (U1,), _ = G.run(g, W, 1)
    assert np.array_equal(G.export(g, a), U1)


def test_fused_batch_graph_replays():
    """Uneven batch through the fused path: graph replays == eager == per grid."""
    ext = [(48, 32, 16), (160, 16, 32), (96, 80, 48), (17, 33, 9)]
    grids = [R.make_grid(e, dtype=R.F32, layout=R.SOA, bc=(1, 1, 1)) for e in ext]
    states = [ist.smooth_periodic(e, seed=60 + i) for i, e in enumerate(ext)]
    eager, te = G.run(grids, states, 4)
    for flags in (R.RUN_GRAPH, R.RUN_PER_GRID, R.RUN_GRAPH | R.RUN_PER_GRID, R.RUN_GRAPH):
        outs, ts = G.run(grids, states, 4, flags=flags)
        assert ts == te
        for x, y in zip(outs, eager):
            assert np.array_equal(x, y), flags
    split = [R.copy_grid(g, split_xy=1) for g in grids]
    outs, ts = G.run(split, states, 4)
    assert ts == te
    for x, y in zip(outs, eager):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("split", [0, 1])
def test_graph_step_counts(split):
    """Graph replays of step loops of any length (one graph of up to 64 steps
    repeated, plus a remainder graph; cached by step count and launch mode)
    equal the eager loop, on both the fused and the separate-sweep path."""
    ext = [(24, 20, 16), (17, 30, 12)]
    grids = [R.make_grid(e, dtype=R.F32, layout=R.SOA, bc=(1, 1, 1),
                         tiling=(0, 0, 0, 0, 0, split)) for e in ext]
    states = [ist.smooth_periodic(e, seed=90 + i) for i, e in enumerate(ext)]
    for n in (1, 2, 3, 7, 67, 3):
        eager, te = G.run(grids, states, n)
        for flags in (R.RUN_GRAPH, R.RUN_GRAPH | R.RUN_PER_GRID):
            outs, ts = G.run(grids, states, n, flags=flags)
            assert ts == te, (n, flags)
            for x, y in zip(outs, eager):
                assert np.array_equal(x, y), (n, flags)
