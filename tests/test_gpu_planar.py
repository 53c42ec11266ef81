"""Grids one cell thick along an axis, and the two-dimensional split Euler
solver built on them (the paper's scaling application, section "Scaling
Performance": a Mach 3.81 shock hitting a low-density bubble, 6400 x 4000
and 9600 x 6000 cells).

A sweep along a one-cell axis reads the same state on both faces of every
cell and changes nothing, so a grid with n[2] = 1 is a 2D problem; with
dx[2] large the z wave speed never sets dt, which then equals the 2D
solver's dt = CFL min(dx / S_x, dy / S_y).  The library skips the z sweep
on such grids and runs the x and y sweeps as one pass (wave strips) that
also reduces the next step's wave speeds, so the buffers alternate from
step to step; with split_xy = 1 the sweeps run separately and the y sweep
reduces the wave speeds.  Parity is against the FP64 oracle, which runs the
full three-sweep step.
"""
import numpy as np
import pytest
import torch

import gpu_util as G
from paper_2104_08571_amd import initial_states as ist
from paper_2104_08571_amd import ripple_fv as R

pytestmark = pytest.mark.gpu

TOL = {R.F32: 1e-5, R.F64: 1e-12}


def assert_parity_momentum_scaled(gpu, ref, tol, what):
    """Relative L1 and Linf per variable, with the three momenta measured against the
    total momentum sum(|m_x| + |m_y| + |m_z|): early in the shock-bubble run
    m_y is zero in exact arithmetic, and so in the oracle, while rounding
    leaves ulp-level values on the device (an FP64 contact is stationary only
    up to the rounding of S * (1 / S) in HLLC's star state)."""
    assert np.isfinite(gpu).all(), what
    mom = sum(np.abs(ref[c]).sum() for c in (1, 2, 3))
    for c in range(5):
        den = mom if c in (1, 2, 3) else np.abs(ref[c]).sum()
        err = np.abs(gpu[c] - ref[c]).sum() / den
        assert err <= tol, f"{what}: variable {c} relative L1 {err:.3e} exceeds {tol}"
    # elementwise, with the momenta scaled alike (gpu_util.rel_linf)
    inf = G.rel_linf(gpu, ref)
    assert (inf <= G.LINF_FACTOR * tol).all(), f"{what}: relative Linf {inf}"


def oracle_run(oracle, W, nsteps, dx, bc):
    U, t, _ = oracle.run(oracle.prim_to_cons(np.asarray(W)), nsteps, list(dx), list(bc))
    return U, t


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("shape,bc,split", [
    ((40, 24, 1), (1, 1, 1), 1), ((40, 24, 1), (1, 1, 1), 0), ((37, 29, 1), (0, 1, 0), 1),
    ((1, 30, 20), (0, 1, 1), 1), ((30, 1, 20), (1, 0, 1), 1), ((30, 1, 20), (1, 0, 1), 0),
    ((1, 1, 9), (0, 0, 1), 1), ((12, 20, 1), (1, 0, 1), 0), ((70, 9, 1), (0, 1, 0), 3)])
def test_one_cell_axes_match_oracle(oracle, dtype, shape, bc, split):
    W = ist.random_physical(shape, 12) if min(shape) == 1 and shape.count(1) > 1 else \
        ist.smooth_periodic(shape, seed=21)
    dx = [1.0 / max(n, 2) for n in shape]
    g = R.make_grid(shape, dtype=dtype, layout=R.SOA, bc=bc, dx=dx,
                    tiling=(0, 0, 0, 0, 0, split))
    (U,), (t,) = G.run(g, W, 5)
    ref, t_ref = oracle_run(oracle, W.numpy(), 5, dx, bc)
    G.assert_parity(U, ref, TOL[dtype], f"{shape} bc {bc} split {split}")
    assert abs(t - t_ref) <= (1e-6 if dtype == R.F32 else 1e-14) * t_ref


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_planar_equals_two_identical_planes(dtype):
    """A planar grid (one x-y pass per step, no z sweep, or separate x and y
    sweeps) and the same state on two identical periodic z planes (x-y pass
    and a z sweep that changes nothing) give the same bits in every plane,
    for 1, 2 and 5 steps: rows inside one workgroup and rows longer than
    one."""
    for nx, ny in ((48, 40), (1100, 12)):
        W1 = ist.smooth_periodic((nx, ny, 1), seed=33)
        W2 = torch.cat([W1, W1], dim=1)
        g2 = R.make_grid((nx, ny, 2), dtype=dtype, layout=R.SOA, bc=(1, 0, 1),
                         dx=(1.0 / nx, 1.0 / ny, 1.0))
        for split in (0, 1):
            g1 = R.make_grid((nx, ny, 1), dtype=dtype, layout=R.SOA, bc=(1, 0, 1),
                             dx=(1.0 / nx, 1.0 / ny, 1.0), tiling=(0, 0, 0, 0, 0, split))
            for n in (1, 2, 5):
                (a,), ta = G.run(g1, W1, n)
                (b,), tb = G.run(g2, W2, n, flags=R.RUN_GRAPH)
                assert ta == tb, (nx, split, n)
                assert np.array_equal(b[:, :1], a) and np.array_equal(b[:, 1:], a), (nx, split, n)


@pytest.mark.parametrize("split", [0, 1])
def test_planar_graph_step_counts(split):
    """Graph replays equal the eager loop for odd and even step counts (the
    one-pass planar step alternates buffers and copies back after odd
    counts; the separate sweeps return the state in place)."""
    shape = (600, 40, 1)   # rows longer than one workgroup
    W = ist.smooth_periodic(shape, seed=34)
    g = R.make_grid(shape, dtype=R.F32, layout=R.SOA, bc=(1, 1, 1),
                    tiling=(0, 0, 0, 0, 0, split))
    for n in (1, 3, 67, 2):
        (a,), ta = G.run(g, W, n)
        (b,), tb = G.run(g, W, n, flags=R.RUN_GRAPH)
        assert ta == tb and np.array_equal(a, b), n
    a_, b_ = G.load(g, W), G.buffer(g)
    R.ripple_fv_step(G.ctx(), g, a_.data_ptr(), b_.data_ptr(), 0.9, 0.0, None, G.stream())
    (one,), _ = G.run(g, W, 1)
    assert np.array_equal(G.export(g, a_), one)      # ripple_fv_step leaves the state in u


@pytest.mark.parametrize("split", [0, 1])
def test_planar_partition_matches_whole(split):
    shape = (64, 48, 1)
    whole = R.make_grid(shape, dtype=R.F64, layout=R.SOA, bc=(0, 1, 1),
                        tiling=(0, 0, 0, 0, 0, split))
    W = ist.smooth_periodic(shape, seed=35)
    (ref,), (t_ref,) = G.run(whole, W, 4)
    parts = (2, 2, 1)
    subs = R.ripple_fv_partition(whole, parts)
    states, origins = [], []
    for idx, sb in enumerate(subs):
        a, b = idx % 2, idx // 2
        o = [a * (shape[0] // 2), b * (shape[1] // 2), 0]
        origins.append(o)
        states.append(ist.smooth_periodic(list(sb.n), 35, origin=o, n_global=shape))
    outs, ts = G.run(subs, states, 4)
    for sb, U, o, t in zip(subs, outs, origins, ts):
        assert t == t_ref
        assert np.array_equal(U, ref[:, :, o[1]:o[1] + sb.n[1], o[0]:o[0] + sb.n[0]])


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_shock_bubble_small(oracle, dtype):
    nx, ny = 160, 100
    W = ist.shock_bubble(nx, ny)
    dx = (1.0 / ny, 1.0 / ny, 1.0)
    g = R.make_grid((nx, ny, 1), dtype=dtype, layout=R.SOA, bc=(0, 0, 0), dx=dx)
    (U,), (t,) = G.run(g, W, 20)
    ref, t_ref = oracle_run(oracle, W.numpy(), 20, dx, (0, 0, 0))
    assert_parity_momentum_scaled(U, ref, TOL[dtype], "shock bubble 160 x 100")
    assert abs(t - t_ref) <= (1e-6 if dtype == R.F32 else 1e-14) * t_ref


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_shock_bubble_6400x4000(oracle, dtype):
    """The paper's small scaling problem at full size, 3 steps, against the
    oracle over every cell."""
    nx, ny, steps = 6400, 4000, 3
    W = ist.shock_bubble(nx, ny)
    dx = (1.0 / ny, 1.0 / ny, 1.0)
    g = R.make_grid((nx, ny, 1), dtype=dtype, layout=R.SOA, bc=(0, 0, 0), dx=dx)
    (U,), (t,) = G.run(g, W, steps, flags=R.RUN_GRAPH)
    ref, t_ref = oracle_run(oracle, W.numpy(), steps, dx, (0, 0, 0))
    assert_parity_momentum_scaled(U, ref, TOL[dtype], "shock bubble 6400 x 4000")
    assert abs(t - t_ref) <= (1e-6 if dtype == R.F32 else 1e-14) * t_ref
