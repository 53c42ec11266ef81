"""Particle update on the GPU (ripple_particles_update) against the FP64
oracle, through the C ABI.

Tolerance.  The device forms x + v dt with one fused multiply-add in its
working precision, on the stored (rounded) inputs and dt rounded to that
precision; the oracle adds the FP64 product to x.  For FP32 the FP64
oracle's result rounded to FP32 is the correctly rounded value, so the
device is within half an FP32 ulp of the oracle; for FP64 the two differ by
the oracle's extra rounding of the product.  The tests allow one ulp of the
result in the working precision plus one FP64 ulp of the product v dt.
"""
import numpy as np
import pytest
import torch

import gpu_util as G
from oracle import particles as O
from paper_2104_08571_amd import ripple_fv as R

pytestmark = pytest.mark.gpu

LAYOUTS = [(R.SOA, 0), (R.AOS, 0), (R.AOSOA, 16), (R.AOSOA, 32), (R.AOSOA, 64)]
LAYOUT_IDS = ["soa", "aos", "aosoa16", "aosoa32", "aosoa64"]


def state(n, seed):
    rng = np.random.default_rng(seed)
    P = np.empty((6, n))
    P[:3] = rng.uniform(-1.0, 1.0, (3, n))
    P[3:] = rng.uniform(-2.0, 2.0, (3, n))
    return P


def load(p, P):
    buf = torch.empty(p.bytes, dtype=torch.uint8, device="cuda")
    src = torch.as_tensor(P, dtype=torch.float64).to("cuda").contiguous()
    R.ripple_particles_import(G.ctx(), p, src.data_ptr(), buf.data_ptr(), G.stream())
    torch.cuda.synchronize()
    return buf


def export(p, buf):
    dst = torch.empty((6, p.n), dtype=torch.float64, device="cuda")
    R.ripple_particles_export(G.ctx(), p, buf.data_ptr(), dst.data_ptr(), G.stream())
    torch.cuda.synchronize()
    return dst.cpu().numpy()


def tol(ref, P, dt, dtype):
    r = np.abs(ref[:3]).astype(np.float32 if dtype == R.F32 else np.float64)
    return np.spacing(r).astype(np.float64) + np.spacing(np.abs(P[3:] * dt))


@pytest.mark.parametrize("stage", [0, 1], ids=["registers", "lds"])
@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("layout,w", LAYOUTS, ids=LAYOUT_IDS)
def test_parity(dtype, layout, w, stage):
    for n in (1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 4097, 100003):
        p = R.make_particles(n, dtype=dtype, layout=layout, aosoa_w=w, stage=stage)
        buf = load(p, state(n, n))
        P = export(p, buf)                      # the stored, rounded inputs
        dt = 1e-3 * (1 + n % 7)
        dt_w = float(np.float32(dt)) if dtype == R.F32 else dt
        R.ripple_particles_update(G.ctx(), p, buf.data_ptr(), dt, G.stream())
        got = export(p, buf)
        ref = O.update(P, dt_w)
        assert np.array_equal(got[3:], P[3:]), n            # velocities untouched
        assert (np.abs(got[:3] - ref[:3]) <= tol(ref, P, dt_w, dtype)).all(), (n, layout, w)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_layouts_and_blocks_bitwise_equal(dtype):
    n = 77777
    P = state(n, 1)
    ref = None
    for layout, w in LAYOUTS:
        for block, stage in ((0, 0), (64, 0), (1024, 0), (0, 1), (64, 1), (512, 1), (1024, 1)):
            p = R.make_particles(n, dtype=dtype, layout=layout, aosoa_w=w, block=block, stage=stage)
            buf = load(p, P)
            for _ in range(3):
                R.ripple_particles_update(G.ctx(), p, buf.data_ptr(), 0.01, G.stream())
            got = export(p, buf)
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (layout, w, block, stage)


@pytest.mark.parametrize("stage", [0, 1], ids=["registers", "lds"])
def test_zero_dt_and_padding_slots_untouched(stage):
    for dtype, view in ((R.F32, torch.int32), (R.F64, torch.int64)):
        for layout, w in LAYOUTS:
            n = 1000
            p = R.make_particles(n, dtype=dtype, layout=layout, aosoa_w=w, stage=stage)
            buf = torch.empty(p.bytes, dtype=torch.uint8, device="cuda")
            buf.view(view).fill_(-1)
            src = torch.as_tensor(state(n, 2), dtype=torch.float64).to("cuda").contiguous()
            R.ripple_particles_import(G.ctx(), p, src.data_ptr(), buf.data_ptr(), G.stream())
            before = buf.clone()
            R.ripple_particles_update(G.ctx(), p, buf.data_ptr(), 0.0, G.stream())
            torch.cuda.synchronize()
            assert torch.equal(buf, before)          # x + v * 0 = x, slots past n untouched
            R.ripple_particles_update(G.ctx(), p, buf.data_ptr(), 0.5, G.stream())
            torch.cuda.synchronize()
            assert int((buf.view(view) == -1).sum()) == 6 * (p.slots - n)


def test_rejected_arguments():
    p = R.make_particles(100, dtype=R.F32, layout=R.SOA)
    buf = load(p, state(100, 3))
    small = G.RawDeviceBuffer(p.bytes // 2)
    import ctypes
    assert R.call("ripple_particles_update", G.ctx(), ctypes.byref(p), buf.data_ptr(),
                  float("nan"), G.stream()) == R.E_INVALID
    assert R.call("ripple_particles_update", G.ctx(), ctypes.byref(p), small.data_ptr(), 0.1,
                  G.stream()) == R.E_INVALID
    small.free()
    stale = R.make_particles(100)
    stale.slots = 96
    assert R.call("ripple_particles_update", G.ctx(), ctypes.byref(stale), buf.data_ptr(), 0.1,
                  G.stream()) == R.E_INVALID


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_full_size_80M(dtype):
    """80 million particles (the paper's largest size), SoA and AoS, through
    registers and staged through LDS, every particle against the oracle."""
    n = 80_000_000
    rng = torch.Generator(device="cuda").manual_seed(4)
    src = torch.rand((6, n), dtype=torch.float64, device="cuda", generator=rng) * 2 - 1
    for layout, stage in ((R.SOA, 0), (R.AOS, 0), (R.SOA, 1), (R.AOS, 1)):
        p = R.make_particles(n, dtype=dtype, layout=layout, stage=stage)
        buf = torch.empty(p.bytes, dtype=torch.uint8, device="cuda")
        R.ripple_particles_import(G.ctx(), p, src.data_ptr(), buf.data_ptr(), G.stream())
        P = export(p, buf)
        R.ripple_particles_update(G.ctx(), p, buf.data_ptr(), 0.002, G.stream())
        got = export(p, buf)
        dt_w = float(np.float32(0.002)) if dtype == R.F32 else 0.002
        ref = O.update(P, dt_w)
        assert np.array_equal(got[3:], P[3:])
        assert (np.abs(got[:3] - ref[:3]) <= tol(ref, P, dt_w, dtype)).all(), (layout, stage)
        del buf
        torch.cuda.empty_cache()
