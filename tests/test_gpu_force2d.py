"""2D FORCE flux difference on the GPU (ripple_force2d_flux_difference)
against the FP64 oracle, through the C ABI.

Tolerance.  Each face flux is a short chain of roundings (about ten
operations) over terms bounded by S_c = max|F_c| + max|G_c| + max|U_c| /
min(lam) per component; the flux difference adds two faces per axis.  The
absolute error is therefore bounded by a few tens of ulps of S_c: the tests
allow 1e-5 S_c in FP32 (about 170 ulps) and 1e-13 S_c in FP64 (about 450
ulps; FP64 reciprocals are refined hardware estimates, about an ulp).
Inputs the oracle sees are the stored values (FP32 states are first rounded
to FP32 by the import and read back), so both sides start from the same
numbers.  Cell-wise random states make every flux difference O(1), which
turns the normwise bound into a tight relative check; smooth fields cover
the paper's workload shape.
"""
import ctypes

import numpy as np
import pytest
import torch

import gpu_util as G
from oracle import force2d as O
from paper_2104_08571_amd import initial_states as ist
from paper_2104_08571_amd import ripple_fv as R

pytestmark = pytest.mark.gpu

LAYOUTS = [(R.SOA, 0), (R.AOS, 0), (R.AOSOA, 16), (R.AOSOA, 32), (R.AOSOA, 64)]
LAYOUT_IDS = ["soa", "aos", "aosoa16", "aosoa32", "aosoa64"]
TOL = {R.F32: 1e-5, R.F64: 1e-13}


def buffer(g, fill=float("nan")):
    b = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
    (b.view(torch.float32) if g.dtype == R.F32 else b.view(torch.float64)).fill_(fill)
    return b


def load(g, W, variables=R.PRIMITIVE, buf=None):
    """Import FP64 [4, ny, nx] (or [4, ny + 2, nx + 2] with WITH_PADDING)."""
    buf = buffer(g) if buf is None else buf
    src = torch.as_tensor(W, dtype=torch.float64).to("cuda").contiguous()
    R.ripple_force2d_import(G.ctx(), g, src.data_ptr(), variables, buf.data_ptr(), G.stream())
    torch.cuda.synchronize()
    return buf


def export(g, buf):
    dst = torch.empty((4, g.n[1], g.n[0]), dtype=torch.float64, device="cuda")
    R.ripple_force2d_export(G.ctx(), g, buf.data_ptr(), dst.data_ptr(), G.stream())
    torch.cuda.synchronize()
    return dst.cpu().numpy()


def flux_difference(g, u, lam):
    d = buffer(g)
    R.ripple_force2d_flux_difference(G.ctx(), g, u.data_ptr(), lam[0], lam[1], d.data_ptr(),
                                     G.stream())
    torch.cuda.synchronize()
    return d


def scale(U, lam):
    """S_c of the tolerance, per component, as a [4, 1, 1] array."""
    F, Gy = O.flux(U, 0), O.flux(U, 1)
    s = np.abs(F).max(axis=(1, 2)) + np.abs(Gy).max(axis=(1, 2)) + \
        np.abs(U).max(axis=(1, 2)) / min(lam)
    return s[:, None, None]


def assert_close(D, ref, U, lam, dtype, what):
    assert np.isfinite(D).all(), what
    err = np.abs(D - ref)
    bound = TOL[dtype] * scale(U, lam)
    assert (err <= bound).all(), f"{what}: max err / S = {(err / scale(U, lam)).max():.3e}"


def random_state(shape, seed):
    return ist.random_physical_2d(shape, seed)


# -- parity against the oracle ----------------------------------------------------

SHAPES = [(1, 1), (2, 1), (1, 5), (3, 2), (61, 3), (62, 17), (63, 33), (64, 16), (130, 70),
          (125, 129)]


@pytest.mark.parametrize("stage", [0, 1], ids=["registers", "lds"])
@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
@pytest.mark.parametrize("layout,w", LAYOUTS, ids=LAYOUT_IDS)
def test_parity_random_states(dtype, layout, w, stage):
    """Cell-wise random states, every boundary combination, grids from one
    cell to several strips (62 columns) and segments with ragged ends; rows
    through registers and staged through LDS."""
    lam = (0.3, 0.2)
    for k, shape in enumerate(SHAPES):
        for bc in ((0, 0), (1, 1), (0, 1), (1, 0)):
            g = R.make_force2d_grid(shape, dtype=dtype, layout=layout, aosoa_w=w, bc=bc,
                                    stage=stage)
            u = load(g, random_state(shape, 100 + k))
            U = export(g, u)
            D = export(g, flux_difference(g, u, lam))
            ref = O.flux_difference(U, lam, bc)
            assert_close(D, ref, U, lam, dtype, f"{shape} bc {bc}")
            den = np.abs(ref).sum()
            if den == 0.0:   # every neighbour equals the cell (one cell, transmissive)
                assert np.all(D == 0.0), (shape, bc)
                continue
            rel = np.abs(D - ref).sum() / den
            assert rel < (2e-6 if dtype == R.F32 else 1e-14), (shape, bc, rel)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_parity_smooth_field(dtype):
    """The benchmark's smooth periodic field at 1000 x 700 (17 strips, ragged
    last strip and segment)."""
    shape, lam = (1000, 700), (0.25, 0.25)
    g = R.make_force2d_grid(shape, dtype=dtype, layout=R.SOA, bc=(1, 1))
    u = load(g, ist.smooth_periodic_2d(shape, 2104))
    U = export(g, u)
    D = export(g, flux_difference(g, u, lam))
    assert_close(D, O.flux_difference(U, lam, (1, 1)), U, lam, dtype, "smooth")


def test_sod_exact_values():
    """Sod data along x and along y, FP64: the GPU equals the oracle to
    rounding, and cells away from the jump have exactly zero difference."""
    for axis in (0, 1):
        shape = (40, 6) if axis == 0 else (6, 40)
        g = R.make_force2d_grid(shape, dtype=R.F64, layout=R.SOA, bc=(0, 0))
        u = load(g, ist.sod_2d(shape, axis=axis))
        U = export(g, u)
        D = export(g, flux_difference(g, u, (0.4, 0.4)))
        ref = O.flux_difference(U, (0.4, 0.4), (0, 0))
        assert_close(D, ref, U, (0.4, 0.4), R.F64, f"sod axis {axis}")
        far = [0, 1, 2, 17, 22, 37, 38, 39]
        Dn = D[:, :, far] if axis == 0 else D[:, far, :]
        assert np.all(Dn == 0.0)


# -- invariances (bitwise) ------------------------------------------------------------

@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_uniform_state_gives_zero(dtype):
    W = np.broadcast_to(np.array([1.3, 0.2, -0.1, 0.8])[:, None, None], (4, 19, 70)).copy()
    for layout, w in LAYOUTS:
        for bc in ((0, 0), (1, 1)):
            g = R.make_force2d_grid((70, 19), dtype=dtype, layout=layout, aosoa_w=w, bc=bc)
            D = export(g, flux_difference(g, load(g, W), (0.3, 0.7)))
            assert np.all(D == 0.0), (layout, w, bc)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_layouts_and_tilings_bitwise_equal(dtype):
    """Layout, workgroup size, segment length and LDS staging never change
    the bits."""
    shape, lam, bc = (150, 77), (0.3, 0.2), (1, 0)
    W = random_state(shape, 7)
    ref = None
    for layout, w in LAYOUTS:
        for block, seg, stage in ((0, 0, 0), (64, 1, 0), (128, 2, 0), (256, 3, 0), (512, 5, 0),
                                  (64, 16, 0), (512, 200, 0), (0, 0, 1), (64, 1, 1), (256, 3, 1),
                                  (1024, 16, 1), (512, 200, 1)):
            g = R.make_force2d_grid(shape, dtype=dtype, layout=layout, aosoa_w=w, bc=bc,
                                    block=block, segment=seg, stage=stage)
            D = export(g, flux_difference(g, load(g, W), lam))
            if ref is None:
                ref = D
            assert np.array_equal(D, ref), (layout, w, block, seg, stage)


@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_padded_boundary_reads_storage(dtype):
    """PADDED axes read the padding ring as stored: a ring holding the
    periodic (or transmissive) neighbours reproduces that boundary bitwise."""
    shape, lam = (70, 33), (0.3, 0.2)
    W = random_state(shape, 8).numpy()
    for bc in ((1, 1), (0, 0), (1, 0)):
        P = np.empty((4, shape[1] + 2, shape[0] + 2))
        P[:, 1:-1, 1:-1] = W
        P[:, 1:-1, 0] = W[:, :, -1] if bc[0] else W[:, :, 0]
        P[:, 1:-1, -1] = W[:, :, 0] if bc[0] else W[:, :, -1]
        P[:, 0, :] = P[:, -2, :] if bc[1] else P[:, 1, :]
        P[:, -1, :] = P[:, 1, :] if bc[1] else P[:, -2, :]
        ref_g = R.make_force2d_grid(shape, dtype=dtype, layout=R.SOA, bc=bc)
        ref = export(ref_g, flux_difference(ref_g, load(ref_g, W), lam))
        for padded in ((2, 2), (2, bc[1]), (bc[0], 2)):
            for layout, stage in ((R.AOS, 0), (R.AOS, 1), (R.SOA, 1)):
                g = R.make_force2d_grid(shape, dtype=dtype, layout=layout, bc=padded, stage=stage)
                u = load(g, P, variables=R.PRIMITIVE | R.WITH_PADDING)
                D = export(g, flux_difference(g, u, lam))
                assert np.array_equal(D, ref), (bc, padded, layout, stage)


@pytest.mark.parametrize("stage", [0, 1], ids=["registers", "lds"])
def test_output_padding_and_input_untouched(stage):
    shape = (100, 40)
    for dtype, view in ((R.F32, torch.int32), (R.F64, torch.int64)):
        g = R.make_force2d_grid(shape, dtype=dtype, layout=R.SOA, bc=(0, 1), stage=stage)
        u = load(g, random_state(shape, 9))
        before = u.clone()
        d = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
        d.view(view).fill_(-1)
        R.ripple_force2d_flux_difference(G.ctx(), g, u.data_ptr(), 0.3, 0.3, d.data_ptr(),
                                         G.stream())
        torch.cuda.synchronize()
        assert torch.equal(u, before)
        assert int((d.view(view) != -1).sum()) == 4 * shape[0] * shape[1]


def test_rejected_arguments_enqueue_nothing():
    g = R.make_force2d_grid((64, 8), dtype=R.F32, layout=R.SOA)
    u = load(g, random_state((64, 8), 10))
    d = buffer(g, 0.0)
    small = G.RawDeviceBuffer(g.bytes // 2)   # exact size: visible to the range check
    bad = [
        dict(lam=(0.0, 0.1)), dict(lam=(0.1, -1.0)), dict(lam=(float("nan"), 0.1)),
        dict(lam=(float("inf"), 0.1)), dict(d=u), dict(d=small), dict(u=small),
    ]
    for b in bad:
        lam = b.get("lam", (0.2, 0.2))
        uu, dd = b.get("u", u), b.get("d", d)
        st = R.call("ripple_force2d_flux_difference", G.ctx(), ctypes.byref(g),
                    uu.data_ptr(), lam[0], lam[1], dd.data_ptr(), G.stream())
        assert st == R.E_INVALID, b
    torch.cuda.synchronize()
    small.free()
    assert int((d != 0).sum()) == 0
    stale = R.make_force2d_grid((64, 8), dtype=R.F32, layout=R.SOA)
    stale.bytes += 64
    with pytest.raises(R.RippleFVError) as e:
        R.ripple_force2d_flux_difference(G.ctx(), stale, u.data_ptr(), 0.2, 0.2, d.data_ptr(),
                                         G.stream())
    assert e.value.status == R.E_INVALID


# -- full size: sampled cells against the oracle ---------------------------------------

def window(U_dev, bc, cells):
    """3 x 3 neighbourhoods (boundary mapping written out here) of the given
    (i, j) cells of a device state [4, ny, nx], as padded 1 x 1 arrays."""
    ny, nx = U_dev.shape[1], U_dev.shape[2]

    def idx(k, n, b):
        if 0 <= k < n:
            return k
        return k % n if b == 1 else (0 if k < 0 else n - 1)

    out = []
    for i, j in cells:
        ii = [idx(i + o, nx, bc[0]) for o in (-1, 0, 1)]
        jj = [idx(j + o, ny, bc[1]) for o in (-1, 0, 1)]
        out.append(U_dev[:, jj][:, :, ii].cpu().numpy())
    return out


@pytest.mark.parametrize("stage", [0, 1], ids=["registers", "lds"])
@pytest.mark.parametrize("dtype", [R.F32, R.F64], ids=["f32", "f64"])
def test_full_size_sampled(dtype, stage):
    """32768^2 (the largest size of the paper's table) smooth periodic field,
    SoA, in the benchmark's launch configurations (rows through registers
    and staged through LDS): sampled cells -- corners, edges, strip and
    segment boundaries, random interior cells -- against the oracle on their
    neighbourhoods; the periodic sum of the flux differences vanishes to
    rounding."""
    n, lam = 32768, (0.25, 0.25)
    g = R.make_force2d_grid((n, n), dtype=dtype, layout=R.SOA, bc=(1, 1), stage=stage)
    W = ist.smooth_periodic_2d((n, n), 8571, device="cuda")
    u = buffer(g)
    R.ripple_force2d_import(G.ctx(), g, W.data_ptr(), R.PRIMITIVE, u.data_ptr(), G.stream())
    torch.cuda.synchronize()
    del W
    d = flux_difference(g, u, lam)
    U = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    R.ripple_force2d_export(G.ctx(), g, u.data_ptr(), U.data_ptr(), G.stream())
    del u
    D = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    R.ripple_force2d_export(G.ctx(), g, d.data_ptr(), D.data_ptr(), G.stream())
    torch.cuda.synchronize()
    del d
    rng = np.random.default_rng(5)
    cells = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (61, 127), (62, 128), (123, 255),
             (124, 256), (n - 1, 5000), (7, n - 1)]
    cells += [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(300)]
    Wins = window(U, (1, 1), cells)
    S = torch.stack([U[c].abs().max() for c in range(4)]).cpu().numpy()
    total = D.sum(dim=(1, 2)).cpu().numpy()
    Dabs = D.abs().sum(dim=(1, 2)).cpu().numpy()
    for (i, j), Pw in zip(cells, Wins):
        ref = O.flux_difference_padded(Pw, lam)[:, 0, 0]
        got = D[:, j, i].cpu().numpy()
        Ssc = np.abs(O.flux(Pw, 0)).max(axis=(1, 2)) + np.abs(O.flux(Pw, 1)).max(axis=(1, 2)) + \
            S / min(lam)
        assert (np.abs(got - ref) <= TOL[dtype] * Ssc).all(), ((i, j), got, ref)
    assert (np.abs(total) <= 1e-9 * Dabs + 1e-9).all() if dtype == R.F64 else \
        (np.abs(total) <= 1e-4 * Dabs + 1e-4).all(), (total, Dabs)
