"""The C-ABI library loads, exports every declared entry point, and its
host-only logic (descriptor validation, partitioning) behaves as declared.
No GPU needed: nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

from paper_2104_08571_amd import ripple_fv as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for header in sorted(os.listdir(os.path.join(ROOT, "include"))):
        with open(os.path.join(ROOT, "include", header)) as f:
            text = f.read()
        decl = r"^(?:ripple_fv_status|void|const char\*)\s+(ripple_(?:fv|force2d|particles)_[a-z_]+)\("
        names.update(re.findall(decl, text, flags=re.M))
    return sorted(names)


def test_header_and_binding_agree():
    assert declared_functions() == sorted(R.EXPORTED)


def test_library_exports_every_symbol():
    lib = R.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_grid_struct_size():
    # 3*4 + 3*4 + 3*8 + 4*4 + 6*4 + 8*4 + 3*8 + 8, no padding holes
    assert ctypes.sizeof(R.Grid) == 152
    assert R.Grid.pitch.offset == 120


def slots(px, py, pz, ox):
    return (px * py * pz + ox + 63) // 64 * 64


def test_grid_init_pitches():
    # SoA: interior rows start on 128-byte lines (x_origin = 128 B / element)
    g = R.make_grid((10, 7, 5), dtype=R.F32, layout=R.SOA)
    assert list(g.pitch) == [32, 11, 9] and g.x_origin == 32
    assert g.bytes == slots(32, 11, 9, 32) * 5 * 4
    g = R.make_grid((512, 7, 5), dtype=R.F32, layout=R.SOA)
    assert g.pitch[0] == 544
    g = R.make_grid((512, 7, 5), dtype=R.F64, layout=R.SOA)
    assert list(g.pitch) == [528, 11, 9] and g.x_origin == 16
    # AoS: row pitch rounded up to even, interior at x index 2
    g = R.make_grid((11, 7, 5), dtype=R.F32, layout=R.AOS)
    assert list(g.pitch) == [16, 11, 9] and g.x_origin == 2
    assert g.bytes == slots(16, 11, 9, 2) * 5 * 4
    # AoSoA: rows start on a block and on a 128-byte line
    g = R.make_grid((10, 7, 5), dtype=R.F64, layout=R.AOSOA, aosoa_w=16)
    assert list(g.pitch) == [16, 11, 9] and g.x_origin == 16
    assert g.bytes == slots(16, 11, 9, 16) * 5 * 8
    g = R.make_grid((60, 7, 5), dtype=R.F64, layout=R.AOSOA, aosoa_w=64)
    assert g.pitch[0] == 64 and g.x_origin == 64


def test_grid_rows_do_not_overlap():
    """Every cell of [-2, n+2)^3 has its own slot inside the buffer."""
    import numpy as np
    for layout, w in ((R.AOS, 0), (R.SOA, 0), (R.AOSOA, 16), (R.AOSOA, 64)):
        for dt in (R.F32, R.F64):
            g = R.make_grid((13, 5, 4), dtype=dt, layout=layout, aosoa_w=w)
            px, py = g.pitch[0], g.pitch[1]
            i = np.arange(-2, 15)[None, None, :]
            j = np.arange(-2, 7)[None, :, None]
            k = np.arange(-2, 6)[:, None, None]
            q = ((k + 2) * py + (j + 2)) * px + i + g.x_origin
            assert len(np.unique(q)) == q.size
            assert q.min() >= 0 and q.max() < g.bytes // (5 * (4 if dt == R.F32 else 8))


@pytest.mark.parametrize("bad", [
    dict(n=(0, 4, 4)), dict(n=(4, 4, 0)), dict(n=(4, -1, 4)), dict(dx=(0.0, 0.1, 0.1)), dict(dx=(-1.0, 0.1, 0.1)),
    dict(dtype=2), dict(layout=3), dict(layout=R.AOSOA, aosoa_w=8), dict(layout=R.SOA, aosoa_w=16),
    dict(bc=(0, 2, 0)), dict(tiling=(64, 0, 0, 0)), dict(tiling=(0, 512, 0, 0)),
    dict(tiling=(0, 0, 2, 0)), dict(tiling=(0, 0, 0, -1)), dict(tiling=(0, 0, 0, 0, 3)),
    dict(tiling=(0, 0, 0, 0, 0, 4)), dict(tiling=(0, 0, 0, 0, 0, -1)),
    dict(n=(2000, 2000, 2000)),
])
def test_grid_init_rejects(bad):
    kw = dict(n=(8, 8, 8))
    kw.update(bad)
    with pytest.raises(R.RippleFVError) as e:
        R.make_grid(**kw)
    assert e.value.status == R.E_INVALID


def test_lane_offset_bound():
    """Tiles address their lanes by 32-bit byte offsets from a wave-uniform
    base; the rows form of the fused pass and the separate y sweep span up to
    512 / n0 planes.  A thin x extent with large planes in AoS FP64 would
    pass the cell-count bound but overflow the offsets: rejected.  The same
    extents in SoA (one element per cell between lanes), and planar grids
    (whose tiles stay within a row), are accepted."""
    with pytest.raises(R.RippleFVError) as e:
        R.make_grid((16, 90000, 32), dtype=R.F64, layout=R.AOS)
    assert e.value.status == R.E_INVALID
    R.make_grid((16, 90000, 32), dtype=R.F64, layout=R.SOA)
    R.make_grid((9600, 6000, 1), dtype=R.F64, layout=R.AOS)
    # the benchmark's largest grids stay far inside the bound
    R.make_grid((1024, 1024, 1024), dtype=R.F64, layout=R.AOS)
    R.make_grid((388, 384, 384), dtype=R.F32, layout=R.AOSOA, aosoa_w=64)


def test_status_strings():
    assert R.ripple_fv_status_string(R.OK) == "ok"
    assert R.ripple_fv_status_string(R.E_NONPHYSICAL) == "non-physical state"
    assert R.ripple_fv_status_string(99) == "unknown status"


def test_partition_links_and_extents():
    whole = R.make_grid((10, 9, 8), dtype=R.F32, bc=(R.TRANSMISSIVE, R.PERIODIC, R.TRANSMISSIVE))
    subs = R.ripple_fv_partition(whole, (2, 3, 1), first_index=4)
    assert len(subs) == 6
    # extents split as evenly as possible; x fastest
    assert [list(s.n) for s in subs] == [[5, 3, 8], [5, 3, 8]] * 3
    for idx, s in enumerate(subs):
        a, b = idx % 2, idx // 2
        assert s.group == 4
        assert list(s.dx) == list(whole.dx)
        # x: transmissive, two parts -> inner faces linked only
        assert s.nbr[0] == (-1 if a == 0 else 4 + idx - 1)
        assert s.nbr[1] == (-1 if a == 1 else 4 + idx + 1)
        # y: periodic, three parts -> linked around
        assert s.nbr[2] == 4 + a + 2 * ((b - 1) % 3)
        assert s.nbr[3] == 4 + a + 2 * ((b + 1) % 3)
        # z: one part, transmissive -> physical
        assert s.nbr[4] == -1 and s.nbr[5] == -1
        assert s.bytes == slots(s.pitch[0], s.pitch[1], s.pitch[2], s.x_origin) * 5 * 4
    odd = R.ripple_fv_partition(R.make_grid((11, 4, 4)), (2, 1, 1))
    assert [o.n[0] for o in odd] == [6, 5]


def test_partition_rejects_too_thin():
    whole = R.make_grid((6, 6, 6))
    with pytest.raises(R.RippleFVError):
        R.ripple_fv_partition(whole, (4, 1, 1))


def test_planar_grids_and_partition():
    """One-cell axes are accepted; a periodic one-cell axis is not linked to
    itself by the partition, and a split axis keeps two cells per block."""
    g = R.make_grid((64, 40, 1), bc=(1, 1, 1))
    assert list(g.pitch) == [g.pitch[0], 44, 5]
    subs = R.ripple_fv_partition(g, (2, 1, 1))
    assert [list(s.nbr) for s in subs] == [[1, 1, 0, 0, -1, -1], [0, 0, 1, 1, -1, -1]]
    assert all(s.n[2] == 1 for s in subs)
    with pytest.raises(R.RippleFVError):
        R.ripple_fv_partition(g, (1, 1, 2))
    R.make_grid((1, 1, 1))


# -- two-dimensional flux-difference descriptors ----------------------------------

def test_force2d_struct_size():
    # 2*4 + 2*4 + 8*4 + 2*8 + 8, no padding holes
    assert ctypes.sizeof(R.Force2DGrid) == 72
    assert R.Force2DGrid.pitch.offset == 48


def test_force2d_grid_init_pitches():
    def slots2(px, py, ox):
        return (px * py + ox + 63) // 64 * 64
    g = R.make_force2d_grid((1000, 37), dtype=R.F32, layout=R.SOA)
    assert list(g.pitch) == [1024, 39] and g.x_origin == 32
    assert g.bytes == slots2(1024, 39, 32) * 4 * 4
    g = R.make_force2d_grid((14, 3), dtype=R.F64, layout=R.SOA)
    assert list(g.pitch) == [16, 5] and g.x_origin == 16
    g = R.make_force2d_grid((15, 3), dtype=R.F64, layout=R.SOA)
    assert list(g.pitch) == [32, 5]
    g = R.make_force2d_grid((5, 3), dtype=R.F64, layout=R.AOS)
    assert list(g.pitch) == [7, 5] and g.x_origin == 1
    assert g.bytes == slots2(7, 5, 1) * 4 * 8
    g = R.make_force2d_grid((5, 3), dtype=R.F32, layout=R.AOSOA, aosoa_w=64)
    assert list(g.pitch) == [64, 5] and g.x_origin == 64
    g = R.make_force2d_grid((1, 1), dtype=R.F32, layout=R.AOSOA, aosoa_w=16)
    assert list(g.pitch) == [32, 3] and g.x_origin == 32


def test_force2d_rows_do_not_overlap():
    """Every cell of [-1, n]^2 has its own slot inside the buffer, and SoA /
    AoSoA interior rows start on 128-byte lines."""
    import numpy as np
    for layout, w in ((R.AOS, 0), (R.SOA, 0), (R.AOSOA, 16), (R.AOSOA, 64)):
        for dt in (R.F32, R.F64):
            for n in ((13, 5), (1, 1), (64, 2)):
                g = R.make_force2d_grid(n, dtype=dt, layout=layout, aosoa_w=w)
                s = 4 if dt == R.F32 else 8
                i = np.arange(-1, n[0] + 1)[None, :]
                j = np.arange(-1, n[1] + 1)[:, None]
                q = (j + 1) * g.pitch[0] + i + g.x_origin
                assert len(np.unique(q)) == q.size
                assert q.min() >= 0 and q.max() < g.bytes // (4 * s)
                if layout != R.AOS:
                    assert all(((jj + 1) * g.pitch[0] + g.x_origin) * s % 128 == 0
                               for jj in range(n[1]))


@pytest.mark.parametrize("bad", [
    dict(n=(0, 4)), dict(n=(4, 0)), dict(n=((1 << 20) + 1, 4)), dict(dtype=2), dict(layout=3),
    dict(layout=R.AOSOA, aosoa_w=8), dict(layout=R.SOA, aosoa_w=16), dict(bc=(0, 3)),
    dict(bc=(-1, 0)), dict(block=32), dict(block=2048), dict(segment=-1),
])
def test_force2d_grid_init_rejects(bad):
    kw = dict(n=(8, 8))
    kw.update(bad)
    with pytest.raises(R.RippleFVError) as e:
        R.make_force2d_grid(**kw)
    assert e.value.status == R.E_INVALID


@pytest.mark.parametrize("stage,status", [(0, R.OK), (1, R.OK), (2, R.E_INVALID), (-1, R.E_INVALID)])
def test_force2d_stage_values(stage, status):
    g = R.Force2DGrid()
    g.n[0] = g.n[1] = 8
    g.layout = R.SOA
    g.stage = stage
    assert R.call("ripple_force2d_grid_init", ctypes.byref(g)) == status


# -- particle descriptors ------------------------------------------------------------

def test_particles_descriptor():
    assert ctypes.sizeof(R.Particles) == 48 and R.Particles.slots.offset == 32
    p = R.make_particles(1000, dtype=R.F32, layout=R.SOA)
    assert p.slots == 1024 and p.bytes == 1024 * 6 * 4
    p = R.make_particles(1, dtype=R.F64, layout=R.AOSOA, aosoa_w=16)
    assert p.slots == 64 and p.bytes == 64 * 6 * 8


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(n=(1 << 34) + 1), dict(dtype=2), dict(layout=3), dict(layout=R.SOA, aosoa_w=16),
    dict(layout=R.AOSOA, aosoa_w=8), dict(block=96), dict(stage=2), dict(stage=-1),
])
def test_particles_rejects(bad):
    kw = dict(n=100)
    kw.update(bad)
    with pytest.raises(R.RippleFVError) as e:
        R.make_particles(**kw)
    assert e.value.status == R.E_INVALID
