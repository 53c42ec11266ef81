"""ctypes binding of libripple_fv.so (declared in include/ripple_fv.h,
include/ripple_force2d.h and include/ripple_particles.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions keep the C names; each raises RippleFVError on a non-OK status
(``call`` returns the raw status instead).  Device pointers are plain ints
(``tensor.data_ptr()``), streams are ``torch.cuda.Stream.cuda_stream`` ints
or None for the default stream.

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_HERE, "libripple_fv.so")

OK, E_INVALID, E_UNSUPPORTED, E_DEVICE, E_NONPHYSICAL, E_NOMEM = range(6)
AOS, SOA, AOSOA = 0, 1, 2
F32, F64 = 0, 1
TRANSMISSIVE, PERIODIC = 0, 1
PRIMITIVE, CONSERVED = 0, 1
RUN_EAGER, RUN_GRAPH, RUN_PER_GRID, RUN_PROFILE = 0, 1, 2, 4
COPY_NONTEMPORAL = 1
NOALLOC_MAX_GRIDS = 64
NOALLOC_SCRATCH_BYTES = 32768
K_WAVESPEED, K_DT, K_SWEEP_X, K_SWEEP_Y, K_SWEEP_Z, K_HALO, K_SWEEP_XY, NKERNELS = range(8)
KERNEL_NAMES = ["wavespeed", "dt", "sweep_x", "sweep_y", "sweep_z", "halo", "sweep_xy"]
AXIS_XY = 3
HALO = 2
NVAR = 5

EXPORTED = [
    "ripple_fv_grid_init", "ripple_fv_create", "ripple_fv_destroy", "ripple_fv_import",
    "ripple_fv_export", "ripple_fv_convert", "ripple_fv_max_wavespeed", "ripple_fv_sweep",
    "ripple_fv_step", "ripple_fv_run_batch", "ripple_fv_run_batch_noalloc",
    "ripple_fv_batch_time", "ripple_fv_batch_tune",
    "ripple_fv_partition", "ripple_fv_halo_exchange", "ripple_fv_conserved_sums",
    "ripple_fv_error_norms", "ripple_fv_stream_copy", "ripple_fv_check", "ripple_fv_profile",
    "ripple_fv_status_string",
    "ripple_fv_last_error",
    "ripple_force2d_grid_init", "ripple_force2d_import", "ripple_force2d_export",
    "ripple_force2d_flux_difference",
    "ripple_particles_init", "ripple_particles_import", "ripple_particles_export",
    "ripple_particles_update",
]

PADDED = 2             # ripple_force2d boundary kind: padding read as stored
WITH_PADDING = 2       # ripple_force2d_import flag: source covers the padding ring
NVAR2D = 4


class Grid(ctypes.Structure):
    """ripple_fv_grid."""
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("layout", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("aosoa_w", ctypes.c_int32),
        ("group", ctypes.c_int32),
        ("nbr", ctypes.c_int32 * 6),
        ("x_block", ctypes.c_int32),
        ("yz_block", ctypes.c_int32),
        ("yz_segment", ctypes.c_int32),
        ("persist", ctypes.c_int32),
        ("yz_cols", ctypes.c_int32),
        ("split_xy", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("x_origin", ctypes.c_int32),
        ("pitch", ctypes.c_int64 * 3),
        ("bytes", ctypes.c_int64),
    ]

    def __repr__(self):
        return (f"Grid(n={list(self.n)}, bc={list(self.bc)}, layout={self.layout}, "
                f"dtype={self.dtype}, aosoa_w={self.aosoa_w}, group={self.group}, "
                f"nbr={list(self.nbr)}, tiling=({self.x_block}, {self.yz_block}, "
                f"{self.yz_segment}, {self.persist}, {self.yz_cols}), split_xy={self.split_xy}, "
                f"bytes={self.bytes})")


class Force2DGrid(ctypes.Structure):
    """ripple_force2d_grid."""
    _fields_ = [
        ("n", ctypes.c_int32 * 2),
        ("bc", ctypes.c_int32 * 2),
        ("layout", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("aosoa_w", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("segment", ctypes.c_int32),
        ("stage", ctypes.c_int32),
        ("x_origin", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("pitch", ctypes.c_int64 * 2),
        ("bytes", ctypes.c_int64),
    ]

    def __repr__(self):
        return (f"Force2DGrid(n={list(self.n)}, bc={list(self.bc)}, layout={self.layout}, "
                f"dtype={self.dtype}, aosoa_w={self.aosoa_w}, block={self.block}, "
                f"segment={self.segment}, bytes={self.bytes})")


class Particles(ctypes.Structure):
    """ripple_particles."""
    _fields_ = [
        ("n", ctypes.c_int64),
        ("layout", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("aosoa_w", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("stage", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("slots", ctypes.c_int64),
        ("bytes", ctypes.c_int64),
    ]


class RippleFVError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(message)


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise ImportError(f"{LIBRARY} is missing: build it with "
                              "`python paper_2104_08571_amd/build.py` (no fallback exists)")
        L = ctypes.CDLL(LIBRARY)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    st = ctypes.c_int32
    vp = ctypes.c_void_p
    gp = ctypes.POINTER(Grid)
    fp = ctypes.POINTER(Force2DGrid)
    pp = ctypes.POINTER(Particles)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ripple_fv_grid_init": (st, [gp]),
        "ripple_fv_create": (st, [ctypes.POINTER(vp), ctypes.c_int32]),
        "ripple_fv_destroy": (None, [vp]),
        "ripple_fv_import": (st, [vp, gp, vp, ctypes.c_int32, vp, vp]),
        "ripple_fv_export": (st, [vp, gp, vp, vp, vp]),
        "ripple_fv_convert": (st, [vp, gp, vp, gp, vp, vp]),
        "ripple_fv_max_wavespeed": (st, [vp, gp, vp, vp, vp]),
        "ripple_fv_sweep": (st, [vp, gp, ctypes.c_int32, vp, vp, ctypes.c_double, vp]),
        "ripple_fv_step": (st, [vp, gp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp]),
        "ripple_fv_run_batch": (st, [vp, ctypes.c_int32, gp, ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int32, vp]),
        "ripple_fv_run_batch_noalloc": (st, [vp, ctypes.c_int32, gp, ctypes.POINTER(vp),
                                             ctypes.POINTER(vp), ctypes.c_int32,
                                             ctypes.c_double, vp]),
        "ripple_fv_batch_time": (st, [vp, ctypes.c_int32, gp, dp, dp]),
        "ripple_fv_batch_tune": (st, [vp, ctypes.c_int32, gp, gp, vp]),
        "ripple_fv_partition": (st, [gp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, gp]),
        "ripple_fv_halo_exchange": (st, [vp, ctypes.c_int32, gp, ctypes.POINTER(vp),
                                         ctypes.c_int32, vp]),
        "ripple_fv_conserved_sums": (st, [vp, gp, vp, vp, vp]),
        "ripple_fv_error_norms": (st, [vp, gp, vp, vp, vp, vp, vp]),
        "ripple_fv_stream_copy": (st, [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp]),
        "ripple_fv_check": (st, [vp]),
        "ripple_fv_profile": (st, [vp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "ripple_fv_status_string": (ctypes.c_char_p, [st]),
        "ripple_fv_last_error": (ctypes.c_char_p, [vp]),
        "ripple_force2d_grid_init": (st, [fp]),
        "ripple_force2d_import": (st, [vp, fp, vp, ctypes.c_int32, vp, vp]),
        "ripple_force2d_export": (st, [vp, fp, vp, vp, vp]),
        "ripple_force2d_flux_difference": (st, [vp, fp, vp, ctypes.c_double, ctypes.c_double,
                                                vp, vp]),
        "ripple_particles_init": (st, [pp]),
        "ripple_particles_import": (st, [vp, pp, vp, vp, vp]),
        "ripple_particles_export": (st, [vp, pp, vp, vp, vp]),
        "ripple_particles_update": (st, [vp, pp, vp, ctypes.c_double, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _check(status, ctx=None):
    if status != OK:
        msg = lib().ripple_fv_status_string(status).decode()
        if ctx is not None:
            detail = lib().ripple_fv_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise RippleFVError(status, msg)
    return status


def _grids(grids):
    if isinstance(grids, Grid):
        grids = [grids]
    arr = (Grid * len(grids))(*grids)
    return arr, len(grids)


def _ptrs(values):
    return (ctypes.c_void_p * len(values))(*[ctypes.c_void_p(int(v)) for v in values])


# -- C functions, same names --------------------------------------------------

def ripple_fv_grid_init(g):
    _check(lib().ripple_fv_grid_init(ctypes.byref(g)))
    return g


def ripple_fv_create(device=0):
    ctx = ctypes.c_void_p()
    _check(lib().ripple_fv_create(ctypes.byref(ctx), int(device)))
    return ctx


def ripple_fv_destroy(ctx):
    lib().ripple_fv_destroy(ctx)


def ripple_fv_import(ctx, g, src, variables, u, stream=None):
    _check(lib().ripple_fv_import(ctx, ctypes.byref(g), src, variables, u, stream), ctx)


def ripple_fv_export(ctx, g, u, dst, stream=None):
    _check(lib().ripple_fv_export(ctx, ctypes.byref(g), u, dst, stream), ctx)


def ripple_fv_convert(ctx, gs, src, gd, dst, stream=None):
    _check(lib().ripple_fv_convert(ctx, ctypes.byref(gs), src, ctypes.byref(gd), dst, stream), ctx)


def ripple_fv_max_wavespeed(ctx, g, u, s_dev, stream=None):
    _check(lib().ripple_fv_max_wavespeed(ctx, ctypes.byref(g), u, s_dev, stream), ctx)


def ripple_fv_sweep(ctx, g, axis, u_in, u_out, dt, stream=None):
    _check(lib().ripple_fv_sweep(ctx, ctypes.byref(g), axis, u_in, u_out, float(dt), stream), ctx)


def ripple_fv_step(ctx, g, u, work, cfl=0.9, dt=0.0, dt_dev=None, stream=None):
    _check(lib().ripple_fv_step(ctx, ctypes.byref(g), u, work, float(cfl), float(dt),
                                dt_dev, stream), ctx)


def ripple_fv_run_batch(ctx, grids, u, work, nsteps, cfl=0.9, flags=RUN_EAGER, stream=None):
    arr, n = _grids(grids)
    _check(lib().ripple_fv_run_batch(ctx, n, arr, _ptrs(u), _ptrs(work), int(nsteps),
                                     float(cfl), int(flags), stream), ctx)


def ripple_fv_run_batch_noalloc(ctx, grids, u, work, nsteps, cfl=0.9, stream=None):
    arr, n = _grids(grids)
    _check(lib().ripple_fv_run_batch_noalloc(ctx, n, arr, _ptrs(u), _ptrs(work), int(nsteps),
                                             float(cfl), stream), ctx)


def ripple_fv_batch_time(ctx, grids):
    """Returns (t, dt) lists per grid."""
    arr, n = _grids(grids)
    t = (ctypes.c_double * n)()
    dt = (ctypes.c_double * n)()
    _check(lib().ripple_fv_batch_time(ctx, n, arr, t, dt), ctx)
    return list(t), list(dt)


def ripple_fv_batch_tune(ctx, grids, stream=None):
    arr, n = _grids(grids)
    out = (Grid * n)()
    _check(lib().ripple_fv_batch_tune(ctx, n, arr, out, stream), ctx)
    return list(out)


def ripple_fv_partition(whole, parts, first_index=0):
    count = parts[0] * parts[1] * parts[2]
    out = (Grid * count)()
    p = (ctypes.c_int32 * 3)(*parts)
    _check(lib().ripple_fv_partition(ctypes.byref(whole), p, int(first_index), out))
    return list(out)


def ripple_fv_halo_exchange(ctx, grids, u, axis, stream=None):
    arr, n = _grids(grids)
    _check(lib().ripple_fv_halo_exchange(ctx, n, arr, _ptrs(u), int(axis), stream), ctx)


def ripple_fv_conserved_sums(ctx, g, u, sums_dev, stream=None):
    _check(lib().ripple_fv_conserved_sums(ctx, ctypes.byref(g), u, sums_dev, stream), ctx)


def ripple_fv_error_norms(ctx, g, u, ref_dev, l1_dev, linf_dev, stream=None):
    _check(lib().ripple_fv_error_norms(ctx, ctypes.byref(g), u, ref_dev, l1_dev, linf_dev, stream),
           ctx)


def ripple_fv_stream_copy(ctx, dst, src, nbytes, flags=0, stream=None):
    _check(lib().ripple_fv_stream_copy(ctx, dst, src, int(nbytes), int(flags), stream), ctx)


def ripple_fv_check(ctx):
    """Returns the status (OK or E_NONPHYSICAL); raises on other errors."""
    st = lib().ripple_fv_check(ctx)
    if st not in (OK, E_NONPHYSICAL):
        _check(st, ctx)
    return st


def ripple_fv_profile(ctx):
    """Returns {kernel name: (total ms, launches)} since the last call."""
    ms = (ctypes.c_double * NKERNELS)()
    cnt = (ctypes.c_int64 * NKERNELS)()
    _check(lib().ripple_fv_profile(ctx, ms, cnt), ctx)
    return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(NKERNELS)}


def ripple_fv_status_string(status):
    return lib().ripple_fv_status_string(int(status)).decode()


def ripple_fv_last_error(ctx):
    return lib().ripple_fv_last_error(ctx).decode()


def ripple_force2d_grid_init(g):
    _check(lib().ripple_force2d_grid_init(ctypes.byref(g)))
    return g


def ripple_force2d_import(ctx, g, src, variables, u, stream=None):
    _check(lib().ripple_force2d_import(ctx, ctypes.byref(g), src, int(variables), u, stream), ctx)


def ripple_force2d_export(ctx, g, u, dst, stream=None):
    _check(lib().ripple_force2d_export(ctx, ctypes.byref(g), u, dst, stream), ctx)


def ripple_force2d_flux_difference(ctx, g, u, lam_x, lam_y, d, stream=None):
    _check(lib().ripple_force2d_flux_difference(ctx, ctypes.byref(g), u, float(lam_x),
                                                float(lam_y), d, stream), ctx)


def ripple_particles_init(p):
    _check(lib().ripple_particles_init(ctypes.byref(p)))
    return p


def ripple_particles_import(ctx, p, src, buf, stream=None):
    _check(lib().ripple_particles_import(ctx, ctypes.byref(p), src, buf, stream), ctx)


def ripple_particles_export(ctx, p, buf, dst, stream=None):
    _check(lib().ripple_particles_export(ctx, ctypes.byref(p), buf, dst, stream), ctx)


def ripple_particles_update(ctx, p, buf, dt, stream=None):
    _check(lib().ripple_particles_update(ctx, ctypes.byref(p), buf, float(dt), stream), ctx)


def call(name, *args):
    """Raw call of a C entry point; returns its status without raising."""
    return getattr(lib(), name)(*args)


# -- descriptor helper ----------------------------------------------------------

def make_grid(n, dtype=F64, layout=SOA, bc=(TRANSMISSIVE,) * 3, dx=None, aosoa_w=0,
              group=-1, nbr=(-1,) * 6, tiling=(0, 0, 0, 0, 0, 0)):
    """A ripple_fv_grid with pitch and bytes filled (ripple_fv_grid_init).
    tiling = (x_block, yz_block, yz_segment, persist, yz_cols, split_xy)."""
    g = Grid()
    n = [int(v) for v in n]
    for d in range(3):
        g.n[d] = n[d]
        g.bc[d] = int(bc[d])
        g.dx[d] = float(dx[d]) if dx is not None else 1.0 / max(n[d], 1)
    for f in range(6):
        g.nbr[f] = int(nbr[f])
    g.layout = int(layout)
    g.dtype = int(dtype)
    g.aosoa_w = int(aosoa_w)
    g.group = int(group)
    tiling = list(tiling) + [0] * (6 - len(tiling))
    (g.x_block, g.yz_block, g.yz_segment, g.persist, g.yz_cols,
     g.split_xy) = [int(v) for v in tiling]
    return ripple_fv_grid_init(g)


def copy_grid(g, **changes):
    """A copy of a descriptor with some fields changed, re-initialised."""
    h = Grid()
    ctypes.memmove(ctypes.byref(h), ctypes.byref(g), ctypes.sizeof(Grid))
    for k, v in changes.items():
        if k in ("n", "bc", "dx", "nbr"):
            arr = getattr(h, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(h, k, v)
    return ripple_fv_grid_init(h)


def make_force2d_grid(n, dtype=F64, layout=SOA, bc=(TRANSMISSIVE,) * 2, aosoa_w=0, block=0,
                      segment=0, stage=0):
    """A ripple_force2d_grid with x_origin, pitch and bytes filled (stage 1:
    rows staged through LDS)."""
    g = Force2DGrid()
    for d in range(2):
        g.n[d] = int(n[d])
        g.bc[d] = int(bc[d])
    g.layout = int(layout)
    g.dtype = int(dtype)
    g.aosoa_w = int(aosoa_w)
    g.block = int(block)
    g.segment = int(segment)
    g.stage = int(stage)
    return ripple_force2d_grid_init(g)


def make_particles(n, dtype=F32, layout=SOA, aosoa_w=0, block=0, stage=0):
    """A ripple_particles descriptor with slots and bytes filled (stage 1:
    staged through LDS)."""
    p = Particles()
    p.n = int(n)
    p.layout = int(layout)
    p.dtype = int(dtype)
    p.aosoa_w = int(aosoa_w)
    p.block = int(block)
    p.stage = int(stage)
    return ripple_particles_init(p)
