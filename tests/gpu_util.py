"""Helpers for the GPU tests: device buffers, import/export through the C ABI,
and comparison against the FP64 oracle."""
import numpy as np
import torch

from paper_2104_08571_amd import ripple_fv as R

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = R.ripple_fv_create(0)
    return _CTX


def stream():
    return torch.cuda.current_stream().cuda_stream


def buffer(g, poison=True):
    """A state buffer for grid g; NaN-filled so that reading padding that
    nothing wrote shows up as NaN in the result."""
    b = torch.empty(g.bytes, dtype=torch.uint8, device="cuda")
    if poison:
        (b.view(torch.float32) if g.dtype == R.F32 else b.view(torch.float64)).fill_(float("nan"))
    return b


def load(g, W, buf=None, variables=R.PRIMITIVE):
    """Import an FP64 [5, nz, ny, nx] array (primitive by default) into a buffer."""
    if buf is None:
        buf = buffer(g)
    src = torch.as_tensor(np.asarray(W) if not torch.is_tensor(W) else W,
                          dtype=torch.float64).to("cuda").contiguous()
    assert tuple(src.shape) == (5, g.n[2], g.n[1], g.n[0])
    R.ripple_fv_import(ctx(), g, src.data_ptr(), variables, buf.data_ptr(), stream())
    torch.cuda.synchronize()
    return buf


def export(g, buf):
    dst = torch.empty((5, g.n[2], g.n[1], g.n[0]), dtype=torch.float64, device="cuda")
    R.ripple_fv_export(ctx(), g, buf.data_ptr(), dst.data_ptr(), stream())
    torch.cuda.synchronize()
    return dst.cpu().numpy()


def run(grids, states, nsteps, cfl=0.9, flags=R.RUN_EAGER):
    """Run a batch from primitive initial states; returns (list of FP64
    conserved arrays, list of times).  The state advances in place in the
    first buffer; the second is workspace."""
    if isinstance(grids, R.Grid):
        grids = [grids]
        states = [states]
    a = [load(g, W) for g, W in zip(grids, states)]
    b = [buffer(g) for g in grids]
    R.ripple_fv_run_batch(ctx(), grids, [x.data_ptr() for x in a], [x.data_ptr() for x in b],
                          nsteps, cfl, flags, stream())
    torch.cuda.synchronize()
    assert R.ripple_fv_check(ctx()) == R.OK
    t, _ = R.ripple_fv_batch_time(ctx(), grids)
    return [export(g, x) for g, x in zip(grids, a)], t


def rel_l1(a, b):
    """Per-variable relative L1 error sum|a - b| / sum|b| (0 when both vanish)."""
    out = []
    for c in range(5):
        den = np.abs(b[c]).sum()
        num = np.abs(a[c] - b[c]).sum()
        out.append(num / den if den > 0 else (0.0 if num == 0 else np.inf))
    return np.array(out)


def rel_linf(a, b):
    """Per-variable relative maximum error max|a - b| / scale: the scale of
    rho and E is max|b| of that variable, the scale of each momentum
    component the largest max|b| over the three components (a component that
    vanishes in the reference, such as the transverse momenta of a planar
    problem, is measured against the momentum the flow has).  0 when both
    vanish, inf when only the reference does."""
    mom = max(np.abs(b[c]).max() for c in (1, 2, 3))
    out = []
    for c in range(5):
        den = mom if c in (1, 2, 3) else np.abs(b[c]).max()
        num = np.abs(a[c] - b[c]).max()
        out.append(num / den if den > 0 else (0.0 if num == 0 else np.inf))
    return np.array(out)


# Elementwise bound beside the relative L1 bound: ten times the L1 tolerance,
# relative to the variable's largest magnitude.  An L1 sum alone lets a few
# wrong cells through (one wrong row of a 512^3 grid is 4e-6 of its cells);
# the largest errors measured after the full step counts stay a factor of
# ten or more below this (FP32: 1.3e-5 on rho u after 50 steps at 512^3).
LINF_FACTOR = 10.0


def assert_parity(gpu, ref, tol, what="", tol_inf=None):
    """Per-variable relative L1 <= tol and relative Linf (rel_linf) <=
    tol_inf (default LINF_FACTOR * tol); returns the L1 errors."""
    assert np.isfinite(gpu).all(), f"{what}: non-finite values in the GPU result"
    err = rel_l1(gpu, ref)
    assert (err <= tol).all(), f"{what}: relative L1 per variable {err} exceeds {tol}"
    tol_inf = LINF_FACTOR * tol if tol_inf is None else tol_inf
    inf = rel_linf(gpu, ref)
    assert (inf <= tol_inf).all(), f"{what}: relative Linf per variable {inf} exceeds {tol_inf}"
    return err


def unit_dx(n):
    return [1.0 / n[0], 1.0 / n[1], 1.0 / n[2]]


def padded_cells(g, buf):
    """The buffer as an FP64 array [5, nz+4, ny+4, nx+4] over the cells
    (i, j, k) in [-2, n+2)^3, interior plus padding (SoA only)."""
    assert g.layout == R.SOA
    px, py, _ = g.pitch
    slots = g.bytes // (5 * (4 if g.dtype == R.F32 else 8))
    flat = (buf.view(torch.float32) if g.dtype == R.F32 else buf.view(torch.float64))
    flat = flat.reshape(5, slots).cpu().numpy().astype(np.float64)
    i = np.arange(-2, g.n[0] + 2)[None, None, :]
    j = np.arange(-2, g.n[1] + 2)[None, :, None]
    k = np.arange(-2, g.n[2] + 2)[:, None, None]
    q = ((k + 2) * py + (j + 2)) * px + i + g.x_origin
    return flat[:, q]


class RawDeviceBuffer:
    """An exact-size hipMalloc allocation (torch's caching allocator carves
    tensors out of larger segments, which hides undersized buffers from the
    library's allocation-range check)."""

    def __init__(self, nbytes):
        import ctypes
        self._hip = ctypes.CDLL("libamdhip64.so")
        self.ptr = ctypes.c_void_p()
        err = self._hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(int(nbytes)))
        assert err == 0, f"hipMalloc failed: {err}"

    def data_ptr(self):
        return int(self.ptr.value)

    def free(self):
        if self.ptr:
            self._hip.hipFree(self.ptr)
            self.ptr = None
