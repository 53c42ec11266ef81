"""Seeded synthetic initial states (primitive variables, FP64).

This module holds only input recipes: it draws seeded random numbers and
evaluates the initial fields.  It contains none of the finite-volume scheme's
arithmetic (no equation of state, flux or update); both the FP64 oracle and
the HIP library convert the primitive fields it returns to conserved
variables with their own code.

Every three-dimensional generator returns a float64 torch tensor
``[5, nz, ny, nx]`` holding (rho, u, v, w, p) at cell centres
x_c = (i + 1/2) / N of the unit cube, on the requested device; the ``_2d``
generators return ``[4, ny, nx]`` holding (rho, u, v, p) on the unit square.
Sub-blocks of a larger grid are produced by passing the global extents and
the block's origin.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), uniform u = (x >> 11) * 2^-53.
"""
import math

import torch

_MASK = (1 << 64) - 1
N_MODES = 8
DEFAULT_SEEDS = {"smooth_256": 2104, "smooth_512": 8571, "batch_extents": 42,
                 "batch_grid_base": 1000}


class SplitMix64:
    """SplitMix64 stream (Steele, Lea, Flood 2014)."""

    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next_u64(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self):
        """Uniform double in [0, 1): the top 53 bits times 2^-53."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def fourier_modes(rng, count=N_MODES):
    """Draw `count` modes (kx, ky, kz, a, phi) in the order kx, ky, kz, a, phi.

    Wavenumbers are integers in 1..4, amplitudes U(0,1), phases U(0, 2 pi)."""
    modes = []
    for _ in range(count):
        kx = 1 + int(4.0 * rng.uniform())
        ky = 1 + int(4.0 * rng.uniform())
        kz = 1 + int(4.0 * rng.uniform())
        a = rng.uniform()
        phi = 2.0 * math.pi * rng.uniform()
        modes.append((kx, ky, kz, a, phi))
    return modes


def _f64(value, device):
    """A float64 scalar tensor (torch.where on Python floats would give float32)."""
    return torch.tensor(float(value), dtype=torch.float64, device=device)


def _centres(n_local, origin, n_global, device):
    """Cell-centre coordinates along one axis for a block of a global grid."""
    i = torch.arange(origin, origin + n_local, dtype=torch.float64, device=device)
    return (i + 0.5) / float(n_global)


def _coords(n_local, origin, n_global, device):
    x = _centres(n_local[0], origin[0], n_global[0], device)
    y = _centres(n_local[1], origin[1], n_global[1], device)
    z = _centres(n_local[2], origin[2], n_global[2], device)
    return x, y, z


def _normalise(n, origin, n_global):
    n = tuple(int(v) for v in n)
    origin = (0, 0, 0) if origin is None else tuple(int(v) for v in origin)
    n_global = n if n_global is None else tuple(int(v) for v in n_global)
    return n, origin, n_global


def fourier_field(modes, x, y, z):
    """f = sum_m (a_m / sum a) cos(2 pi (k_m . x_c) + phi_m), a [nz, ny, nx] tensor.

    Normalising by the sum of amplitudes bounds |f| by 1."""
    total = sum(m[3] for m in modes)
    f = torch.zeros((z.numel(), y.numel(), x.numel()), dtype=torch.float64, device=x.device)
    two_pi = 2.0 * math.pi
    for kx, ky, kz, a, phi in modes:
        arg = (two_pi * kz * z)[:, None, None] + (two_pi * ky * y)[None, :, None] \
            + (two_pi * kx * x)[None, None, :] + phi
        f.add_(torch.cos(arg), alpha=a / total)
    return f


def smooth_periodic(n, seed, origin=None, n_global=None, device="cpu"):
    """Smooth periodic state: rho = 1 + 0.2 f_rho, u_d = 0.1 f_d, p = 1.

    Four independent Fourier fields (rho, u, v, w) are drawn in that order
    from one SplitMix64 stream seeded with `seed`; each has 8 modes with
    integer wavenumbers 1..4 per axis, so every field is periodic on the
    unit cube."""
    n, origin, n_global = _normalise(n, origin, n_global)
    rng = SplitMix64(seed)
    modes = [fourier_modes(rng) for _ in range(4)]
    x, y, z = _coords(n, origin, n_global, device)
    W = torch.empty((5, n[2], n[1], n[0]), dtype=torch.float64, device=device)
    W[0] = 1.0 + 0.2 * fourier_field(modes[0], x, y, z)
    for d in range(3):
        W[1 + d] = 0.1 * fourier_field(modes[1 + d], x, y, z)
    W[4] = 1.0
    return W


def sod(n, axis=0, origin=None, n_global=None, device="cpu",
        left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0=0.5):
    """Planar Riemann problem along `axis`: left state where x_c < x0.

    left/right are (rho, normal velocity, p); the default is Sod's problem."""
    n, origin, n_global = _normalise(n, origin, n_global)
    coords = _coords(n, origin, n_global, device)
    c = coords[axis]
    is_left = c < x0
    shape = [1, 1, 1]
    shape[2 - axis] = n[axis]
    is_left = is_left.reshape(shape).expand(n[2], n[1], n[0])
    W = torch.zeros((5, n[2], n[1], n[0]), dtype=torch.float64, device=device)
    W[0] = torch.where(is_left, _f64(left[0], device), _f64(right[0], device))
    W[1 + axis] = torch.where(is_left, _f64(left[1], device), _f64(right[1], device))
    W[4] = torch.where(is_left, _f64(left[2], device), _f64(right[2], device))
    return W


def blast(n, origin=None, n_global=None, device="cpu", radius=0.1,
          p_in=1000.0, p_out=0.01, rho=1.0):
    """Spherical blast: rho = 1, u = 0, p = p_in where the cell centre lies
    strictly within `radius` of (1/2, 1/2, 1/2), else p_out."""
    n, origin, n_global = _normalise(n, origin, n_global)
    x, y, z = _coords(n, origin, n_global, device)
    r2 = ((z - 0.5) ** 2)[:, None, None] + ((y - 0.5) ** 2)[None, :, None] \
        + ((x - 0.5) ** 2)[None, None, :]
    inside = r2 < radius * radius
    W = torch.zeros((5, n[2], n[1], n[0]), dtype=torch.float64, device=device)
    W[0] = rho
    W[4] = torch.where(inside, _f64(p_in, device), _f64(p_out, device))
    return W


def shock_bubble(nx, ny, device="cpu", mach=3.81, x_shock=0.1, centre=(0.4, 0.5),
                 radius=0.2, rho_bubble=0.1, gamma=1.4):
    """Planar shock-bubble interaction on an nx x ny x 1 grid of square cells
    over [0, nx/ny] x [0, 1]: ambient gas at rest (rho = 1, p = 1); a shock of
    Mach number `mach` at x = x_shock moving towards +x, the gas behind it
    (x_c < x_shock) in the post-shock state of the normal-shock relations,
        rho2 = (g + 1) M^2 / ((g - 1) M^2 + 2),
        p2 = (2 g M^2 - (g - 1)) / (g + 1),
        u2 = M c1 (1 - 1 / rho2),  c1 = sqrt(g);
    and a bubble of density rho_bubble at ambient pressure, at rest, where
    the cell centre lies strictly within `radius` of `centre`."""
    h = 1.0 / ny
    x = (torch.arange(nx, dtype=torch.float64, device=device) + 0.5) * h
    y = (torch.arange(ny, dtype=torch.float64, device=device) + 0.5) * h
    m2 = mach * mach
    rho2 = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u2 = mach * math.sqrt(gamma) * (1.0 - 1.0 / rho2)
    behind = (x < x_shock)[None, :].expand(ny, nx)
    inside = ((x - centre[0]) ** 2)[None, :] + ((y - centre[1]) ** 2)[:, None] < radius * radius
    W = torch.zeros((5, 1, ny, nx), dtype=torch.float64, device=device)
    W[0, 0] = torch.where(behind, _f64(rho2, device),
                          torch.where(inside, _f64(rho_bubble, device), _f64(1.0, device)))
    W[1, 0] = torch.where(behind, _f64(u2, device), _f64(0.0, device))
    W[4, 0] = torch.where(behind, _f64(p2, device), _f64(1.0, device))
    return W


def uniform(n, rho=1.0, u=0.0, v=0.0, w=0.0, p=1.0, device="cpu"):
    """Constant state."""
    n = tuple(int(v_) for v_ in n)
    W = torch.empty((5, n[2], n[1], n[0]), dtype=torch.float64, device=device)
    for c, val in enumerate((rho, u, v, w, p)):
        W[c] = val
    return W


def random_physical(n, seed, device="cpu", spread=0.25, speed=0.3):
    """Cell-wise independent random states for brute-force comparisons on
    tiny grids: rho and p uniform in [1 - spread, 1 + spread), velocities
    uniform in [-speed, speed)."""
    n = tuple(int(v_) for v_ in n)
    rng = SplitMix64(seed)
    count = n[0] * n[1] * n[2]
    vals = torch.tensor([rng.uniform() for _ in range(5 * count)], dtype=torch.float64)
    vals = vals.reshape(5, n[2], n[1], n[0])
    W = torch.empty_like(vals)
    W[0] = 1.0 - spread + 2.0 * spread * vals[0]
    W[1:4] = speed * (2.0 * vals[1:4] - 1.0)
    W[4] = 1.0 - spread + 2.0 * spread * vals[4]
    return W.to(device)


# Two-dimensional states for the flux-difference workload: float64
# [4, ny, nx] holding (rho, u, v, p) at cell centres of the unit square.

def fourier_modes_2d(rng, count=N_MODES):
    """`count` modes (kx, ky, a, phi) drawn in that order: wavenumbers
    integers in 1..4, amplitudes U(0,1), phases U(0, 2 pi)."""
    modes = []
    for _ in range(count):
        kx = 1 + int(4.0 * rng.uniform())
        ky = 1 + int(4.0 * rng.uniform())
        a = rng.uniform()
        phi = 2.0 * math.pi * rng.uniform()
        modes.append((kx, ky, a, phi))
    return modes


def fourier_field_2d(modes, x, y):
    """f = sum_m (a_m / sum a) cos(2 pi (kx x + ky y) + phi_m), [ny, nx]."""
    total = sum(m[2] for m in modes)
    f = torch.zeros((y.numel(), x.numel()), dtype=torch.float64, device=x.device)
    two_pi = 2.0 * math.pi
    for kx, ky, a, phi in modes:
        # cos(A + B) = cos A cos B - sin A sin B with A along y, B along x:
        # two outer products instead of a cosine per cell
        A = two_pi * ky * y + phi
        B = two_pi * kx * x
        f.addr_(torch.cos(A), torch.cos(B), alpha=a / total)
        f.addr_(torch.sin(A), torch.sin(B), alpha=-a / total)
    return f


def smooth_periodic_2d(n, seed, device="cpu"):
    """Smooth periodic 2D state on an n = (nx, ny) grid: rho = 1 + 0.2 f_rho,
    (u, v) = 0.1 (f_u, f_v), p = 1; three independent 8-mode Fourier fields
    drawn in the order rho, u, v from one SplitMix64 stream."""
    nx, ny = int(n[0]), int(n[1])
    rng = SplitMix64(seed)
    modes = [fourier_modes_2d(rng) for _ in range(3)]
    x = _centres(nx, 0, nx, device)
    y = _centres(ny, 0, ny, device)
    W = torch.empty((4, ny, nx), dtype=torch.float64, device=device)
    W[0] = fourier_field_2d(modes[0], x, y).mul_(0.2).add_(1.0)
    W[1] = fourier_field_2d(modes[1], x, y).mul_(0.1)
    W[2] = fourier_field_2d(modes[2], x, y).mul_(0.1)
    W[3] = 1.0
    return W


def random_physical_2d(n, seed, device="cpu", spread=0.25, speed=0.3):
    """Cell-wise independent random 2D states: rho and p uniform in
    [1 - spread, 1 + spread), velocities uniform in [-speed, speed)."""
    nx, ny = int(n[0]), int(n[1])
    rng = SplitMix64(seed)
    vals = torch.tensor([rng.uniform() for _ in range(4 * nx * ny)], dtype=torch.float64)
    vals = vals.reshape(4, ny, nx)
    W = torch.empty_like(vals)
    W[0] = 1.0 - spread + 2.0 * spread * vals[0]
    W[1:3] = speed * (2.0 * vals[1:3] - 1.0)
    W[3] = 1.0 - spread + 2.0 * spread * vals[3]
    return W.to(device)


def sod_2d(n, axis=0, device="cpu", left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0=0.5):
    """Planar Riemann problem along `axis` (0 = x, 1 = y) on an n = (nx, ny)
    grid: left = (rho, normal velocity, p) where the cell centre < x0."""
    nx, ny = int(n[0]), int(n[1])
    c = _centres((nx, ny)[axis], 0, (nx, ny)[axis], device)
    is_left = (c < x0).reshape((1, nx) if axis == 0 else (ny, 1)).expand(ny, nx)
    W = torch.zeros((4, ny, nx), dtype=torch.float64, device=device)
    W[0] = torch.where(is_left, _f64(left[0], device), _f64(right[0], device))
    W[1 + axis] = torch.where(is_left, _f64(left[1], device), _f64(right[1], device))
    W[3] = torch.where(is_left, _f64(left[2], device), _f64(right[2], device))
    return W


def batch_extents(count=64, seed=42, choices=tuple(range(32, 193, 16))):
    """`count` grid extents (nx, ny, nz), each drawn uniformly from `choices`."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        ext = tuple(choices[int(len(choices) * rng.uniform())] for _ in range(3))
        out.append(ext)
    return out
