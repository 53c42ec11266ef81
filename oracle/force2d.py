"""FP64 CPU oracle for the two-dimensional flux difference with the FORCE flux.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the HIP library.  Plain numpy in FP64, written for
reading, not for speed.

What it computes (Ripple paper, section "Flux Difference in Two
Dimensions"): for every cell of a two-dimensional grid of Euler states, the
sum over both axes of the difference between the numerical fluxes at the
cell's upper and lower face along that axis,

    D_ij = (F_{i+1/2,j} - F_{i-1/2,j}) + (G_{i,j+1/2} - G_{i,j-1/2}),

with each face flux from the FORCE scheme (Toro 1996; Toro, "Riemann Solvers
and Numerical Methods for Fluid Dynamics", section 7.4.2), the average of the
Lax-Friedrichs flux and the flux of the Richtmyer (two-step Lax-Wendroff)
intermediate state.  The first and last cell along each axis read one
padding cell beyond the grid, filled from the boundary condition of that
axis (paper, section "Tensors": padded tensors; constant extrapolation for
transmissive faces, wrap-around for periodic ones).

State: the conserved variables of the two-dimensional Euler equations,
(rho, m_x, m_y, E) with m = rho (u, v), stored planar as U[c, j, i] (j = y,
i = x).  Ideal gas, gamma = 1.4.  lam = (dt/dx, dt/dy) are inputs: the paper
fixes neither the time step nor the cell widths of this benchmark.
"""
import numpy as np

GAMMA = 1.4
TRANSMISSIVE = 0
PERIODIC = 1


def pressure(U):
    """p = (gamma - 1) (E - |m|^2 / (2 rho))."""
    rho, mx, my, E = U
    return (GAMMA - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)


def flux(U, d):
    """Physical flux along axis d (0 = x, 1 = y): (m_d, m_x u_d + p [d == x],
    m_y u_d + p [d == y], u_d (E + p)), u_d = m_d / rho."""
    rho, mx, my, E = U
    un = U[1 + d] / rho
    p = pressure(U)
    F = np.array([U[1 + d], mx * un, my * un, un * (E + p)])
    F[1 + d] = F[1 + d] + p
    return F


def force_flux(UL, UR, lam, d):
    """FORCE flux along axis d between the states UL (lower side) and UR
    (upper side), lam = dt/dx_d:
        Lax-Friedrichs  F_LF = (F(UL) + F(UR)) / 2 + (UL - UR) / (2 lam)
        Richtmyer       U_RI = (UL + UR) / 2 + lam (F(UL) - F(UR)) / 2
        FORCE           F    = (F_LF + F(U_RI)) / 2
    """
    FL = flux(UL, d)
    FR = flux(UR, d)
    F_lf = 0.5 * (FL + FR) + (0.5 / lam) * (UL - UR)
    U_ri = 0.5 * (UL + UR) + (0.5 * lam) * (FL - FR)
    return 0.5 * (F_lf + flux(U_ri, d))


def pad(U, bc):
    """U [4, ny, nx] with a ring of one padding cell, filled per axis:
    transmissive copies the nearest interior cell, periodic the cell at the
    other end.  bc = (bc_x, bc_y)."""
    P = np.empty((4, U.shape[1] + 2, U.shape[2] + 2))
    P[:, 1:-1, 1:-1] = U
    # x first over the interior rows, then y over whole padded rows (corners
    # are never read by a flux difference)
    if bc[0] == PERIODIC:
        P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, -1], U[:, :, 0]
    else:
        P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, 0], U[:, :, -1]
    if bc[1] == PERIODIC:
        P[:, 0, :], P[:, -1, :] = P[:, -2, :], P[:, 1, :]
    else:
        P[:, 0, :], P[:, -1, :] = P[:, 1, :], P[:, -2, :]
    return P


def flux_difference_padded(P, lam):
    """Flux difference of the interior of a padded array P [4, ny + 2, nx + 2]
    whose padding ring holds the neighbours of the boundary cells."""
    # face k along x lies between padded columns k and k + 1, i.e. between
    # cells k - 1 and k, for k = 0 .. nx; likewise along y
    Fx = force_flux(P[:, 1:-1, :-1], P[:, 1:-1, 1:], lam[0], 0)   # [4, ny, nx + 1]
    Gy = force_flux(P[:, :-1, 1:-1], P[:, 1:, 1:-1], lam[1], 1)   # [4, ny + 1, nx]
    return (Fx[:, :, 1:] - Fx[:, :, :-1]) + (Gy[:, 1:, :] - Gy[:, :-1, :])


def flux_difference(U, lam, bc):
    """D [4, ny, nx] for the conserved state U [4, ny, nx] (FP64)."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim != 3 or U.shape[0] != 4 or U.shape[1] < 1 or U.shape[2] < 1:
        raise ValueError("U must be [4, ny, nx] with nx, ny >= 1")
    return flux_difference_padded(pad(U, bc), lam)


def prim_to_cons(W):
    """Primitive (rho, u, v, p) [4, ...] to conserved (rho, rho u, rho v, E),
    E = p / (gamma - 1) + rho (u^2 + v^2) / 2."""
    rho, u, v, p = np.asarray(W, dtype=np.float64)
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])
