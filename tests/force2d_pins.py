"""Pins that tie the 2D FORCE flux-difference oracle to the mathematics.

Each pin takes the oracle module (``oracle.force2d`` or a planted mutant of
it) and raises AssertionError when the oracle disagrees with a hand-derived
value, a closed form or an exact invariant.  None of them re-evaluates the
oracle's own formulas: the flux is checked against the textbook Jacobian
(the Euler flux is homogeneous of degree one, F(U) = A(U) U), the FORCE flux
against its linearisation in terms of that Jacobian, the assembly against
telescoping sums, symmetries and a per-cell loop with explicit neighbours.
``test_oracle_force2d.py`` runs them on the oracle and on planted mistakes.
"""
import json
import os

import numpy as np

from paper_2104_08571_amd import initial_states as ist

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GAMMA = 1.4


def cons(rho, u, v, p):
    """Conserved state from primitives, written out independently of the oracle."""
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def jacobian(U, d):
    """Flux Jacobian dF_d/dU of the 2D Euler equations in conserved variables
    (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics",
    section 3.1), in terms of u, v and the total enthalpy H = (E + p)/rho."""
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    q2 = u * u + v * v
    p = (GAMMA - 1.0) * (E - 0.5 * rho * q2)
    H = (E + p) / rho
    g1 = GAMMA - 1.0
    if d == 0:
        return np.array([
            [0.0, 1.0, 0.0, 0.0],
            [0.5 * g1 * q2 - u * u, (3.0 - GAMMA) * u, -g1 * v, g1],
            [-u * v, v, u, 0.0],
            [u * (0.5 * g1 * q2 - H), H - g1 * u * u, -g1 * u * v, GAMMA * u]])
    return np.array([
        [0.0, 0.0, 1.0, 0.0],
        [-u * v, v, u, 0.0],
        [0.5 * g1 * q2 - v * v, -g1 * u, (3.0 - GAMMA) * v, g1],
        [v * (0.5 * g1 * q2 - H), -g1 * u * v, H - g1 * v * v, GAMMA * v]])


def random_states(seed, count):
    W = ist.random_physical_2d((count, 1), seed).numpy()[:, 0, :]
    return [cons(*W[:, k]) for k in range(count)]


def state_2d(shape, seed):
    """Conserved [4, ny, nx] from the seeded random primitive generator."""
    W = ist.random_physical_2d(shape, seed).numpy()
    return cons(W[0], W[1], W[2], W[3])


# --------------------------------------------------------------------------
# point functions
# --------------------------------------------------------------------------

def pin_force_hand_values(O):
    """FORCE fluxes derived by hand in exact arithmetic (Sod pair along x,
    shearing pair along y)."""
    with open(os.path.join(GOLDEN, "force_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        F = O.force_flux(np.array(c["UL"]), np.array(c["UR"]), c["lam"], c["axis"])
        assert np.allclose(F, c["F"], rtol=1e-14, atol=1e-15), (c["name"], F, c["F"])


def pin_prim_to_cons_hand(O):
    """(rho, u, v, p) = (2, 1, 1/2, 1): m = (2, 1), E = 1/0.4 + 2 (1 + 1/4)/2 = 3.75."""
    U = O.prim_to_cons(np.array([2.0, 1.0, 0.5, 1.0]))
    assert np.allclose(U, [2.0, 2.0, 1.0, 3.75], rtol=1e-15), U


def pin_flux_homogeneous(O):
    """F_d(U) = A_d(U) U (homogeneity of the Euler flux) for random states,
    both axes."""
    for U in random_states(5, 12):
        for d in (0, 1):
            want = jacobian(U, d) @ U
            assert np.allclose(O.flux(U, d), want, rtol=1e-13, atol=1e-14), (d, U)


def pin_force_consistency(O):
    """FORCE(U, U) = F(U): the Lax-Friedrichs and Richtmyer parts both reduce
    to the physical flux for equal states."""
    for U in random_states(6, 8):
        for d in (0, 1):
            for lam in (0.1, 0.7):
                want = jacobian(U, d) @ U
                assert np.allclose(O.force_flux(U, U, lam, d), want, rtol=1e-13, atol=1e-14)


def pin_force_linearisation(O):
    """For UL = U0 + e a, UR = U0 + e b the FORCE flux is, to first order in e,
        F(U0) + e [A (a + b)/2 + (a - b)/(4 lam) + lam A^2 (a - b)/4]
    (the Lax-Friedrichs part contributes A (a+b)/2 + (a-b)/(2 lam), the
    Richtmyer state U0 + e [(a+b)/2 + lam A (a-b)/2]).  The central difference
    in e cancels the second-order term."""
    rng = np.random.default_rng(11)
    for U0 in random_states(7, 6):
        for d in (0, 1):
            for lam in (0.2, 0.9):
                a, b = rng.standard_normal(4), rng.standard_normal(4)
                A = jacobian(U0, d)
                want = 0.5 * A @ (a + b) + (a - b) / (4.0 * lam) + lam * (A @ (A @ (a - b))) / 4.0
                e = 1e-5
                got = (O.force_flux(U0 + e * a, U0 + e * b, lam, d)
                       - O.force_flux(U0 - e * a, U0 - e * b, lam, d)) / (2.0 * e)
                assert np.allclose(got, want, rtol=1e-6, atol=1e-7), (d, lam, got, want)


# --------------------------------------------------------------------------
# assembly of the flux difference
# --------------------------------------------------------------------------

def pin_uniform_zero(O):
    """A constant state has zero flux difference, exactly, for either boundary."""
    U = np.broadcast_to(cons(1.3, 0.2, -0.1, 0.8)[:, None, None], (4, 5, 7)).copy()
    for bc in ((0, 0), (1, 1), (0, 1)):
        D = O.flux_difference(U, (0.3, 0.4), bc)
        assert D.shape == (4, 5, 7)
        assert np.all(D == 0.0), bc


def pin_periodic_telescoping(O):
    """With periodic faces every face flux enters two cells with opposite
    signs: the flux differences sum to zero."""
    U = state_2d((9, 7), 21)
    D = O.flux_difference(U, (0.3, 0.2), (1, 1))
    scale = np.abs(D).sum(axis=(1, 2)) + 1.0
    assert np.all(np.abs(D.sum(axis=(1, 2))) < 1e-13 * scale), D.sum(axis=(1, 2))


def pin_transmissive_boundary_sum(O):
    """With transmissive faces the outermost face fluxes are FORCE(U_b, U_b)
    = F(U_b) of the boundary cells, so the sum over all cells is the sum of
    the boundary cells' physical fluxes (written with the Jacobian form)."""
    U = state_2d((6, 5), 22)
    for bc, lam in (((0, 0), (0.3, 0.2)), ((0, 1), (0.25, 0.5)), ((1, 0), (0.4, 0.1))):
        D = O.flux_difference(U, lam, bc)
        want = np.zeros(4)
        if bc[0] == 0:
            for j in range(U.shape[1]):
                want += jacobian(U[:, j, -1], 0) @ U[:, j, -1] - jacobian(U[:, j, 0], 0) @ U[:, j, 0]
        if bc[1] == 0:
            for i in range(U.shape[2]):
                want += jacobian(U[:, -1, i], 1) @ U[:, -1, i] - jacobian(U[:, 0, i], 1) @ U[:, 0, i]
        assert np.allclose(D.sum(axis=(1, 2)), want, rtol=1e-12, atol=1e-12), (bc, D.sum(axis=(1, 2)), want)


def pin_mirror_x(O):
    """Reflecting x (i -> nx - 1 - i, m_x -> -m_x) reflects the result, with
    its m_x component negated and the others' x-part sign flipped back:
    D'(i) = M D(nx - 1 - i), M = diag(1, -1, 1, 1)."""
    U = state_2d((7, 5), 23)
    M = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None]
    Um = (U * M)[:, :, ::-1].copy()
    for bc in ((0, 0), (1, 1), (0, 1)):
        D = O.flux_difference(U, (0.3, 0.2), bc)
        Dm = O.flux_difference(Um, (0.3, 0.2), bc)
        assert np.allclose(Dm, (D * M)[:, :, ::-1], rtol=1e-12, atol=1e-13), bc


def pin_transpose(O):
    """Swapping the axes (and m_x with m_y, lam_x with lam_y, bc_x with bc_y)
    transposes the result with m_x and m_y swapped."""
    U = state_2d((6, 4), 24)
    Ut = U[[0, 2, 1, 3]].transpose(0, 2, 1).copy()
    D = O.flux_difference(U, (0.3, 0.2), (0, 1))
    Dt = O.flux_difference(Ut, (0.2, 0.3), (1, 0))
    assert np.allclose(Dt, D[[0, 2, 1, 3]].transpose(0, 2, 1), rtol=1e-12, atol=1e-13)


def _neighbour(k, n, bc):
    """Index of cell k along an axis of n cells, k in -1 .. n, per boundary."""
    if 0 <= k < n:
        return k
    if bc == 1:
        return k % n
    return 0 if k < 0 else n - 1


def pin_loop_brute_force(O):
    """Per-cell loop: each cell's four faces from its explicit neighbours
    (boundary mapping written out here), on grids down to a single cell."""
    for shape, bc, seed in (((3, 4), (0, 1), 25), ((4, 3), (1, 0), 26), ((1, 1), (0, 0), 27),
                            ((2, 1), (1, 1), 28), ((1, 3), (1, 0), 29)):
        U = state_2d(shape, seed)
        lam = (0.35, 0.15)
        nx, ny = shape
        D = O.flux_difference(U, lam, bc)
        for j in range(ny):
            for i in range(nx):
                c = U[:, j, i]
                xm = U[:, j, _neighbour(i - 1, nx, bc[0])]
                xp = U[:, j, _neighbour(i + 1, nx, bc[0])]
                ym = U[:, _neighbour(j - 1, ny, bc[1]), i]
                yp = U[:, _neighbour(j + 1, ny, bc[1]), i]
                want = (O.force_flux(c, xp, lam[0], 0) - O.force_flux(xm, c, lam[0], 0)) \
                    + (O.force_flux(c, yp, lam[1], 1) - O.force_flux(ym, c, lam[1], 1))
                assert np.allclose(D[:, j, i], want, rtol=1e-13, atol=1e-14), (shape, bc, i, j)


ALL_PINS = [pin_force_hand_values, pin_prim_to_cons_hand, pin_flux_homogeneous,
            pin_force_consistency, pin_force_linearisation, pin_uniform_zero,
            pin_periodic_telescoping, pin_transmissive_boundary_sum, pin_mirror_x,
            pin_transpose, pin_loop_brute_force]
