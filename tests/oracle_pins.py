"""Pins that tie the FP64 oracle to the mathematics, independent of itself.

Each pin is a function taking an ``oracle.Oracle`` and raising AssertionError
when the oracle disagrees with a closed form, a textbook value, an exact
invariant of the scheme, or the exact Riemann solution.  The pins are chosen
so that a plausible mistake anywhere in the oracle (a dropped term, a wrong
sign or index, a transposed operand) fails at least one of them;
``test_oracle_mutants.py`` plants such mistakes and checks exactly that.
"""
import json
import math
import os

import numpy as np

from oracle import OracleNonPhysical, exact_riemann
from paper_2104_08571_amd import initial_states as ist

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GAMMA = 1.4


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def cons(rho, u, v, w, p):
    """Conserved state from primitives, written out independently of the oracle."""
    return np.array([rho, rho * u, rho * v, rho * w,
                     p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def unit_dx(U):
    return [1.0 / U.shape[3], 1.0 / U.shape[2], 1.0 / U.shape[1]]


# --------------------------------------------------------------------------
# point functions
# --------------------------------------------------------------------------

def pin_minmod_table(o):
    """minmod: same-sign arguments give the smaller magnitude, else zero."""
    cases = [((1.0, 2.0), 1.0), ((2.0, 1.0), 1.0), ((-1.0, -2.0), -1.0),
             ((-2.0, -1.0), -1.0), ((1.0, -1.0), 0.0), ((-3.0, 2.0), 0.0),
             ((0.0, 5.0), 0.0), ((5.0, 0.0), 0.0), ((0.0, -5.0), 0.0),
             ((3.0, 3.0), 3.0), ((-3.0, -3.0), -3.0),
             ((1e-300, 1e-300), 1e-300), ((-1e-300, -2e-300), -1e-300)]
    for (a, b), want in cases:
        got = o.minmod(a, b)
        assert got == want, f"minmod({a}, {b}) = {got}, want {want}"


def pin_flux_hand_values(o):
    """F_d on a hand-computed state (values derived in tests/golden/flux_hand.json)."""
    g = golden("flux_hand.json")
    U = np.array(g["U"])
    for d, key in enumerate(("F_x", "F_y", "F_z")):
        F = o.flux(U, d)
        np.testing.assert_allclose(F, g[key], rtol=1e-14, atol=1e-14,
                                   err_msg=f"flux along axis {d}")


def pin_eos_roundtrip(o):
    """primitive -> conserved -> primitive returns the input to a few ulp,
    and the energy matches p/(gamma-1) + rho |u|^2 / 2."""
    W = ist.random_physical((3, 4, 5), seed=7).numpy()
    U = o.prim_to_cons(W)
    W2 = o.cons_to_prim(U)
    np.testing.assert_allclose(W2, W, rtol=1e-14, atol=1e-15)
    rho, u, v, w, p = W
    E = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)
    np.testing.assert_allclose(U[4], E, rtol=1e-12)
    np.testing.assert_allclose(U[1], rho * u, rtol=1e-15)


def pin_hllc_consistency(o):
    """HLLC(U, U) = F(U) for any state and axis (consistency)."""
    for st in [(1.0, 0.3, -0.2, 0.1, 1.0), (0.5, -2.0, 0.4, 0.0, 0.2),
               (2.0, 5.0, 1.0, -1.0, 3.0), (0.125, -0.1, 0.0, 0.7, 0.1)]:
        U = cons(*st)
        for d in range(3):
            np.testing.assert_allclose(o.hllc(U, U, d), o.flux(U, d), rtol=1e-13,
                                       atol=1e-13, err_msg=f"state {st} axis {d}")


def pin_hllc_stationary_contact(o):
    """Stationary contact (u = 0, equal p, different rho): S* = 0, so the
    mass and energy fluxes vanish and the normal momentum flux equals p."""
    for d in range(3):
        UL = cons(1.0, 0.0, 0.0, 0.0, 0.7)
        UR = cons(0.125, 0.0, 0.0, 0.0, 0.7)
        F = o.hllc(UL, UR, d)
        assert abs(F[0]) < 1e-15 and abs(F[4]) < 1e-15, F
        want = np.zeros(3)
        want[d] = 0.7
        np.testing.assert_allclose(F[1:4], want, rtol=1e-14, atol=1e-15)


def pin_hllc_moving_contact(o):
    """An isolated contact moving at speed u (equal u and p): HLLC resolves
    it exactly, so the flux is the upwind state's physical flux, here
    computed independently from the definition."""
    for speed in (0.4, -0.3):
        rho_l, rho_r, p, vt = 1.0, 0.25, 0.9, 0.2
        UL = cons(rho_l, speed, vt, -vt, p)
        UR = cons(rho_r, speed, -vt, vt, p)
        up = UL if speed > 0 else UR
        rho = up[0]
        want = np.array([rho * speed, rho * speed * speed + p, up[2] * speed, up[3] * speed,
                         speed * (up[4] + p)])
        np.testing.assert_allclose(o.hllc(UL, UR, 0), want, rtol=1e-13, atol=1e-14)


def pin_hllc_supersonic(o):
    """Supersonic flow: S_L >= 0 selects F(U_L), S_R <= 0 selects F(U_R)."""
    UL = cons(1.0, 4.0, 0.1, 0.2, 1.0)
    UR = cons(0.5, 3.5, -0.1, 0.0, 0.8)
    F = o.hllc(UL, UR, 0)
    assert np.array_equal(F, o.flux(UL, 0))
    UL = cons(1.0, -4.0, 0.1, 0.2, 1.0)
    UR = cons(0.5, -3.5, -0.1, 0.0, 0.8)
    F = o.hllc(UL, UR, 0)
    assert np.array_equal(F, o.flux(UR, 0))


def pin_hllc_mirror(o):
    """Reflecting the face (swap sides, negate normal velocity) negates the
    mass, tangential-momentum and energy fluxes and keeps the normal one."""
    UL = cons(1.0, 0.3, 0.2, -0.1, 1.0)
    UR = cons(0.4, -0.2, 0.5, 0.3, 0.3)
    for d in range(3):
        F = o.hllc(UL, UR, d)
        ml, mr = UR.copy(), UL.copy()
        ml[1 + d] *= -1
        mr[1 + d] *= -1
        G = o.hllc(ml, mr, d)
        sign = -np.ones(5)
        sign[1 + d] = 1.0
        np.testing.assert_allclose(G, sign * F, rtol=1e-13, atol=1e-14, err_msg=f"axis {d}")


def pin_hllc_sod_closed_form(o):
    """HLLC on Sod's data, worked by hand from Toro eqs. 10.37, 10.39, 10.26
    with Davis speeds.  c_L = sqrt(1.4), c_R = sqrt(1.12), so S_L = -sqrt(1.4),
    S_R = sqrt(1.4); S* = (0.1 - 1) / (-sqrt(1.4) - 0.125 sqrt(1.4))
    = 0.8 / sqrt(1.4) > 0, so the flux is F_L + S_L (U*_L - U_L) with the
    star factor rho_L (S_L - u_L) / (S_L - S*) = 1.4 / 2.2 = 7/11 and
    E*_L = (7/11) (2.5 + S* (S* - 1/sqrt(1.4))) = 16.7 / 11.  Hence
    F = ((4/11) sqrt(1.4), 5.4/11, 0, 0, (10.8/11) sqrt(1.4)), along every axis."""
    s = math.sqrt(1.4)
    want_n = [4.0 / 11.0 * s, 5.4 / 11.0, 10.8 / 11.0 * s]
    for d in range(3):
        vel = [0.0, 0.0, 0.0]
        UL = cons(1.0, *vel, 1.0)
        UR = cons(0.125, *vel, 0.1)
        F = o.hllc(UL, UR, d)
        want = np.zeros(5)
        want[0], want[1 + d], want[4] = want_n
        np.testing.assert_allclose(F, want, rtol=1e-14, atol=1e-15, err_msg=f"axis {d}")


def pin_exact_riemann_toro(o=None):
    """The exact solver reproduces Toro's tabulated Sod star values."""
    g = golden("sod_exact_toro.json")
    ws = exact_riemann.wave_structure(*g["left"], *g["right"])
    for key, want in g["star"].items():
        assert abs(ws[key] - want) < 6e-6, (key, ws[key], want)


# --------------------------------------------------------------------------
# grid functions
# --------------------------------------------------------------------------

def pin_dt_sod_closed_form(o):
    """Sod initial state: S_x = S_y = S_z = sqrt(1.4), so for 32^3 and CFL 0.9
    dt_0 = 0.9 / (32 sqrt(1.4))."""
    U = o.prim_to_cons(ist.sod((32, 32, 32)).numpy())
    S = o.max_wavespeed(U)
    np.testing.assert_allclose(S, [math.sqrt(1.4)] * 3, rtol=1e-15)
    dt = o.dt(S, [1 / 32] * 3, 0.9)
    assert abs(dt - 0.9 / (32 * math.sqrt(1.4))) < 1e-16
    _, t, dts = o.run(U, 1, [1 / 32] * 3, [0, 0, 0], cfl=0.9)
    assert abs(dts[0] - 0.9 / (32 * math.sqrt(1.4))) < 1e-16


def pin_max_wavespeed_closed_form(o):
    """A uniform moving state has S_d = |u_d| + c exactly."""
    W = ist.uniform((4, 3, 5), rho=0.8, u=-0.3, v=0.5, w=0.0, p=1.3).numpy()
    S = o.max_wavespeed(o.prim_to_cons(W))
    c = math.sqrt(1.4 * 1.3 / 0.8)
    np.testing.assert_allclose(S, [0.3 + c, 0.5 + c, c], rtol=1e-14)


def pin_uniform_preserved(o):
    """A uniform state is preserved bitwise, for both boundary conditions."""
    W = ist.uniform((6, 5, 4), rho=1.3, u=0.4, v=-0.2, w=0.7, p=2.1).numpy()
    U = o.prim_to_cons(W)
    for bc in ([0, 0, 0], [1, 1, 1], [0, 1, 0]):
        U2, _, _ = o.run(U, 3, unit_dx(U), bc, cfl=0.9)
        assert np.array_equal(U2, U), f"bc {bc}"


def pin_periodic_conservation(o, n=24, steps=10):
    """Periodic grid: the totals of all five conserved variables are
    unchanged to round-off (fluxes telescope)."""
    U = o.prim_to_cons(ist.smooth_periodic((n, n, n), seed=2104).numpy())
    U2, _, _ = o.run(U, steps, unit_dx(U), [1, 1, 1], cfl=0.9)
    assert not np.array_equal(U2, U)
    s0 = U.reshape(5, -1).sum(1)
    s1 = U2.reshape(5, -1).sum(1)
    scale = np.abs(U).reshape(5, -1).sum(1)
    rel = np.abs(s1 - s0) / scale
    assert rel.max() < 1e-13, rel


def pin_sod_momentum_identity(o, n=64, steps=12):
    """Transmissive Sod: while the waves are far from both ends the boundary
    faces carry the fluxes of the end states, so sum(m_x) dV grows by
    (p_L - p_R) dt per step and mass and energy totals are unchanged."""
    U = o.prim_to_cons(ist.sod((n, 2, 2)).numpy())
    U2, t, dts = o.run(U, steps, unit_dx(U), [0, 0, 0], cfl=0.9)
    assert t < 0.5 / 1.8  # shock has not reached the right end
    dV = 1.0 / (n * 2 * 2)
    mom = U2[1].sum() * dV
    assert abs(mom - (1.0 - 0.1) * t) < 1e-13, (mom, 0.9 * t)
    for c in (0, 4):
        assert abs(U2[c].sum() - U[c].sum()) * dV < 1e-13


def pin_planar_equals_1d(o):
    """A planar problem in N x 3 x 2 equals the same problem in N x 1 x 1
    bitwise: the transverse sweeps see uniform data and are exact no-ops."""
    W = ist.sod((40, 3, 2)).numpy()
    W1 = ist.sod((40, 1, 1)).numpy()
    U3, t3, _ = o.run(o.prim_to_cons(W), 8, [1 / 40, 1 / 3, 1 / 2], [0, 1, 0])
    U1, t1, _ = o.run(o.prim_to_cons(W1), 8, [1 / 40, 1.0, 1.0], [0, 0, 0])
    assert t3 == t1
    for j in range(3):
        for k in range(2):
            assert np.array_equal(U3[:, k, j, :], U1[:, 0, 0, :])


def pin_sod_axis_permutation(o, n=24, steps=6):
    """Sod along y or z is the Sod run along x, transposed, bitwise."""
    Ux, _, _ = o.run(o.prim_to_cons(ist.sod((n, 4, 4), axis=0).numpy()), steps,
                     [1 / n, 1 / 4, 1 / 4], [0, 0, 0])
    Uy, _, _ = o.run(o.prim_to_cons(ist.sod((4, n, 4), axis=1).numpy()), steps,
                     [1 / 4, 1 / n, 1 / 4], [0, 0, 0])
    Uz, _, _ = o.run(o.prim_to_cons(ist.sod((4, 4, n), axis=2).numpy()), steps,
                     [1 / 4, 1 / 4, 1 / n], [0, 0, 0])
    # state [c, z, y, x]; compare along the sweep axis, normal momentum with normal
    ref = Ux[:, 0, 0, :]
    y_line = Uy[:, 0, :, 0][[0, 2, 1, 3, 4]]
    z_line = Uz[:, :, 0, 0][[0, 3, 2, 1, 4]]
    assert np.array_equal(y_line, ref)
    assert np.array_equal(z_line, ref)


def pin_general_axis_permutation(o):
    """Swapping the x and y axes of general 3D data, together with the sweep
    order, swaps the result bitwise; a cyclic permutation agrees to round-off."""
    W = ist.smooth_periodic((10, 12, 8), seed=5).numpy()
    U = o.prim_to_cons(W)
    dx = unit_dx(U)
    R, _, _ = o.run(U, 3, dx, [1, 1, 1], order=(0, 1, 2))
    # swap x <-> y: array axes [c, z, y, x] -> [c, z, x, y], momentum 1 <-> 2
    Us = U.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]].copy()
    Rs, _, _ = o.run(Us, 3, [dx[1], dx[0], dx[2]], [1, 1, 1], order=(1, 0, 2))
    assert np.array_equal(Rs.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]], R)
    # cyclic (x, y, z) -> (y, z, x): new x = old y, new y = old z, new z = old x
    Uc = U.transpose(0, 3, 1, 2)[[0, 2, 3, 1, 4]].copy()
    Rc, _, _ = o.run(Uc, 3, [dx[1], dx[2], dx[0]], [1, 1, 1], order=(2, 0, 1))
    back = Rc.transpose(0, 2, 3, 1)[[0, 3, 1, 2, 4]]
    np.testing.assert_allclose(back, R, rtol=1e-13, atol=1e-14)


def pin_mirror_symmetry(o):
    """Reflecting x (reverse the index, negate m_x) reflects the result."""
    W = ist.smooth_periodic((12, 6, 5), seed=11).numpy()
    U = o.prim_to_cons(W)
    R, _, _ = o.run(U, 3, unit_dx(U), [0, 1, 0])
    M = U[:, :, :, ::-1].copy()
    M[1] *= -1
    RM, _, _ = o.run(M, 3, unit_dx(U), [0, 1, 0])
    back = RM[:, :, :, ::-1].copy()
    back[1] *= -1
    np.testing.assert_allclose(back, R, rtol=1e-12, atol=1e-13)


def pin_sod_converges_to_exact(o):
    """Planar Sod to t = 0.2: the L1 density error against the exact
    solution falls with resolution at an order between 0.6 and 1.1, and is
    small in absolute terms."""
    errs = []
    ns = (100, 200, 400)
    for n in ns:
        U, t, _ = o.run(o.prim_to_cons(ist.sod((n, 1, 1)).numpy()), 100000,
                        [1 / n, 1.0, 1.0], [0, 0, 0], cfl=0.9, t_end=0.2)
        assert abs(t - 0.2) < 1e-14
        rho_ex, _, _ = exact_riemann.cell_averages(n, t, 0.5, (1, 0, 1), (0.125, 0, 0.1))
        errs.append(np.abs(U[0, 0, 0, :] - rho_ex).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(0.6 <= q <= 1.1 for q in orders), (errs, orders)
    assert errs[-1] < 3e-3, errs


def pin_smooth_wave_second_order(o):
    """Smooth entropy wave (rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1) on a
    periodic line: the exact solution is the shifted profile.  The L1 error
    falls at an observed order above 1.5 (second order away from extrema)."""
    errs = []
    for n in (32, 64, 128):
        xc = (np.arange(n) + 0.5) / n
        W = np.zeros((5, 1, 1, n))
        W[0, 0, 0] = 1.0 + 0.2 * np.sin(2 * np.pi * xc)
        W[1] = 1.0
        W[4] = 1.0
        U, t, _ = o.run(o.prim_to_cons(W), 100000, [1 / n, 1.0, 1.0], [1, 1, 1],
                        cfl=0.8, t_end=0.5)
        # exact cell average of 1 + 0.2 sin(2 pi (x - t))
        lo, hi = np.arange(n) / n - t, (np.arange(n) + 1) / n - t
        avg = 1.0 + 0.2 * (np.cos(2 * np.pi * lo) - np.cos(2 * np.pi * hi)) / (2 * np.pi) * n
        errs.append(np.abs(U[0, 0, 0] - avg).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 1.5, (errs, orders)


def pin_sod_32_against_exact(o):
    """The 32^3 Sod run (CFL 0.9, 20 steps, transmissive) against the exact
    solution at its own final time: locked bounds on the L1 errors of
    density, velocity and pressure along x."""
    g = golden("sod32_bounds.json")
    U, t, dts = o.run(o.prim_to_cons(ist.sod((32, 32, 32)).numpy()), 20,
                      [1 / 32] * 3, [0, 0, 0], cfl=0.9)
    W = o.cons_to_prim(U)
    rho_ex, u_ex, p_ex = exact_riemann.cell_averages(32, t, 0.5, (1, 0, 1), (0.125, 0, 0.1))
    # the run is planar: every (j, k) line is identical
    assert np.array_equal(U[:, 5, 7, :], U[:, 0, 0, :])
    errs = {"rho": np.abs(W[0, 0, 0] - rho_ex).mean(),
            "u": np.abs(W[1, 0, 0] - u_ex).mean(),
            "p": np.abs(W[4, 0, 0] - p_ex).mean()}
    for k, v in errs.items():
        assert v < g["l1_max"][k], (k, v, g["l1_max"][k])
    assert abs(t - g["t_final"]) < 1e-12, (t, g["t_final"])


def pin_nonphysical_detected(o):
    """A negative pressure in the input is reported with its cell."""
    W = ist.uniform((5, 4, 3)).numpy()
    W[4, 2, 1, 3] = -0.5
    U = o.prim_to_cons(W)
    try:
        o.run(U, 1, unit_dx(U), [0, 0, 0])
    except OracleNonPhysical as e:
        assert e.info[0] == 0 and e.info[2:5] == [3, 1, 2], e.info
    else:
        raise AssertionError("negative pressure not reported")


ALL_PINS = [
    pin_minmod_table, pin_flux_hand_values, pin_eos_roundtrip, pin_hllc_consistency,
    pin_hllc_stationary_contact, pin_hllc_moving_contact, pin_hllc_supersonic,
    pin_hllc_mirror, pin_hllc_sod_closed_form, pin_dt_sod_closed_form,
    pin_max_wavespeed_closed_form, pin_uniform_preserved, pin_periodic_conservation,
    pin_sod_momentum_identity, pin_planar_equals_1d, pin_sod_axis_permutation,
    pin_general_axis_permutation, pin_mirror_symmetry, pin_sod_converges_to_exact,
    pin_smooth_wave_second_order, pin_sod_32_against_exact, pin_nonphysical_detected,
]
