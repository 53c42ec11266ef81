"""The 2D FORCE flux-difference oracle against its pins, and planted mistakes
in it caught by them.

Each mutant is the oracle's source with one plausible mistake (a dropped
term, a wrong sign or index, a transposed operand, a wrong boundary fill),
executed as its own module; at least one pin must fail for each.
"""
import types

import pytest

import force2d_pins as P
from oracle import force2d


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=[p.__name__ for p in P.ALL_PINS])
def test_pin(pin):
    pin(force2d)


MUTANTS = [
    ("pressure kinetic sign", "(E - 0.5 * (mx * mx + my * my) / rho)",
     "(E + 0.5 * (mx * mx + my * my) / rho)"),
    ("pressure drops m_y^2", "0.5 * (mx * mx + my * my) / rho", "0.5 * (mx * mx) / rho"),
    ("flux pressure on wrong component", "F[1 + d] = F[1 + d] + p", "F[1] = F[1] + p"),
    ("energy flux drops p", "un * (E + p)", "un * E"),
    ("tangential flux uses m_x", "mx * un, my * un", "mx * un, mx * un"),
    ("mass flux uses the other momentum", "F = np.array([U[1 + d],", "F = np.array([U[2 - d],"),
    ("Lax-Friedrichs diffusion sign", "(0.5 / lam) * (UL - UR)", "(0.5 / lam) * (UR - UL)"),
    ("Lax-Friedrichs diffusion times lam", "(0.5 / lam) * (UL - UR)", "(0.5 * lam) * (UL - UR)"),
    ("Richtmyer flux sign", "(0.5 * lam) * (FL - FR)", "(0.5 * lam) * (FR - FL)"),
    ("Richtmyer drops the flux term", "U_ri = 0.5 * (UL + UR) + (0.5 * lam) * (FL - FR)",
     "U_ri = 0.5 * (UL + UR)"),
    ("FORCE weights", "return 0.5 * (F_lf + flux(U_ri, d))", "return 0.5 * F_lf + flux(U_ri, d)"),
    ("FORCE is Lax-Friedrichs only", "return 0.5 * (F_lf + flux(U_ri, d))", "return F_lf"),
    ("x faces transposed operands", "force_flux(P[:, 1:-1, :-1], P[:, 1:-1, 1:], lam[0], 0)",
     "force_flux(P[:, 1:-1, 1:], P[:, 1:-1, :-1], lam[0], 0)"),
    ("y faces use lam_x", "P[:, 1:, 1:-1], lam[1], 1)", "P[:, 1:, 1:-1], lam[0], 1)"),
    ("y difference sign", "(Gy[:, 1:, :] - Gy[:, :-1, :])", "(Gy[:, :-1, :] - Gy[:, 1:, :])"),
    ("periodic x padding swapped", "P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, -1], U[:, :, 0]",
     "P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, 0], U[:, :, -1]"),
    ("transmissive y padding swapped", "P[:, 0, :], P[:, -1, :] = P[:, 1, :], P[:, -2, :]",
     "P[:, 0, :], P[:, -1, :] = P[:, -2, :], P[:, 1, :]"),
    ("transmissive x padding from the second cell",
     "P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, 0], U[:, :, -1]",
     "P[:, 1:-1, 0], P[:, 1:-1, -1] = U[:, :, min(1, U.shape[2] - 1)], U[:, :, -1]"),
    ("energy from primitives drops 1/2", "0.5 * rho * (u * u + v * v)", "rho * (u * u + v * v)"),
]


@pytest.fixture(scope="module")
def source():
    with open(force2d.__file__) as f:
        return f.read()


def test_mutations_apply_once(source):
    for name, old, new in MUTANTS:
        assert source.count(old) == 1, f"mutation '{name}' does not match exactly once"
        assert old != new


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, name, old, new):
    mod = types.ModuleType("force2d_mutant")
    exec(compile(source.replace(old, new, 1), "force2d_mutant.py", "exec"), mod.__dict__)
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin(mod)
        except Exception as e:  # any failure counts
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"mutant '{name}' passes every pin"
