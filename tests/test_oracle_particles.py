"""The particle-update oracle against closed forms and a per-particle loop,
and planted mistakes in it caught by these pins."""
import types

import numpy as np
import pytest

from oracle import particles

RNG = np.random.default_rng(3)


def pin_dyadic_closed_form(O):
    """Dyadic positions, velocities and dt: x + v dt is exact; written out."""
    P = np.array([[1.0, -2.5], [0.25, 4.0], [-8.0, 0.0],
                  [3.0, -0.5], [-1.0, 2.0], [0.5, 8.0]])
    got = O.update(P, 0.25)
    want = np.array([[1.75, -2.625], [0.0, 4.5], [-7.875, 2.0],
                     [3.0, -0.5], [-1.0, 2.0], [0.5, 8.0]])
    assert np.array_equal(got, want), got


def pin_zero_dt_is_identity(O):
    P = RNG.standard_normal((6, 17))
    assert np.array_equal(O.update(P, 0.0), P)


def pin_velocities_and_input_unchanged(O):
    P = RNG.standard_normal((6, 9))
    keep = P.copy()
    out = O.update(P, 0.3)
    assert np.array_equal(P, keep)
    assert np.array_equal(out[3:], keep[3:])


def pin_per_particle_loop(O):
    """Each position component moves by its own velocity component."""
    P = RNG.standard_normal((6, 11))
    out = O.update(P, 0.125)
    for k in range(11):
        for d in range(3):
            assert abs(out[d, k] - (P[d, k] + 0.125 * P[3 + d, k])) <= 1e-15 * (1 + abs(out[d, k]))


def pin_two_half_steps(O):
    """Two updates of dt/2 equal one of dt for dyadic data (exact)."""
    P = np.arange(36, dtype=np.float64).reshape(6, 6) / 8.0
    assert np.array_equal(O.update(O.update(P, 0.5), 0.5), O.update(P, 1.0))


ALL_PINS = [pin_dyadic_closed_form, pin_zero_dt_is_identity, pin_velocities_and_input_unchanged,
            pin_per_particle_loop, pin_two_half_steps]


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin):
    pin(particles)


MUTANTS = [
    ("velocity sign", "P[d] = P[d] + P[3 + d] * dt", "P[d] = P[d] - P[3 + d] * dt"),
    ("wrong velocity component", "P[d] = P[d] + P[3 + d] * dt", "P[d] = P[d] + P[3] * dt"),
    ("velocity not scaled by dt", "P[d] = P[d] + P[3 + d] * dt", "P[d] = P[d] + P[3 + d]"),
    ("z not updated", "for d in range(3):", "for d in range(2):"),
    ("updates velocities too", "for d in range(3):\n        P[d] = P[d] + P[3 + d] * dt",
     "for d in range(3):\n        P[d] = P[d] + P[3 + d] * dt\n        P[3 + d] = P[3 + d] * (1 + dt)"),
]


@pytest.fixture(scope="module")
def source():
    with open(particles.__file__) as f:
        return f.read()


def test_mutations_apply_once(source):
    for name, old, new in MUTANTS:
        assert source.count(old) == 1, name


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, name, old, new):
    mod = types.ModuleType("particles_mutant")
    exec(compile(source.replace(old, new, 1), "particles_mutant.py", "exec"), mod.__dict__)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(mod)
        except Exception as e:
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"mutant '{name}' passes every pin"
