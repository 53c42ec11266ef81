"""Planted mistakes in the oracle are caught by the pins.

Each mutant is a copy of the oracle source with one plausible mistake (a
dropped term, a wrong sign, a wrong index, a transposed operand), built into
its own library in a temporary directory.  The test asserts that at least one
pin of ``oracle_pins`` fails for every mutant: the pins do not merely agree
with whatever the oracle happens to compute.
"""
import os
import shutil

import pytest

import oracle_pins as P
from oracle import Oracle, load
from oracle import build as oracle_build

MUTANTS = [
    ("pressure kinetic sign", "(GAMMA - 1.0) * (U[4] - kinetic)", "(GAMMA - 1.0) * (U[4] + kinetic)"),
    ("pressure drops m_z^2", "0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho",
     "0.5 * (U[1] * U[1] + U[2] * U[2]) / rho"),
    ("flux pressure on wrong component", "F[1 + d] += p;", "F[1] += p;"),
    ("energy flux drops p", "F[4] = un * (U[4] + p);", "F[4] = un * U[4];"),
    ("minmod positive picks max", "if (a > 0.0 && b > 0.0) return a < b ? a : b;",
     "if (a > 0.0 && b > 0.0) return a > b ? a : b;"),
    ("minmod negative picks min", "if (a < 0.0 && b < 0.0) return a > b ? a : b;",
     "if (a < 0.0 && b < 0.0) return a < b ? a : b;"),
    ("star tangential momentum not divided by rho",
     "Us[1 + a] = factor * (U[1 + a] / rho);", "Us[1 + a] = factor * U[1 + a];"),
    ("star energy sign", "(Ss - un) * (Ss + p / (rho * (S - un)))",
     "(Ss - un) * (Ss - p / (rho * (S - un)))"),
    ("star normal momentum uses u", "Us[1 + d] = factor * Ss;", "Us[1 + d] = factor * un;"),
    ("Davis S_L wrong index", "double SL = fmin(uL - cL, uR - cR);",
     "double SL = fmin(uL - cL, uL - cR);"),
    ("Davis S_R sign", "double SR = fmax(uL + cL, uR + cR);", "double SR = fmax(uL + cL, uR - cR);"),
    ("contact speed pressure sign", "double Ss = (pR - pL +", "double Ss = (pL - pR +"),
    ("star flux transposed operand", "F[c] = FL[c] + SL * (Us[c] - UL[c]);",
     "F[c] = FL[c] + SL * (Us[c] - UR[c]);"),
    ("branch test uses S_R", "} else if (0.0 <= Ss) {", "} else if (0.0 <= SR) {"),
    ("half step sign", "double h = 0.5 * lam * (FLx[c] - FRx[c]);",
     "double h = 0.5 * lam * (FRx[c] - FLx[c]);"),
    ("slope not halved", "UL[c] = U0[c] - 0.5 * slope;", "UL[c] = U0[c] - slope;"),
    ("slope wrong neighbour", "double slope = oracle_minmod(U0[c] - Um[c], Up[c] - U0[c]);",
     "double slope = oracle_minmod(U0[c] - Um[c], Up[c] - Um[c]);"),
    ("Riemann data transposed", "oracle_hllc(&BR[s * NV], &BL[(s + 1) * NV], d, &FF[s * NV]);",
     "oracle_hllc(&BL[s * NV], &BR[(s + 1) * NV], d, &FF[s * NV]);"),
    ("update sign", "out[i * NV + c] = U0[c] - lam * (Fp[c] - Fm[c]);",
     "out[i * NV + c] = U0[c] + lam * (Fp[c] - Fm[c]);"),
    ("periodic ghost off by one", "if (bc == 1) return ((i % n) + n) % n;",
     "if (bc == 1) return ((i % n) + n - 1) % n;"),
    ("ghost fill shifted", "int64_t src = ghost_source(s - 2, len, bc[d]);",
     "int64_t src = ghost_source(s - 1, len, bc[d]);"),
    ("dt takes max over axes", "if (q < r) r = q;", "if (q > r) r = q;"),
    ("sound speed drops gamma", "double c = sqrt(GAMMA * pressure_of(st) / rho);",
     "double c = sqrt(pressure_of(st) / rho);"),
    ("wavespeed y uses m_x", "double a1 = fabs(st[2] / rho) + c;", "double a1 = fabs(st[1] / rho) + c;"),
    ("sweep uses dx of x", "st = sweep_grid(n, bc, d, dt / dx[d], cur, nxt, info);",
     "st = sweep_grid(n, bc, d, dt / dx[0], cur, nxt, info);"),
    ("energy from primitives drops 1/2",
     "U[4 * ncell + q] = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w);",
     "U[4 * ncell + q] = p / (GAMMA - 1.0) + rho * (u * u + v * v + w * w);"),
]


@pytest.fixture(scope="module")
def source():
    with open(oracle_build.SOURCE) as f:
        return f.read()


def test_mutations_apply_once(source):
    for name, old, new in MUTANTS:
        assert source.count(old) == 1, f"mutation '{name}' does not match exactly once"
        assert old != new


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, name, old, new):
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new, 1))
    lib = oracle_build.build(str(src), str(tmp_path / "libmutant.so"))
    o = Oracle(load(lib))
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin(o)
        except Exception as e:  # any failure (assertion, non-physical state) counts
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"mutant '{name}' passes every pin"
