"""The FP64 oracle against closed forms, textbook values and exact invariants."""
import numpy as np
import pytest

import oracle_pins as P
from paper_2104_08571_amd import initial_states as ist


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(oracle, pin):
    pin(oracle)


def test_exact_riemann_matches_toro():
    P.pin_exact_riemann_toro()


def test_thread_count_independent(oracle):
    """Each output cell is written by one thread from read-only input, so the
    result does not depend on the number of OpenMP threads."""
    U = oracle.prim_to_cons(ist.smooth_periodic((20, 18, 16), seed=3).numpy())
    dx = P.unit_dx(U)
    nt = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        R1, t1, _ = oracle.run(U, 3, dx, [1, 0, 1])
        oracle.set_num_threads(max(nt, 4))
        R4, t4, _ = oracle.run(U, 3, dx, [1, 0, 1])
    finally:
        oracle.set_num_threads(nt)
    assert t1 == t4 and np.array_equal(R1, R4)


def test_sweep_equals_step_pieces(oracle):
    """A step is wavespeed -> dt -> x, y, z sweeps with one dt."""
    U = oracle.prim_to_cons(ist.smooth_periodic((12, 10, 9), seed=8).numpy())
    dx = P.unit_dx(U)
    S = oracle.max_wavespeed(U)
    dt = oracle.dt(S, dx, 0.9)
    V = U
    for d in range(3):
        V = oracle.sweep(V, d, dt, dx, [1, 1, 1])
    R, t, dts = oracle.run(U, 1, dx, [1, 1, 1], cfl=0.9)
    assert dts[0] == dt and np.array_equal(R, V)


def test_generators_deterministic():
    a = ist.smooth_periodic((8, 6, 4), seed=2104)
    b = ist.smooth_periodic((8, 6, 4), seed=2104)
    c = ist.smooth_periodic((8, 6, 4), seed=2105)
    assert a.equal(b) and not a.equal(c)
    assert float(a[0].min()) >= 0.8 - 1e-12 and float(a[0].max()) <= 1.2 + 1e-12
    assert float(a[1:4].abs().max()) <= 0.1 + 1e-12
    assert ist.batch_extents() == ist.batch_extents()
    ext = ist.batch_extents()
    assert len(ext) == 64 and all(v in range(32, 193, 16) for e in ext for v in e)
    # SplitMix64 first outputs for seed 0 (published reference values)
    r = ist.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_subblock_generation_matches_global():
    """A sub-block generated with an origin equals the slice of the global field."""
    g = ist.smooth_periodic((12, 10, 8), seed=4)
    s = ist.smooth_periodic((6, 5, 4), seed=4, origin=(6, 5, 4), n_global=(12, 10, 8))
    assert np.allclose(g[:, 4:, 5:, 6:].numpy(), s.numpy(), rtol=0, atol=1e-15)
    b = ist.blast((8, 8, 8))
    bs = ist.blast((4, 4, 4), origin=(4, 0, 4), n_global=(8, 8, 8))
    assert b[:, 4:, 0:4, 4:].equal(bs)
