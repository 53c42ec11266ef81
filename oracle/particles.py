"""FP64 CPU oracle for the particle update.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the HIP library.

What it computes (Ripple paper, section "Particle Update in Three
Dimensions"): every particle's position advanced by its velocity over one
time step, x <- x + v dt, for three-dimensional positions and velocities.
State: planar FP64 [6, n] holding (x, y, z, v_x, v_y, v_z) per particle.
The time step is an input; the device evaluates the update in its working
precision with dt rounded to it, and the oracle takes that rounded dt.
"""
import numpy as np


def update(P, dt):
    """Return a copy of P [6, n] with positions advanced: x_d += v_d dt."""
    P = np.array(P, dtype=np.float64, copy=True)
    if P.ndim != 2 or P.shape[0] != 6:
        raise ValueError("particles must be [6, n]")
    for d in range(3):
        P[d] = P[d] + P[3 + d] * dt
    return P
