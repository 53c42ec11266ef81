"""Write sod32_bounds.json: locked L1 error bounds of the oracle's 32^3 Sod run.

The run is 32^3 cells, FP64, transmissive, CFL 0.9, 20 steps.  Its density,
velocity and pressure along x are compared with the exact Riemann solution at
the run's final time; each bound is the measured error times 1.25, so a later
change to the scheme that degrades accuracy fails the pin.  Calls only the
oracle package and the seeded input generator.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, exact_riemann  # noqa: E402
from paper_2104_08571_amd import initial_states as ist  # noqa: E402


def main():
    o = Oracle()
    U, t, _ = o.run(o.prim_to_cons(ist.sod((32, 32, 32)).numpy()), 20, [1 / 32] * 3,
                    [0, 0, 0], cfl=0.9)
    W = o.cons_to_prim(U)
    rho, u, p = exact_riemann.cell_averages(32, t, 0.5, (1, 0, 1), (0.125, 0, 0.1))
    errs = {"rho": float(np.abs(W[0, 0, 0] - rho).mean()),
            "u": float(np.abs(W[1, 0, 0] - u).mean()),
            "p": float(np.abs(W[4, 0, 0] - p).mean())}
    out = {"source": "written by make_sod32_bounds.py from the FP64 oracle; bound = 1.25 x measured L1",
           "t_final": t, "l1_measured": errs,
           "l1_max": {k: 1.25 * v for k, v in errs.items()}}
    with open(os.path.join(HERE, "sod32_bounds.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    main()
