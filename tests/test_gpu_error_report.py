"""Error of the GPU path against the FP64 oracle on the 512^3 smooth periodic
workload after 50 steps: L1 and Linf per conserved variable, FP32 and FP64.

The oracle needs minutes of host time for this (about 4 s per step at 512^3
on 16 cores), so the test runs only when RFV_ERROR_REPORT=1 is set; it prints
one JSON line with the errors.  The oracle is advanced one step per call,
which gives the same steps as one 50-step call (each step takes its dt from
the state it starts from) and lets the run report progress.
"""
import json
import os
import time

import numpy as np
import pytest

import gpu_util as G
from paper_2104_08571_amd import initial_states as ist
from paper_2104_08571_amd import ripple_fv as R

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skipif(os.environ.get("RFV_ERROR_REPORT") != "1",
                       reason="long run (minutes of oracle time at 512^3): set RFV_ERROR_REPORT=1"),
]

N = int(os.environ.get("RFV_ERROR_REPORT_N", "512"))
STEPS = int(os.environ.get("RFV_ERROR_REPORT_STEPS", "50"))


def errors(gpu, ref):
    out = {}
    for c, name in enumerate(("rho", "mx", "my", "mz", "E")):
        d = np.abs(gpu[c] - ref[c])
        out[name] = {"rel_L1": float(d.sum() / np.abs(ref[c]).sum()),
                     "rel_Linf": float(d.max() / np.abs(ref[c]).max()),
                     "L1": float(d.mean()), "Linf": float(d.max())}
    return out


def test_error_report_512_50_steps(oracle):
    n = (N, N, N)
    W = ist.smooth_periodic(n, seed=8571, device="cuda")
    results = {"workload": f"smooth periodic {N}^3, seed 8571, {STEPS} steps, CFL 0.9"}
    gpu = {}
    for name, dt in (("f32", R.F32), ("f64", R.F64)):
        g = R.make_grid(n, dtype=dt, layout=R.SOA, bc=(1, 1, 1))
        (U,), (t,) = G.run(g, W, STEPS, flags=R.RUN_GRAPH)
        gpu[name] = (U, t)
        print(f"[error-report] gpu {name} done, t = {t!r}", flush=True)
    U = oracle.prim_to_cons(W.cpu().numpy())
    del W
    t_ref = 0.0
    t0 = time.time()
    for s in range(STEPS):
        U, t, _ = oracle.run(U, 1, G.unit_dx(n), [1, 1, 1])
        t_ref += t
        print(f"[error-report] oracle step {s + 1}/{STEPS} ({time.time() - t0:.0f} s)", flush=True)
    results["t_oracle"] = t_ref
    for name, (Ug, t) in gpu.items():
        results[name] = {"t": t, "errors": errors(Ug, U)}
    print("[error-report] " + json.dumps(results), flush=True)
    for c in results["f32"]["errors"].values():
        assert c["rel_L1"] <= 1e-5
    for c in results["f64"]["errors"].values():
        assert c["rel_L1"] <= 1e-12
