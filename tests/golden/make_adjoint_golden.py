"""Write kuramoto_adjoint_n32.json: the FP64 oracle's window-averaged order
parameters and loss gradient for the full n = 32 gradient workload.

Calls only oracle/ (and the seeded input generator).  The inputs are the
workload's X0 and p rounded to float32 -- the values the binary32 library
receives -- so the stored gradient is the exact FP64 gradient for the very
inputs the GPU test integrates.  Takes a few minutes on 8 threads:

    python tests/golden/make_adjoint_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    w = workloads.kuramoto_adjoint()
    X0 = w["X0"].astype(np.float32).astype(np.float64)
    p = w["p"].astype(np.float32).astype(np.float64)
    R, _, rows = oracle.kuramoto_adjoint_parallel(
        w["n"], X0, p, 0.0, w["dt"], w["nsteps"], w["win_lo"], w["win_hi"], w["seed"],
        threads=max(1, min(16, os.cpu_count() or 1)))
    orbits = len(R)
    dLdR = 2.0 * (R - w["target"]) / orbits
    grad = np.zeros(rows.shape[1])
    for o in range(orbits):
        grad = grad + dLdR[o] * rows[o]
    out = {
        "source": "oracle.kuramoto_adjoint on workloads.kuramoto_adjoint() with float32-rounded "
                  "X0 and p; loss = mean_o (R_o - target)^2",
        "n": w["n"], "orbits": orbits, "dt": w["dt"], "nsteps": w["nsteps"],
        "win_lo": w["win_lo"], "win_hi": w["win_hi"], "seed": w["seed"], "target": w["target"],
        "loss": float(np.mean((R - w["target"]) ** 2)),
        "R_mean": float(R.mean()),
        "R_first8": [float(x) for x in R[:8]],
        "grad": [float(x) for x in grad],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kuramoto_adjoint_n32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
