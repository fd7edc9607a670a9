"""Write kuramoto_adjoint_n32.json: the FP64 oracle's window-averaged order
parameters and loss gradient for the full n = 32 gradient workload, and how
far that gradient moves when the inputs move by one binary32 ulp.

Calls only oracle/ (and the seeded input generator).  The inputs are the
workload's X0 and p rounded to float32 -- the values the binary32 library
receives -- so the stored gradient is the exact FP64 gradient for the very
inputs the GPU test integrates.

The one-ulp response: for three seeded sign patterns, X0 and p are moved by
one binary32 ulp in relative terms (2^-24, random signs per entry) and the
oracle gradient is taken again (the loss weights dL/dR stay those of the
unperturbed run); the largest relative L2 change of the whole vector and of
each block (K, frequencies, noise strengths) over the patterns is stored.  It
measures how strongly the gradient responds to perturbations at the scale of
binary32 rounding.  Takes ~20 minutes on 8 threads:

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


def blocks(n):
    return {"K": slice(0, 1), "omega": slice(1, n + 1), "sigma": slice(n + 1, 2 * n + 1)}


def gradient(w, X0, p, dLdR, threads):
    _, _, rows = oracle.kuramoto_adjoint_parallel(
        w["n"], X0, p, 0.0, w["dt"], w["nsteps"], w["win_lo"], w["win_hi"], w["seed"],
        threads=threads)
    grad = np.zeros(rows.shape[1])
    for o in range(rows.shape[0]):
        grad = grad + dLdR[o] * rows[o]
    return grad


def main():
    threads = max(1, min(16, os.cpu_count() or 1))
    w = workloads.kuramoto_adjoint()
    X0 = w["X0"].astype(np.float32).astype(np.float64)
    p = w["p"].astype(np.float32).astype(np.float64)
    R, _, rows = oracle.kuramoto_adjoint_parallel(
        w["n"], X0, p, 0.0, w["dt"], w["nsteps"], w["win_lo"], w["win_hi"], w["seed"],
        threads=threads)
    orbits = len(R)
    dLdR = 2.0 * (R - w["target"]) / orbits
    grad = np.zeros(rows.shape[1])
    for o in range(orbits):
        grad = grad + dLdR[o] * rows[o]
    resp = {"all": 0.0, **{k: 0.0 for k in blocks(w["n"])}}
    for k in range(3):
        rng = np.random.default_rng(2000 + k)
        Xk = X0 * (1.0 + rng.choice([-1.0, 1.0], X0.shape) * 2.0 ** -24)
        pk = p * (1.0 + rng.choice([-1.0, 1.0], p.shape) * 2.0 ** -24)
        gk = gradient(w, Xk, pk, dLdR, threads)
        this = {"all": float(np.linalg.norm(gk - grad) / np.linalg.norm(grad))}
        for name, s in blocks(w["n"]).items():
            this[name] = float(np.linalg.norm(gk[s] - grad[s]) / np.linalg.norm(grad[s]))
        for key in resp:
            resp[key] = max(resp[key], this[key])
        print(f"sign pattern {k}: {this}", flush=True)
    out = {
        "source": "oracle.kuramoto_adjoint on workloads.kuramoto_adjoint() with float32-rounded "
                  "X0 and p; loss = mean_o (R_o - target)^2",
        "n": w["n"], "orbits": orbits, "dt": w["dt"], "nsteps": w["nsteps"],
        "win_lo": w["win_lo"], "win_hi": w["win_hi"], "seed": w["seed"], "target": w["target"],
        "loss": float(np.mean((R - w["target"]) ** 2)),
        "R_mean": float(R.mean()),
        "R_first8": [float(x) for x in R[:8]],
        "grad": [float(x) for x in grad],
        "ulp_response": {
            "what": "largest relative L2 change of the gradient (whole vector and per block) "
                    "over 3 seeded sign patterns moving X0 and p by 2^-24 relative",
            **resp},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kuramoto_adjoint_n32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
