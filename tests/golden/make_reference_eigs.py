"""Writes ``reference_eigs.json``: the lowest eigenvalues of the Gaussian-well
benchmark operators, computed by the oracle's library eigensolver
(``oracle.lowest_eigenpairs``: preconditioned LOBPCG plus a Rayleigh-Ritz
step), never by the scheme.  They are the converged result the GPU solves are
compared with (1e-10 relative) and the spectral data of the step-count model
for the 64^3, N = 128 workload.

It also holds the lowest eigenvalues of the finite-difference oscillator of
Section 5.1 (99 x 99, -1/2 Lap + 1/2 |x|^2 on (-5.5, 5.5)^2), whose
ground-state energy is the reference of the relative energy error stop, and
of the finite-difference softened hydrogen atom standing in for Section 5.2
(48^3 on (-10, 10)^3, shifted by 1).

Run from the repository root:  python tests/golden/make_reference_eigs.py
(``--oscillator-only`` or ``--hydrogen-only`` recomputes just that case).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

CASES = [("wells3d_64^3_seed0", 64, 0, 17), ("wells3d_96^3_seed0", 96, 0, 17), ("wells3d_64^3_seed0", 64, 0, 136)]
# the finite-difference stand-in for Section 5.1's oscillator (99 x 99 interior grid, -1/2 Lap + 1/2 |x|^2)
OSC = ("oscillator2d_99", 99, 15)
# the finite-difference stand-in for Section 5.2's hydrogen atom (48^3 interior grid on (-10, 10)^3,
# -1/2 Lap - 1/sqrt(|x|^2 + 0.1^2), diagonal shift 1 so that the operator is positive definite), N = 5
HYD = ("hydrogen_soft_48", 48, 5, 10.0, 1.0)


def oscillator_case():
    name, m, N = OSC
    p = W.oscillator_2d_paper(m=m, N=N)
    op = O.Operator(p.grid.m, p.grid.h, p.V, kinetic=p.kinetic)
    vals, vecs, res = O.lowest_eigenpairs(op, N + 3)
    return {"name": name, "m": m, "seed": 0, "k": N + 3, "eigenvalues": vals.tolist(),
            "residual_norms": res.tolist(), "energy_of_lowest_15": 0.5 * float(np.sum(vals[:N]))}


def hydrogen_case():
    name, m, N, half, shift = HYD
    p = W.hydrogen_softened(m=m, N=N, half=half, shift=shift)
    op = O.Operator(p.grid.m, p.grid.h, p.V, kinetic=p.kinetic, shift=p.shift)
    t0 = time.time()
    vals, vecs, res = O.lowest_eigenpairs(op, N + 3, tol=1e-9, max_iter=5000)
    return {"name": name, "m": m, "N": N, "half": half, "shift": shift, "soft": 0.1, "k": N + 3,
            "eigenvalues": vals.tolist(), "residual_norms": res.tolist(), "seconds": time.time() - t0}


def replace_case(case):
    path = os.path.join(HERE, "reference_eigs.json")
    out = json.load(open(path))
    out["cases"] = [c for c in out["cases"] if c["name"] != case["name"]] + [case]
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def main():
    if "--hydrogen-only" in sys.argv:
        replace_case(hydrogen_case())
        return
    if "--oscillator-only" in sys.argv:
        path = os.path.join(HERE, "reference_eigs.json")
        out = json.load(open(path))
        out["cases"] = [c for c in out["cases"] if c["name"] != OSC[0]] + [oscillator_case()]
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        return
    out = {"source": "oracle.lowest_eigenpairs (LOBPCG, sine-transform preconditioner, tol 1e-7)",
           "operator": "-Lap_h + V on the m^3 interior grid of the unit cube, V = 8 seeded Gaussian wells",
           "cases": []}
    for name, m, seed, k in CASES:
        p = W.wells_3d(m=m, N=k, seed=seed, with_u0=False)
        op = O.Operator(p.grid.m, p.grid.h, p.V)
        t0 = time.time()
        vals, vecs, res = O.lowest_eigenpairs(op, k, extra=max(8, k // 8))
        dt = time.time() - t0
        hinv = 1.0 / p.grid.h[0] ** 2
        gersh = float(np.max(p.V) + 12.0 * hinv)        # upper bound on lambda_max (Gershgorin)
        out["cases"].append({"name": name, "m": m, "seed": seed, "k": k, "eigenvalues": vals.tolist(),
                             "residual_norms": res.tolist(), "lambda_max_upper_bound": gersh,
                             "seconds": dt})
        print(name, k, f"{dt:.1f}s", "max residual", float(res.max()), flush=True)
    out["cases"].append(oscillator_case())
    out["cases"].append(hydrogen_case())
    with open(os.path.join(HERE, "reference_eigs.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
