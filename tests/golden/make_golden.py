"""Writes tests/golden/eps.json: the least-squares floor eps0 = min 1/2||y - Ax||^2
(the paper's eps_0, Appendix) of seeded workloads, and the first CG iterate's
norm used to set gamma0. Calls only the FP64 oracle and the input generator.
Entries: the 64 x 64 workload (three seeds, dense least squares), the 256 x 256
one, and two sizes that are no multiple of any of the library's tiles (97 x 97
with 131 angles and 139 bins, 161 x 161 with 180 angles and 229 bins), whose
floors are CG's upper bounds.

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import algorithms as alg  # noqa: E402
from synth import make_workload  # noqa: E402


def entry(cfg, seed, dense=True, **over):
    w = make_workload(cfg, seed, supersample=2, **over)
    g = oracle.Geometry(w.n, w.n_angles, w.n_bins)
    prob = alg.Problem(g, w.y)
    if dense:
        eps0, _ = alg.ls_floor_dense(g, w.y)
        kind = "dense_lstsq"
    else:
        eps0 = alg.ls_floor_cg(prob, tol=1e-10, max_iter=3000)
        kind = "cg_upper_bound"
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    return {"cfg": cfg, "seed": seed, "n": w.n, "n_angles": w.n_angles, "n_bins": w.n_bins,
            "eps0": eps0, "eps0_kind": kind, "x1_norm": float(np.linalg.norm(x1)),
            "eps_discrepancy": w.eps_discrepancy}


def main():
    out = {}
    for seed in (0, 1, 2):
        out[f"cfg1_s{seed}"] = entry(1, seed)
    out["cfg2_s0"] = entry(2, 0, dense=False)
    out["ragged97_s0"] = entry(1, 0, dense=False, n=97, n_angles=131, n_bins=139)
    out["ragged161_s0"] = entry(1, 0, dense=False, n=161, n_angles=180, n_bins=229)
    path = os.path.join(HERE, "eps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(path)


if __name__ == "__main__":
    main()
