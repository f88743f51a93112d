"""Reconstruction error, half-squared residual f and TV per iteration, against
time, for the solver variants on a synthetic phantom, continued past the
iteration where the stopping test first holds: the quantities the paper's
experimental section plots (error, f and TV versus time, the stop marked).

For a variant, the point after m steps is the output the solver returns
when it is allowed m steps (max_iter = m, eps below reach): x_{k-1/2} with
k = m + 1 for S-CG, S-CG-CD, S-PCG and the three-operator S-CG, x_m for CG
and PCG, the last perturbed point after m passes for S-CG-K and S-PCG-K
(k = m there). Its time is the device time of that solve.
gamma0 = rho ||x_1|| (x_1 the first CG iterate) with rho picked per variant
from a small grid as the one with the lowest error at the stop (the paper
picks gamma0 per method by hand for the best result).

Usage: python -m paper_1709_04912_amd.curves --config 2 --seed 0 --out FILE
All the solver work runs in libscg; this module drives it and measures.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import scg

VARIANTS_ALL = ["CG", "PCG", "S_CG", "S_CG_CD", "S_PCG", "S_CG_K", "S_PCG_K", "S_CG_3OP"]
RHO_GRID = (0.01, 0.02, 0.05, 0.1, 0.2)


def _rel(x: torch.Tensor, ref: torch.Tensor) -> float:
    return float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))


def _timed_solve(plan, y, params, ws, out, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _, rep, _ = plan.solve(y, params, out=out, ws=ws, trace=False, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return rep, e0.elapsed_time(e1) * 1e-3


def variant_curve(plan, y, x_true, eps, gamma0, variant, prec, k_max, stream):
    """Per-iteration points of one variant: k, time, f, TV, error."""
    dt = torch.float32 if prec == scg.SCG_F32 else torch.float64
    stop_p = plan.params(eps=eps, gamma0=gamma0, variant=variant, prec=prec, max_iter=k_max)
    ws = plan.workspace(stop_p)
    out = torch.empty(plan.n * plan.n, dtype=dt, device=y.device)
    rep, t_stop = _timed_solve(plan, y, stop_p, ws, out, stream)
    stop = {"k": rep.k, "steps": rep.steps, "status": rep.status, "time_s": t_stop,
            "f": rep.f_out, "tv": rep.tv_out, "error": _rel(out.double(), x_true)}
    m_end = min(k_max, max(2 * max(rep.steps, 1), rep.steps + 20))
    points = []
    for m in range(1, m_end + 1):
        p = plan.params(eps=1e-300, gamma0=gamma0, variant=variant, prec=prec, max_iter=m)
        r, t = _timed_solve(plan, y, p, ws, out, stream)
        # the report's f and TV are those of the output the solve returns
        points.append({"steps": m, "k": r.k, "time_s": t, "f": r.f_out, "tv": r.tv_out,
                       "error": _rel(out.double(), x_true)})
    return {"variant": variant, "gamma0": gamma0, "stop": stop, "points": points}


def run(config: int = 2, seed: int = 0, variants=None, prec: int = scg.SCG_F32,
        k_max: int = 200, rho_grid=RHO_GRID, device: int = 0, eps=None, x1_norm=None,
        rho=None) -> dict:
    """eps (default f(x_true)) and x1_norm (default ||x_1|| of the library's
    first CG iterate) may be given; rho fixes gamma0 = rho ||x_1|| for every
    superiorized variant instead of the per-variant search."""
    from synth import make_workload

    variants = variants or VARIANTS_ALL
    w = make_workload(config, seed)
    dev = torch.device("cuda", device)
    dt = torch.float32 if prec == scg.SCG_F32 else torch.float64
    stream = torch.cuda.current_stream(dev)
    y = torch.tensor(w.y.reshape(-1), dtype=dt, device=dev)
    x_true = torch.tensor(w.x_true.reshape(-1), dtype=torch.float64, device=dev)
    plan = scg.Plan(w.n, w.n_angles, w.n_bins, device=device)
    if prec == scg.SCG_F32:
        plan.autotune(scg.SCG_F32)
    if eps is None:
        eps = plan.f(y, x_true.to(dt))              # f(x_true): the stopping value
    if x1_norm is None:
        x1, _, _ = plan.solve(y, plan.params(eps=1e-300, gamma0=0.0, variant="CG", prec=prec,
                                             max_iter=1), trace=False)
        x1_norm = float(torch.linalg.vector_norm(x1.double()))
    out = {"config": config, "seed": seed, "n": w.n, "n_angles": w.n_angles,
           "n_bins": w.n_bins, "eps": eps, "tv_phantom": plan.tv(x_true.to(dt)),
           "precision": "f32" if prec == scg.SCG_F32 else "f64", "curves": []}
    tmp = torch.empty(w.n * w.n, dtype=dt, device=dev)
    for v in variants:
        if v in ("CG", "PCG"):
            gamma0 = 0.0
        elif rho is not None:
            gamma0 = rho * x1_norm
        else:
            best = None
            for rho in rho_grid:
                p = plan.params(eps=eps, gamma0=rho * x1_norm, variant=v, prec=prec,
                                max_iter=k_max)
                _, rep, _ = plan.solve(y, p, out=tmp, trace=False)
                err = _rel(tmp.double(), x_true)
                if rep.status == scg.SCG_OK and (best is None or err < best[0]):
                    best = (err, rho)
            gamma0 = (best[1] if best else 0.05) * x1_norm
        print(f"[curves] {v}: gamma0={gamma0:.4g}", file=sys.stderr, flush=True)
        out["curves"].append(variant_curve(plan, y, x_true, eps, gamma0, v, prec, k_max,
                                           stream))
    plan.close()
    return out


def summary(result: dict) -> str:
    lines = [f"{'variant':10s} {'k stop':>6s} {'time ms':>8s} {'f/eps':>7s} {'TV':>9s} "
             f"{'error':>7s} | past the stop: {'k':>4s} {'f/eps':>7s} {'TV':>9s} {'error':>7s}"]
    # min error over the points: the best iterate the method reaches at all
    lines[0] += f" | {'best error':>10s} {'at k':>5s}"
    eps = result["eps"]
    for c in result["curves"]:
        s, last = c["stop"], c["points"][-1]
        lines.append(f"{c['variant']:10s} {s['k']:6d} {1e3 * s['time_s']:8.2f} {s['f'] / eps:7.4f} "
                     f"{s['tv']:9.2f} {s['error']:7.4f} | {'':14s} {last['k']:4d} "
                     f"{last['f'] / eps:7.4f} {last['tv']:9.2f} {last['error']:7.4f}"
                     + " | {:10.4f} {:5d}".format(*min((p['error'], p['k']) for p in c['points'])))
    lines.append(f"phantom TV {result['tv_phantom']:.2f}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variants", default=",".join(VARIANTS_ALL))
    ap.add_argument("--f64", action="store_true")
    ap.add_argument("--k-max", type=int, default=200)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    r = run(a.config, a.seed, a.variants.split(","), scg.SCG_F64 if a.f64 else scg.SCG_F32,
            a.k_max)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(r, f)
    print(summary(r), flush=True)


if __name__ == "__main__":
    main()
