"""Serving loop and batched runs on top of the batch engine (scg_batch_*).

A request is one reconstruction: a plan (geometry), a sinogram resident on
the device, its stopping value eps and its perturbation scale gamma0. The
served loop admits requests in arrival order as slots and arena memory free
up (admission by workspace footprint, SCG_EAGAIN otherwise), advances every
resident solve with `iters` iterations per engine step, and retires finished
solves between steps; requests that arrive while others are on the device
join them at the next step. Optionally the largest images get an engine of
their own, stepped in alternation with the others (size-aware scheduling).
The plain loop runs the same requests one at a time with scg_solve, in
arrival order. Both report per-request latency (completion minus arrival,
wall clock) and throughput.

All the solver work runs in libscg; this module schedules and measures.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import scg


@dataclass
class Request:
    rid: int
    plan: "scg.Plan"
    y: torch.Tensor
    params: "scg.scg_params"
    arrival: float = 0.0          # seconds after the start of the stream

    @property
    def n(self) -> int:
        return self.plan.n


class PlanCache:
    """One plan per geometry (trig tables, projector windows). Launch shapes:
    `shape` (project_groups, backproject_split, project_angles, swizzle and
    optionally backproject_mirror and project_mirror) for every plan when given - solves that
    share a shape run as one group, one
    launch per phase in a batch - else the autotuner's pick per geometry."""

    def __init__(self, device: int = 0, autotune: bool = True, shape=None):
        self.device = device
        self.autotune = autotune
        self.shape = tuple(shape) if shape is not None else None
        self.plans = {}

    def get(self, n: int, n_angles: int, n_bins: int) -> "scg.Plan":
        key = (n, n_angles, n_bins)
        if key not in self.plans:
            p = scg.Plan(n, n_angles, n_bins, device=self.device)
            if self.shape is not None:
                p.set_tuning(scg.SCG_F32, *self.shape)
            elif self.autotune:
                p.autotune(scg.SCG_F32)
            self.plans[key] = p
        return self.plans[key]

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def make_request(rid: int, cache: PlanCache, y_np: np.ndarray, x_true_np: np.ndarray,
                 n: int, n_angles: int, n_bins: int, rho: float = 0.05,
                 max_iter: int = 500, eps_rule: str = "f_true", ls_factor: float = 1.05,
                 ls_steps: int = 400) -> Request:
    """Device-resident request with gamma0 = rho ||x_1|| (x_1 the first CG
    iterate) and the stopping value eps by `eps_rule`, both computed here
    with the library before any timing:
      "f_true": eps = f(x_true) = 1/2 ||y - A x_true||^2, the misfit of the
                pixelised phantom;
      "ls":     eps = ls_factor * eps0_hat, eps0_hat = f after ls_steps
                iterations of plain CG from zero: an upper bound of the
                least-squares floor eps0 = min f (any point's f is), so
                eps > eps0 and the Appendix's Theorem 1 applies."""
    dev = torch.device(f"cuda:{cache.device}")
    plan = cache.get(n, n_angles, n_bins)
    y = torch.tensor(np.ascontiguousarray(y_np).reshape(-1), dtype=torch.float32, device=dev)
    if eps_rule == "ls":
        _, rep, _ = plan.solve(y, plan.params(eps=1e-300, gamma0=0.0, variant="CG",
                                              max_iter=ls_steps), trace=False)
        eps = ls_factor * rep.f_out
    else:
        xt = torch.tensor(np.ascontiguousarray(x_true_np).reshape(-1), dtype=torch.float32,
                          device=dev)
        eps = plan.f(y, xt)
    x1, _, _ = plan.solve(y, plan.params(eps=1e-30, gamma0=0.0, variant="CG", max_iter=1),
                          trace=False)
    gamma0 = rho * float(torch.linalg.vector_norm(x1.double()))
    params = plan.params(eps=eps, gamma0=gamma0, variant="S_CG", prec=scg.SCG_F32,
                         max_iter=max_iter)
    return Request(rid, plan, y, params)


@dataclass
class Served:
    latency_s: np.ndarray     # per request, completion - arrival
    wall_s: float             # first arrival to last completion
    reports: dict             # rid -> scg.Report
    outputs: dict             # rid -> output tensor
    latency_by_rid: dict = None   # rid -> completion - arrival
    engine_stats: list = None     # scg_batch_get_stats of each engine at the end
    direct: int = 0               # requests solved on their own (serve_batched's idle path)

    @property
    def recons_per_s(self) -> float:
        return len(self.latency_s) / self.wall_s if self.wall_s > 0 else 0.0

    def summary(self, requests=None) -> dict:
        """Throughput and latency percentiles; with the requests, also the
        percentiles per image size."""
        lat = 1e3 * self.latency_s
        out = {"requests": int(len(lat)), "recons_per_s": self.recons_per_s,
               "wall_s": self.wall_s,
               "latency_ms": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99)),
                              "mean": float(np.mean(lat))}}
        if self.direct:
            out["solved_directly"] = self.direct
        if requests is not None and self.latency_by_rid:
            by = {}
            for r in requests:
                by.setdefault(r.n, []).append(1e3 * self.latency_by_rid[r.rid])
            out["latency_ms_by_size"] = {
                f"{n}x{n}": {"requests": len(v), "p50": float(np.percentile(v, 50)),
                             "p99": float(np.percentile(v, 99))} for n, v in sorted(by.items())}
        return out


def _outputs(order: list) -> dict:
    """Output images of every request, allocated before the stream starts
    (a server keeps such a pool), so no allocation falls inside the timing."""
    return {r.rid: torch.empty(r.plan.J, dtype=r.y.dtype, device=r.y.device) for r in order}


def serve_plain(requests: list, keep_outputs: bool = False) -> Served:
    """One solve at a time (scg_solve), in arrival order; a solve starts at
    its arrival or when the previous one ends, whichever is later."""
    order = sorted(requests, key=lambda r: r.arrival)
    ws = {}
    for r in order:
        key = id(r.plan)
        need = r.plan.workspace_bytes(r.params)
        if key not in ws or ws[key].numel() < need:
            ws[key] = r.plan.workspace(r.params)
    pool = _outputs(order)
    lat, reports, outputs, by_rid = [], {}, {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in order:
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        out, rep, _ = r.plan.solve(r.y, r.params, out=pool[r.rid], ws=ws[id(r.plan)],
                                   trace=False)
        done = time.perf_counter() - t0
        lat.append(done - r.arrival)
        by_rid[r.rid] = done - r.arrival
        reports[r.rid] = rep
        if keep_outputs:
            outputs[r.rid] = out
    wall = (time.perf_counter() - t0) - (order[0].arrival if order else 0.0)
    return Served(np.asarray(lat), wall, reports, outputs, by_rid)


def serve_batched(requests: list, arena_bytes: int, max_slots: int = 64, iters: int = 4,
                  graph: bool = False, keep_outputs: bool = False,
                  large_n: Optional[int] = None, large_iters: int = 1,
                  large_slots: int = 1, direct_when_idle: bool = False) -> Served:
    """Continuous batching on the batch engine: admit every arrived request
    that fits (FIFO; a request that does not fit blocks the ones behind it),
    run `iters` iterations of all resident solves, retire the finished ones,
    repeat. graph: replay each iteration as a captured HIP graph (measured a
    few per cent slower than enqueuing the kernels, whose host cost hides
    behind the device's work).

    With large_n, requests of N >= large_n go to a second batch engine of
    their own with `large_slots` slots (1: the large solves run one after
    another, as in a FIFO, instead of sharing the device among themselves),
    each engine getting half the arena, and the loop alternates `iters`
    iterations of the small solves with `large_iters` of the large ones: a
    small solve then advances at its own iteration cost instead of a large
    solve's (one launch per phase covers every resident solve, so in a
    shared batch each small iteration lasts as long as the large one's),
    while the large solves keep most of the device.

    direct_when_idle: a request of the first engine that arrives while
    nothing is resident or waiting is solved on its own with scg_solve (the
    single-solve path, the same result bit for bit); the requests that
    arrive meanwhile wait for it, then are batched as usual. At low load
    most requests find the device idle and skip the engine's per-step host
    work."""
    order = sorted(requests, key=lambda r: r.arrival)
    pool = _outputs(order)
    lat, reports, outputs, by_rid = [], {}, {}, {}
    nxt = 0
    direct = 0
    n_eng = 2 if large_n is not None else 1
    slots = [max_slots] if n_eng == 1 else [max_slots, max(1, large_slots)]
    engines = [scg.Batch(arena_bytes // n_eng, max_slots=slots[e], graph=graph)
               for e in range(n_eng)]
    inflight = [dict() for _ in range(n_eng)]
    waiting = [[] for _ in range(n_eng)]      # arrived, not yet admitted (FIFO per engine)
    steps = [iters, large_iters]

    def engine_of(r):
        return 1 if (large_n is not None and r.n >= large_n) else 0

    ws = {}
    if direct_when_idle:
        for r in order:
            if engine_of(r) == 0:
                need = r.plan.workspace_bytes(r.params)
                if id(r.plan) not in ws or ws[id(r.plan)].numel() < need:
                    ws[id(r.plan)] = r.plan.workspace(r.params)

    def finish(r, rep, out):
        lat.append(time.perf_counter() - t0 - r.arrival)
        by_rid[r.rid] = lat[-1]
        reports[r.rid] = rep
        if keep_outputs:
            outputs[r.rid] = out

    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while nxt < len(order) or any(inflight) or any(waiting):
            now = time.perf_counter() - t0
            if not any(inflight) and not any(waiting) and nxt < len(order) \
                    and order[nxt].arrival > now:
                time.sleep(order[nxt].arrival - now)
                now = time.perf_counter() - t0
            while nxt < len(order) and order[nxt].arrival <= now:
                waiting[engine_of(order[nxt])].append(order[nxt])
                nxt += 1
            if direct_when_idle and not any(inflight) and len(waiting[0]) == 1 \
                    and not any(waiting[1:]):
                r = waiting[0].pop()
                out, rep, _ = r.plan.solve(r.y, r.params, out=pool[r.rid], ws=ws[id(r.plan)],
                                           trace=False)
                finish(r, rep, out)
                direct += 1
                continue
            for e, b in enumerate(engines):
                while waiting[e]:
                    r = waiting[e][0]
                    got = b.submit(r.plan, r.y, r.params, out=pool[r.rid])
                    if got is None:
                        if not inflight[e]:
                            raise RuntimeError(f"request {r.rid} does not fit an empty batch")
                        break
                    inflight[e][got[0]] = (r, got[1])
                    waiting[e].pop(0)
            for e, b in enumerate(engines):
                if not inflight[e]:
                    continue
                b.step(steps[e])
                for t in list(inflight[e]):
                    rep = b.poll(t)
                    if rep is None:
                        continue
                    r, out = inflight[e].pop(t)
                    finish(r, rep, out)
        wall = (time.perf_counter() - t0) - (order[0].arrival if order else 0.0)
        stats = [b.stats() for b in engines]
    finally:
        for b in engines:
            b.close()
    return Served(np.asarray(lat), wall, reports, outputs, by_rid, stats, direct)
