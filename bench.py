#!/usr/bin/env python3
"""Benchmark: S-CG reconstructions per second on one MI355X.

Workload (512 x 512 image, 720 angles over [0, 180 deg), 729 unit bins): a
seeded 30-ellipse phantom with a fine random texture of amplitude 0.02,
exact analytic line integrals, transmission-style noise (I0 = 1e5), and a
discrepancy stopping value: eps = f(x_true) = 1/2 ||y - A x_true||^2, the data
misfit of the pixelised phantom itself (noise plus the model mismatch of the
analytic line integrals; the paper's eps = N sigma^2 counts noise only, which
here lies below the least-squares floor). One step = one complete S-CG solve from the
zero image to f <= eps: FP32 projector, backprojector, TV and vector updates,
FP64 CG scalars and eps test, gamma0 = RHO * ||x_1||, a = 0.975.

Prints one JSON line. `roofline` describes the dominant kernel (its average
duration measured with HIP events on the solve's stream during the timed
solves); `cpu_baseline` times the FP64 oracle on the host for a bounded
sample (the initial step plus two S-CG steps), extrapolated to the GPU's step
count. Unless --no-mix is given, two more objects compare the batch engine
with plain one-at-a-time solves on the same requests (eps = f(x_true) and
gamma0 = RHO ||x_1|| per request, outputs compared bitwise):
  `batched`: 64 solves, N in {128, 256, 384, 512}, angles in {180, 360, 540,
             720} drawn independently, bins ceil(sqrt(2) N) + 1, all submitted
             at once; recons/s of each way (the faster of two runs);
  `served`:  Poisson streams of (N, angles) in {(128, 180), (256, 360),
             (512, 720), (1024, 1440)} with weights 0.4/0.3/0.2/0.1 and
             per-request eps = 1.05 x f after 400 CG iterations (an upper
             bound of the least-squares floor), 2000 requests at the
             specified mean rate of 200 requests/s (several times what one GPU
             sustains at that eps) and 300 at 20 requests/s (--serve-requests,
             --sustained-requests); p50/p99 latency (completion - arrival), also
             per size, and recons/s of continuous batching with the 1024^2
             requests on an engine of their own against a FIFO of plain
             solves.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RHO = 0.05                    # gamma0 = RHO * ||x_1||
N, N_ANGLES, N_BINS = 512, 720, 729
PEAK_LANE_OPS = 256 * 64 * 2.4e9   # VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
OPS_PER_NNZ = 8                    # weight evaluation + multiply-accumulate per nonzero
PEAK_HBM = 8.0e12
ARENA = 16 << 30                   # batch engine arena (bytes of HBM)
SERVE_POOL = 100                   # distinct requests of the served streams
LS_FACTOR, LS_STEPS = 1.05, 400    # served eps = LS_FACTOR x f after LS_STEPS CG iterations
FULL_SOLVE_S = 60.0                # the oracle's 512x512 solve is timed whole below this
PROFILE_EVERY = 8                  # timed solves: events around one dominant launch in 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_kb_project_kb_backproject_512x512_720x729.md")
# the kernels and the host code that lays out their launches (block order)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1709_04912_amd", "csrc", f)
                  for f in ("kernels.hip", "capi.hip")]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE
    / WRITE_SIZE summary, or None when the kernels or their launch layout have
    changed since the counters were taken (the summary records the sha256 of
    kernels.hip followed by capi.hip)."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"kernels\.hip \+ capi\.hip sha256: ([0-9a-f]{64})", text)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    if m is None or m.group(1) != h.hexdigest():
        return None
    m = re.search(rf"^traffic_bytes_per_launch {kernel}: (\d+)$", text, flags=re.M)
    return int(m.group(1)) if m else None


BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles",
                                    "traffic_batched_64_solves_streaming_kernels.md")
STREAMING_HBM = ("kb_xtv", "kb_perturb", "kb_p_update")   # bound by HBM (kb_trials: ALU)


def batched_roofline():
    """HBM roofline of the streaming kernels in the 64-solve batch, from the
    committed rocprofv3 summary (kernel-trace durations, FETCH_SIZE /
    WRITE_SIZE bytes of the same workload), or None when the kernels or
    their launch layout have changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(BATCHED_TRAFFIC_FILE):
        return None
    text = open(BATCHED_TRAFFIC_FILE).read()
    m = re.search(r"kernels\.hip \+ capi\.hip sha256: ([0-9a-f]{64})", text)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    if m is None or m.group(1) != h.hexdigest():
        return None
    per = {}
    for k, n, cb, ab, us in re.findall(
            r"^batched_kernel (\w+): launches=(\d+) counted_bytes=(\d+) "
            r"algorithmic_bytes=(\d+) avg_us=([0-9.]+)$", text, flags=re.M):
        d = float(us) * 1e-6
        per[k] = {"launches": int(n), "avg_us": float(us), "algorithmic_bytes": int(ab),
                  "traffic": int(cb), "achieved_GBs": int(ab) / d / 1e9,
                  "frac": int(ab) / d / PEAK_HBM,
                  "bound": "hbm" if k in STREAMING_HBM else "alu"}
    hbm = {k: v for k, v in per.items() if v["bound"] == "hbm"}
    if not hbm:
        return None
    dom = max(hbm, key=lambda k: hbm[k]["avg_us"] * hbm[k]["launches"])
    v = hbm[dom]
    return {"kernel": dom, "bound": "hbm", "achieved": v["achieved_GBs"],
            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": v["frac"], "traffic": v["traffic"],
            "source": os.path.relpath(BATCHED_TRAFFIC_FILE, ROOT) +
                      " (durations from the rocprofv3 kernel trace of the batched workload, "
                      "bytes from its FETCH_SIZE / WRITE_SIZE runs; full-batch launches)",
            "per_kernel": per}


def count_nnz(n, n_angles, n_bins):
    """Exact number of nonzero entries of A: for every angle and pixel, the
    bins b whose line crosses the pixel square with positive length, i.e.
    |t_b - proj| < (|c|+|s|)/2, or <= 1/2 for axis-aligned rays (a ray on a
    pixel edge has half weight)."""
    import numpy as np
    h, hb = 0.5 * (n - 1), 0.5 * (n_bins - 1)
    X, Y = np.meshgrid(np.arange(n) - h, h - np.arange(n))
    total = 0
    for a in range(n_angles):
        th = a * math.pi / n_angles
        c, s = math.cos(th), math.sin(th)
        c = 0.0 if abs(c) < 1e-12 else c
        s = 0.0 if abs(s) < 1e-12 else s
        u = X * c + Y * s + hb            # bin coordinate of the pixel centre
        if min(abs(c), abs(s)) == 0.0:
            lo, hi = np.ceil(u - 0.5), np.floor(u + 0.5)
        else:
            half = 0.5 * (abs(c) + abs(s))
            lo, hi = np.floor(u - half + 1e-9) + 1, np.ceil(u + half - 1e-9) - 1
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, n_bins - 1)
        total += int(np.maximum(hi - lo + 1, 0).sum())
    return total


def cpu_baseline(w, eps, gamma0, steps_gpu):
    """The FP64 oracle on the host. value: the whole 512x512 S-CG solve on all
    cores, timed when the initial step plus two steps predict it within
    FULL_SOLVE_S, else that prediction. Also one A and one A^T on a single
    core, and full solves of the 64x64 and 256x256 workloads (eps from
    tests/golden/eps.json) on all cores."""
    import numpy as np
    import oracle
    from oracle import algorithms as alg
    from synth import make_workload
    threads = oracle.ops.max_threads()
    g = oracle.Geometry(w.n, w.n_angles, w.n_bins, threads=threads)
    prob = alg.Problem(g, w.y)
    pp = alg.PerturbParams(gamma0)
    x0 = np.zeros(g.J)
    t = time.perf_counter()
    alg.scg(prob, x0, eps=eps, pp=pp, max_iter=0)
    t_init = time.perf_counter() - t
    t = time.perf_counter()
    alg.scg(prob, x0, eps=eps, pp=pp, max_iter=2)
    t_two = time.perf_counter() - t
    per_step = max(t_two - t_init, 1e-9) / 2.0
    est = t_init + per_step * steps_gpu
    out = {"unit": "recons/s", "cores": threads, "kind": "oracle"}
    if est <= FULL_SOLVE_S:
        t = time.perf_counter()
        ref = alg.scg(prob, x0, eps=eps, pp=pp, max_iter=2000)
        t_full = time.perf_counter() - t
        out["value"] = 1.0 / t_full
        out["sample"] = (f"one whole FP64 oracle S-CG solve at {w.n}x{w.n} ({w.n_angles}x"
                         f"{w.n_bins}), {ref.steps} steps, {t_full:.1f} s on {threads} threads")
    else:
        out["value"] = 1.0 / est
        out["sample"] = (f"FP64 oracle at {w.n}x{w.n} ({w.n_angles}x{w.n_bins}): initial step "
                         f"{t_init:.2f} s + 2 S-CG steps ({per_step:.2f} s/step), extrapolated "
                         f"to the GPU solve's {steps_gpu} steps")
    g1 = oracle.Geometry(w.n, w.n_angles, w.n_bins, threads=1)
    xr = np.random.default_rng(0).uniform(0, 1, g.J)
    t = time.perf_counter()
    yr = g1.project(xr)
    t_a1 = time.perf_counter() - t
    t = time.perf_counter()
    g1.backproject(yr)
    t_at1 = time.perf_counter() - t
    out["single_core"] = {"A_s": t_a1, "AT_s": t_at1,
                          "note": "one application each at 512x512 (720x729), one thread"}
    gd = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))
    configs = {}
    for key, cfg, factor in (("cfg1_s0", 1, 1.1), ("cfg2_s0", 2, 1.05)):
        wk = make_workload(cfg, 0, supersample=2)
        gk = oracle.Geometry(wk.n, wk.n_angles, wk.n_bins, threads=threads)
        pk = alg.Problem(gk, wk.y)
        epsk = factor * gd[key]["eps0"]
        ppk = alg.PerturbParams(RHO * gd[key]["x1_norm"])
        t = time.perf_counter()
        rk = alg.scg(pk, np.zeros(gk.J), eps=epsk, pp=ppk, max_iter=1000)
        tk = time.perf_counter() - t
        configs[f"{wk.n}x{wk.n}"] = {"seconds": tk, "recons_per_s": 1.0 / tk, "k": rk.k,
                                     "status": rk.status, "eps": f"{factor} eps0"}
    out["full_solves"] = configs
    return out


def mixed_runs(n_serve, n_sustained, shape):
    """Batched and served runs against plain one-at-a-time solves. Every plan
    gets `shape` (the autotuner's pick at 512^2): one shape makes each phase
    of the mix one launch, and one-at-a-time solves run as fast with it as
    with per-geometry picks (which differ only in the block order)."""
    import torch
    from paper_1709_04912_amd import serve
    from synth.workloads import make_batch_item, make_serve_item, poisson_arrivals

    def build(items):
        reqs = []
        for i, w in enumerate(items):
            reqs.append(serve.make_request(i, cache, w.y, w.x_true, w.n, w.n_angles, w.n_bins,
                                           rho=RHO))
        return reqs

    def warm(reqs):
        seen = {}
        for r in reqs:
            seen.setdefault(id(r.plan), r)
        w = list(seen.values())
        serve.serve_plain(w)
        serve.serve_batched(w, arena_bytes=ARENA, iters=4)

    def same(a, b):
        return sum(int(torch.equal(a.outputs[i], b.outputs[i])) for i in a.outputs)

    cache = serve.PlanCache(shape=shape)
    log("batched run: generating 64 solves")
    reqs = build([make_batch_item(i) for i in range(64)])
    warm(reqs)
    # each way twice, the ways alternating and the faster run of each kept:
    # a first run can still pay one-time costs (graph capture of a new
    # composition), and alternating keeps clock drift from favouring one way
    runs = {"graph": [], "eager": [], "plain": []}
    for _ in range(2):
        runs["graph"].append(serve.serve_batched(reqs, arena_bytes=ARENA, max_slots=256, iters=4,
                                                 graph=True, keep_outputs=True))
        runs["eager"].append(serve.serve_batched(reqs, arena_bytes=ARENA, max_slots=256, iters=4,
                                                 graph=False, keep_outputs=True))
        runs["plain"].append(serve.serve_plain(reqs, keep_outputs=True))
    b, be, p = (min(runs[k], key=lambda r: r.wall_s) for k in ("graph", "eager", "plain"))
    runs.clear()
    # the batched figure is the eager engine's, as the serving loop runs it
    # (an iteration of the mix is milliseconds of GPU work, so the host stays
    # ahead without a graph, and graph replays run a few per cent slower); the
    # graph path is reported beside it
    batched = {
        "workload": "64 S-CG solves, N in {128,256,384,512}, angles in {180,360,540,720}, "
                    "bins ceil(sqrt(2)N)+1, sigma U[0.5%,3%], eps = f(x_true)",
        "batched_recons_per_s": be.recons_per_s, "plain_recons_per_s": p.recons_per_s,
        "speedup": be.recons_per_s / p.recons_per_s,
        "batched_with_graph_recons_per_s": b.recons_per_s,
        "bitwise_equal_outputs": same(p, be), "bitwise_equal_with_graph": same(p, b),
        "graph_engine_stats": {k: b.engine_stats[0][k] for k in
                               ("macro_steps", "graph_builds", "graph_updates", "rebuild_ns")},
        "eager_engine_stats": {k: be.engine_stats[0][k] for k in ("macro_steps", "rebuild_ns")},
        "solves": len(reqs), "launch_shape": list(shape),
        "k_mean": float(sum(r.k for r in p.reports.values()) / len(p.reports)),
        "roofline": batched_roofline()}
    log(f"batched: {batched}")
    # the largest requests run on an engine of their own (below), so their
    # plan takes the autotuner's own pick without splitting the other
    # engine's groups; the plain loop solves them with the same plan
    from paper_1709_04912_amd import scg
    large_shape = cache.get(1024, 1440, 1450).autotune(scg.SCG_F32)
    log(f"served runs: 1024x1024 launch shapes {large_shape}")
    pool = SERVE_POOL
    log(f"served runs: generating {pool} distinct requests (eps = {LS_FACTOR} x f after "
        f"{LS_STEPS} CG iterations) for streams of {n_serve} and {n_sustained}")
    items = [make_serve_item(i) for i in range(pool)]
    base = [serve.make_request(i, cache, w.y, w.x_true, w.n, w.n_angles, w.n_bins, rho=RHO,
                               max_iter=2000, eps_rule="ls", ls_factor=LS_FACTOR,
                               ls_steps=LS_STEPS)
            for i, w in enumerate(items)]
    warm(base)
    served = {
        "workload": (f"(N, angles) in (128,180) (256,360) (512,720) (1024,1440) weights "
                     f"0.4/0.3/0.2/0.1, bins ceil(sqrt(2)N)+1, sigma U[0.5%,3%]; per-request "
                     f"eps = {LS_FACTOR} eps0_hat, eps0_hat = f after {LS_STEPS} CG iterations "
                     f"(an upper bound of the least-squares floor); {pool} distinct requests, "
                     f"the stream takes them in turn"),
        "launch_shape": list(shape),
        "launch_shape_1024": large_shape,
        "size_aware": "1024x1024 requests on an engine of their own (2 slots), 4 iterations of "
                      "it alternating with 4 of the other engine (64 slots); a smaller request "
                      "that finds nothing resident or waiting is solved on its own "
                      "(scg_solve, the same result bit for bit)"}
    for tag, rate, seed, count in (("as_specified_200_per_s", 200.0, 5000, n_serve),
                                   ("sustainable_20_per_s", 20.0, 5001, n_sustained)):
        t_run = time.perf_counter()
        arr = poisson_arrivals(seed, count, rate)
        reqs = [serve.Request(i, base[i % pool].plan, base[i % pool].y, base[i % pool].params,
                              float(arr[i])) for i in range(count)]
        log(f"served {tag}: {count} requests")
        bs = serve.serve_batched(reqs, arena_bytes=ARENA, max_slots=64, iters=4,
                                 keep_outputs=True, large_n=1024, large_iters=4,
                                 large_slots=2, direct_when_idle=True)
        p = serve.serve_plain(reqs, keep_outputs=True)
        run = {"requests": count, "rate_per_s": rate,
               "batched_size_aware": bs.summary(reqs), "plain": p.summary(reqs),
               "bitwise_equal_outputs": same(p, bs),
               "all_eps_met": all(r.status == 0 and r.f_out <= r_.params.eps
                                  for r_ in reqs for r in [bs.reports[r_.rid]])}
        if tag.startswith("sustainable"):
            b1 = serve.serve_batched(reqs, arena_bytes=ARENA, max_slots=64, iters=4)
            run["batched_one_engine"] = b1.summary(reqs)
        run["bench_seconds"] = time.perf_counter() - t_run
        served[tag] = run
        log(f"served {tag}: {run}")
    log(f"served: {served}")
    cache.close()
    return batched, served


def three_operator_run(plan, y, params, out_scg, ws, stream, w, steps):
    """The same solves with CG-PR-STEP evaluated by the q = A p recursion (two
    projections and one backprojection per step): throughput, stopping step
    and the image's distance from the literal S-CG output."""
    import numpy as np
    import torch
    from paper_1709_04912_amd import scg
    p3 = scg.scg_params.from_buffer_copy(params)
    p3.variant = scg.VARIANTS["S_CG_3OP"]
    out = torch.empty_like(out_scg)
    _, rep, _ = plan.solve(y, p3, out=out, ws=ws, trace=False, stream=stream)
    n = max(3, steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        _, rep, _ = plan.solve(y, p3, out=out, ws=ws, trace=False, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    a = out.double().cpu().numpy()
    b = out_scg.double().cpu().numpy()
    return {"variant": "S_CG_3OP", "value": n / elapsed, "unit": "recons/s", "solves": n,
            "status": rep.status, "k": rep.k, "steps_per_solve": rep.steps, "f_out": rep.f_out,
            "rel_diff_vs_s_cg": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "rel_err_vs_phantom": float(np.linalg.norm(a - w.x_true.reshape(-1))
                                        / np.linalg.norm(w.x_true))}


def spcg_run(plan, y, params, ws, stream, w, steps):
    """S-PCG (Alg. S-PCG with PCG-PR-STEP, the filtered-residual preconditioner)
    on the same workload and eps: throughput, stopping step, and the filter's
    share of a solve (its launches timed with events in one more solve)."""
    import numpy as np
    import torch
    from paper_1709_04912_amd import scg
    ps = scg.scg_params.from_buffer_copy(params)
    ps.variant = scg.VARIANTS["S_PCG"]
    out = torch.empty(plan.J, dtype=torch.float32, device=y.device)
    _, rep, _ = plan.solve(y, ps, out=out, ws=ws, trace=False, stream=stream)
    n = max(3, steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        _, rep, _ = plan.solve(y, ps, out=out, ws=ws, trace=False, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.profile(("filter",))
    plan.solve(y, ps, out=out, ws=ws, trace=False, stream=stream)
    torch.cuda.synchronize()
    f = plan.profile_read()["filter"]
    plan.profile(())
    per_solve_ms = 1e3 * elapsed / n
    return {"variant": "S_PCG", "value": n / elapsed, "unit": "recons/s", "solves": n,
            "status": rep.status, "k": rep.k, "steps_per_solve": rep.steps, "f_out": rep.f_out,
            "ms_per_solve": per_solve_ms,
            "filter": {"launches_per_solve": int(f[0]),
                       "avg_us": 1e3 * f[1] / f[0] if f[0] else 0.0,
                       "share_of_solve": f[1] / per_solve_ms},
            "rel_err_vs_phantom": float(np.linalg.norm(out.double().cpu().numpy()
                                                       - w.x_true.reshape(-1))
                                        / np.linalg.norm(w.x_true))}


def counter_workload(shapes):
    """Workload of the FETCH_SIZE / WRITE_SIZE counter runs: two 512x512
    S-CG solves with fixed launch shapes, then three plain device copies of
    64 MiB whose counter readings calibrate the counters' units."""
    import torch
    from paper_1709_04912_amd import scg
    from synth import make_workload
    w = make_workload(3, 0)
    dev = torch.device("cuda:0")
    plan = scg.Plan(N, N_ANGLES, N_BINS, device=0)
    plan.set_tuning(scg.SCG_F32, *shapes)
    y = torch.tensor(w.y.reshape(-1), dtype=torch.float32, device=dev)
    xt = torch.tensor(w.x_true.reshape(-1), dtype=torch.float32, device=dev)
    res = plan.project(xt).double() - y.double()
    eps = 0.5 * float((res * res).sum())
    p1 = plan.params(eps=1e-30, gamma0=0.0, variant="CG", max_iter=1)
    x1, _, _ = plan.solve(y, p1, trace=False)
    gamma0 = RHO * float(torch.linalg.vector_norm(x1.double()))
    p = plan.params(eps=eps, gamma0=gamma0, variant="S_CG", prec=scg.SCG_F32, max_iter=2000)
    for _ in range(2):
        _, rep, _ = plan.solve(y, p, trace=False)
    a = torch.ones(16 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"counter workload done: shapes={shapes} k={rep.k} status={rep.status}")
    plan.close()


def batched_counter_workload(shapes):
    """Workload of the batched counter runs: the benchmark's 64-solve mix
    (make_batch_item 0..63, all submitted at once, 4 iterations per engine
    step, without the graph so every phase is its own dispatch), run twice,
    then three plain device copies of 64 MiB for the counters' units."""
    import torch
    from paper_1709_04912_amd import serve
    from synth.workloads import make_batch_item
    cache = serve.PlanCache(shape=shapes)
    reqs = [serve.make_request(i, cache, w.y, w.x_true, w.n, w.n_angles, w.n_bins, rho=RHO)
            for i, w in enumerate(make_batch_item(i) for i in range(64))]
    for _ in range(2):
        r = serve.serve_batched(reqs, arena_bytes=ARENA, max_slots=256, iters=4, graph=False)
    dev = torch.device("cuda:0")
    a = torch.ones(16 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"batched counter workload done: shapes={shapes} solves={len(r.latency_s)} "
        f"{r.recons_per_s:.1f} recons/s")
    cache.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mix", action="store_true", help="skip the batched and served runs")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the served stream at the specified 200/s")
    ap.add_argument("--sustained-requests", type=int, default=300,
                    help="requests of the served stream at the sustainable 20/s")
    ap.add_argument("--counter-workload", metavar="SHAPES",
                    help="run only the hardware-counter workload with these launch shapes "
                         "(project_groups,backproject_split,project_angles,swizzle"
                         "[,backproject_mirror[,project_mirror]])")
    ap.add_argument("--batched-counter-workload", metavar="SHAPES",
                    help="run only the batched (64-solve) hardware-counter workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(one solve runs on one device)", file=sys.stderr)
        sys.exit(2)
    if args.counter_workload:
        counter_workload([int(v) for v in args.counter_workload.split(",")])
        return
    if args.batched_counter_workload:
        batched_counter_workload([int(v) for v in args.batched_counter_workload.split(",")])
        return

    import numpy as np
    import torch
    from paper_1709_04912_amd import scg
    from synth import make_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("generating the 512x512 workload")
    w = make_workload(3, 0)
    dev = torch.device("cuda:0")
    y = torch.tensor(w.y.reshape(-1), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    plan = scg.Plan(N, N_ANGLES, N_BINS, device=0)
    tuning = plan.autotune(scg.SCG_F32)
    log(f"launch shapes: {tuning}")
    xt = torch.tensor(w.x_true.reshape(-1), dtype=torch.float32, device=dev)
    res = plan.project(xt).double() - y.double()
    eps = 0.5 * float((res * res).sum())
    # gamma0 from the first CG iterate of the library's own CG
    p1 = plan.params(eps=1e-30, gamma0=0.0, variant="CG", max_iter=1)
    x1, _, _ = plan.solve(y, p1, trace=False)
    gamma0 = RHO * float(torch.linalg.vector_norm(x1.double()))
    params = plan.params(eps=eps, gamma0=gamma0, variant="S_CG", prec=scg.SCG_F32,
                         max_iter=2000)
    ws = plan.workspace(params)
    out = torch.empty(N * N, dtype=torch.float32, device=dev)

    # warm-up solves; the first one also profiles every kernel class
    plan.profile(scg.KERNEL_CLASSES)
    rep = None
    for i in range(max(args.warmup, 1)):
        _, rep, _ = plan.solve(y, params, out=out, ws=ws, trace=False)
        if i == 0:
            prof_all = plan.profile_read()
            plan.profile(())
    log(f"warm-up: status={rep.status} k={rep.k} steps={rep.steps} f={rep.f_out:.6g} "
        f"eps={eps:.6g}")
    dominant = max(("project", "backproject"), key=lambda c: prof_all[c][1])

    # timed solves: events around one launch in PROFILE_EVERY of the dominant
    # kernel (an event between two launches delays the second by a few us)
    plan.profile((dominant,), every=PROFILE_EVERY)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, rep, _ = plan.solve(y, params, out=out, ws=ws, trace=False, stream=stream)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(())
    assert rep.status == scg.SCG_OK and rep.f_out <= eps, rep

    launches, ms, tail_launches, tail_ms = prof[dominant]
    avg_s = ms / max(launches, 1) / 1e3
    nnz = count_nnz(N, N_ANGLES, N_BINS)
    achieved = OPS_PER_NNZ * nnz / avg_s
    err = float(np.linalg.norm(out.double().cpu().numpy() - w.x_true.reshape(-1))
                / np.linalg.norm(w.x_true))
    per_class = {c: {"launches": int(v[0]), "avg_us": (1e3 * v[1] / v[0]) if v[0] else 0.0,
                     "tail_launches": int(v[2]),
                     "tail_avg_us": (1e3 * v[3] / v[2]) if v[2] else 0.0}
                 for c, v in prof_all.items()}
    compulsory = 4 * (N * N + N_ANGLES * N_BINS)
    traffic = measured_traffic("kb_" + dominant)

    result = {
        "metric": "S-CG recons/s at 512x512 (720 angles x 729 bins)",
        "value": args.steps / elapsed,
        "unit": "recons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("512x512 S-CG solve to eps: 720 angles x 729 bins, 30 random ellipses "
                         "+ texture 0.02, transmission noise I0=1e5, eps = f(x_true)"),
            "variant": "S_CG", "scalars": "f64", "steps_per_solve": rep.steps, "k": rep.k,
            "launch_shapes": tuning,
            "gamma0": gamma0, "rho": RHO, "a": 0.975, "eps": eps, "f_out": rep.f_out,
            "tv_out": rep.tv_out, "rel_err_vs_phantom": err,
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                           "p99": 1e3 * float(np.percentile(lat, 99))},
            "kernel_avg_us": per_class,
        },
        "roofline": {
            "kernel": dominant,
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "T lane-op/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": traffic,
            # the three bandwidth readings of a matrix-free operator: its
            # counted HBM bytes (null when the counters are stale), the
            # compulsory bytes, and what an explicit sparse matrix (value and
            # column index per nonzero) would have to stream in the same time
            "per_launch": {"nnz": nnz, "ops_per_nnz": OPS_PER_NNZ, "avg_us": avg_s * 1e6,
                           "launches_timed": int(launches), "timed_one_in": PROFILE_EVERY,
                           "tail_launches": int(tail_launches),
                           "measured_hbm_GBs": (traffic / avg_s / 1e9) if traffic else None,
                           "measured_hbm_frac": (traffic / avg_s / PEAK_HBM) if traffic else None,
                           "compulsory_hbm_GBs": compulsory / avg_s / 1e9,
                           "compulsory_hbm_frac": compulsory / avg_s / PEAK_HBM,
                           "sparse_equivalent_GBs": (8 * nnz + compulsory) / avg_s / 1e9},
        },
    }
    result["three_operator"] = three_operator_run(plan, y, params, out, ws, stream, w, args.steps)
    result["s_pcg"] = spcg_run(plan, y, params, ws, stream, w, args.steps)
    log(f"s_pcg: {result['s_pcg']}")
    if not args.no_mix:
        shape = (tuning["project_groups"], tuning["backproject_split"],
                 tuning["project_angles"], tuning["swizzle"], tuning["backproject_mirror"],
                 tuning["project_mirror"])
        result["batched"], result["served"] = mixed_runs(args.serve_requests,
                                                         args.sustained_requests, shape)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        result["cpu_baseline"] = cpu_baseline(w, eps, gamma0, rep.steps)
    print(json.dumps(result), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
