"""Batch engine (scg_batch_*): many resident solves of different sizes,
precisions and variants advanced together with one launch per phase.

Bar: every solve's output image and report are bitwise those of scg_solve on
the same inputs with the same launch shapes (the batched kernels run the same
per-solve arithmetic in the same order), alone or in a mix, with the HIP
graph and without it, and across admissions and retirements while other
solves run. One mixed batch is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import parity_c10 as c10
from oracle import algorithms as alg
from synth import make_workload, random_ellipses, rasterize, analytic_sinogram

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scg():
    from paper_1709_04912_amd import scg as mod
    return mod


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


# launch shapes per case (project_groups, backproject_split, project_angles,
# swizzle, backproject_mirror, project_mirror): solves with different shapes
# run in different groups of a batch; the filtered variants' solves (S-PCG,
# PCG, S-PCG-K) mirror only their h = A^T q (their two-sinogram phase has no
# mirrored form and runs on every tile)
SHAPES = [(4, 4, 8, 0, 0, 1), (4, 8, 8, 0, 1, 0), (2, 1, 4, 1, 0, 1), (4, 4, 8, 0, 1, 1),
          (4, 4, 4, 1, 0, 0), (4, 8, 4, 1, 1, 1), (2, 2, 8, 0, 0, 0), (2, 2, 4, 0, 1, 1),
          (4, 4, 8, 1, 1, 0), (2, 4, 4, 0, 0, 1), (4, 1, 8, 1, 0, 0)]

# (n, n_angles, n_bins, variant, precision, seed)
CASES = [
    (32, 45, 49, "S_CG", "f32", 1),
    (48, 60, 71, "S_CG", "f64", 2),
    (40, 50, 61, "S_CG_CD", "f32", 3),
    (32, 45, 49, "S_PCG", "f32", 4),
    (36, 40, 55, "CG", "f32", 5),
    (64, 90, 95, "S_CG", "f32", 6),
    (24, 30, 37, "S_PCG", "f64", 7),
    (40, 60, 61, "S_CG_K", "f32", 8),
    (44, 60, 67, "S_CG_3OP", "f32", 9),
    (36, 50, 55, "PCG", "f32", 10),
    (40, 48, 61, "S_PCG_K", "f32", 11),
]


def _problem(oracle_lib, case):
    n, na, nb, variant, prec, seed = case
    rng = np.random.default_rng(seed)
    ells = random_ellipses(rng, 6)
    x_true = rasterize(ells, n, 2).reshape(-1)
    y = analytic_sinogram(ells, n, na, nb).reshape(-1)
    y = y + 0.01 * np.abs(y).max() * rng.standard_normal(y.size)
    g = oracle_lib.Geometry(n, na, nb)
    f_true = 0.5 * float(np.sum((g.project(x_true) - y) ** 2))
    return y, 1.2 * f_true, 0.05 * float(np.linalg.norm(x_true))


def _prepared(scg, torch, oracle_lib, cases):
    out = []
    for case, shape in zip(cases, SHAPES):
        n, na, nb, variant, prec, seed = case
        y, eps, gamma0 = _problem(oracle_lib, case)
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = scg.Plan(n, na, nb)
        plan.set_tuning(scg.SCG_F32 if prec == "f32" else scg.SCG_F64, *shape)
        p = plan.params(eps=eps, gamma0=gamma0, variant=variant,
                        prec=scg.SCG_F32 if prec == "f32" else scg.SCG_F64, max_iter=300)
        out.append((case, plan, torch.tensor(y, dtype=dt, device="cuda"), p))
    return out


def _alone(items):
    res = []
    for case, plan, y, p in items:
        x, rep, _ = plan.solve(y, p, trace=False)
        res.append((x.clone(), rep))
    return res


def _same(rep_a, rep_b):
    return (rep_a.status, rep_a.k, rep_a.steps, rep_a.trials_total, rep_a.ell, rep_a.f_out,
            rep_a.tv_out) == (rep_b.status, rep_b.k, rep_b.steps, rep_b.trials_total,
                              rep_b.ell, rep_b.f_out, rep_b.tv_out)


def _run_batch(scg, items, graph, max_slots=64, iters=3, arena=1 << 30):
    results = {}
    with scg.Batch(arena, max_slots=max_slots, graph=graph) as b:
        pending = list(range(len(items)))
        tickets = {}
        steps = 0
        while pending or tickets:
            while pending:
                i = pending[0]
                _, plan, y, p = items[i]
                r = b.submit(plan, y, p)
                if r is None:
                    break
                tickets[r[0]] = (i, r[1])
                pending.pop(0)
            b.step(iters)
            steps += 1
            assert steps < 10000
            for t in list(tickets):
                rep = b.poll(t)
                if rep is not None:
                    i, out = tickets.pop(t)
                    results[i] = (out.clone(), rep)
        stats = b.stats()
    return results, stats


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone(scg, torch_mod, oracle_lib, graph):
    torch = torch_mod
    print(f"[batch] mixed batch graph={graph}", flush=True)
    items = _prepared(scg, torch, oracle_lib, CASES)
    alone = _alone(items)
    got, stats = _run_batch(scg, items, graph)
    assert stats["retired"] == len(items) and stats["active"] == 0
    if graph:
        assert stats["graph_builds"] >= 1
    for i, (x, rep) in enumerate(alone):
        xb, rb = got[i]
        assert rep.status == scg.SCG_OK, (CASES[i], rep)
        assert _same(rep, rb), (CASES[i], rep, rb)
        assert torch.equal(x, xb), CASES[i]
    for _, plan, _, _ in items:
        plan.close()


def test_submit_waits_for_the_callers_stream(scg, torch_mod, oracle_lib):
    """y written on a stream of the caller's, behind a long run of matrix
    products there: the batch's work waits for that stream
    (scg_batch_wait_stream, called by submit), so the solve reads the
    finished y and equals the one run alone, bitwise."""
    torch = torch_mod
    print("[batch] submit from a side stream", flush=True)
    items = _prepared(scg, torch, oracle_lib, CASES[:2])
    alone = _alone(items)
    side = torch.cuda.Stream()
    m = torch.rand(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    with scg.Batch(1 << 30, max_slots=8, graph=False) as b, torch.cuda.stream(side):
        tickets = []
        for _, plan, y, p in items:
            yb = torch.zeros_like(y)
            for _ in range(16):
                m = m @ m
                m = m / m.abs().max()
            yb.copy_(y)
            r = b.submit(plan, yb, p)
            assert r is not None
            tickets.append((r[0], r[1], yb))
        reps = [None] * len(items)
        for _ in range(1000):
            if b.step(3) == 0:
                break
        for i, (t, out, _) in enumerate(tickets):
            reps[i] = (out.clone(), b.poll(t))
    for (x, rep), (xb, rb) in zip(alone, reps):
        assert rb is not None and _same(rep, rb), (rep, rb)
        assert torch.equal(x, xb)
    for _, plan, _, _ in items:
        plan.close()


def test_continuous_admission(scg, torch_mod, oracle_lib):
    """Three slots for seven solves: solves are admitted while others are on
    the device and retire at different iterations; every result is the one
    it has alone."""
    torch = torch_mod
    print("[batch] continuous admission", flush=True)
    items = _prepared(scg, torch, oracle_lib, CASES)
    alone = _alone(items)
    got, stats = _run_batch(scg, items, graph=True, max_slots=3, iters=2)
    assert stats["submitted"] == len(items)
    assert stats["graph_builds"] >= 1 and stats["graph_builds"] + stats["graph_updates"] >= 3
    for i, (x, rep) in enumerate(alone):
        xb, rb = got[i]
        assert _same(rep, rb) and torch.equal(x, xb), CASES[i]
    for _, plan, _, _ in items:
        plan.close()


def test_arena_admission_and_cancel(scg, torch_mod, oracle_lib):
    torch = torch_mod
    print("[batch] arena admission and cancel", flush=True)
    items = _prepared(scg, torch, oracle_lib, CASES[:2])
    (case0, plan0, y0, p0), (case1, plan1, y1, p1) = items
    need = plan0.workspace_bytes(p0)
    # room for one workspace only: the second submit waits for the first
    with scg.Batch(need + 4096, max_slots=8) as b:
        t0, out0 = b.submit(plan0, y0, p0)
        assert b.submit(plan1, y1, p1) is None
        assert b.poll(t0) is None
        while b.step(4) > 0:
            pass
        rep0 = b.poll(t0)
        assert rep0 is not None and rep0.status == scg.SCG_OK
        x_alone, rep_alone, _ = plan0.solve(y0, p0, trace=False)
        assert _same(rep0, rep_alone) and torch.equal(out0, x_alone)
        # a ticket's report is delivered once
        with pytest.raises(scg.ScgError):
            b.poll(t0)
        # cancel an active solve
        t1, _ = b.submit(plan0, y0, p0)
        b.cancel(t1)
        with pytest.raises(scg.ScgError):
            b.poll(t1)
        assert b.stats()["active"] == 0 and b.stats()["arena_used"] == 0
    with pytest.raises(scg.ScgError):
        scg.Batch(1024, max_slots=0)
    plan0.close()
    plan1.close()


def test_batch_against_oracle(scg, torch_mod, oracle_lib):
    """Two 64 x 64 workloads in one batch (one with non-default launch
    shapes: the mirrored backprojector) against the FP64 oracle: each batched output is bitwise the one
    scg_solve gives alone, and that solve matches the oracle (relative L2
    1e-4, eps met) with its decisions checked against the oracle's FP64
    margins (tests/parity_c10.py), so the bound holds for every case."""
    torch = torch_mod
    import json
    import os
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "eps.json")))
    items, refs = [], []
    for seed in (0, 1):
        w = make_workload(1, seed, supersample=2)
        g = oracle_lib.Geometry(w.n, w.n_angles, w.n_bins)
        prob = alg.Problem(g, c10.fp32_data(w.y))
        eps = 1.1 * gd[f"cfg1_s{seed}"]["eps0"]
        gamma0 = 0.05 * gd[f"cfg1_s{seed}"]["x1_norm"]
        pp = alg.PerturbParams(gamma0)
        ref = alg.scg(prob, np.zeros(g.J), eps=eps, pp=pp, max_iter=1000)
        plan = scg.Plan(w.n, w.n_angles, w.n_bins)
        if seed == 1:
            plan.set_tuning(scg.SCG_F32, 2, 8, 4, 1, 1)
        p = plan.params(eps=eps, gamma0=gamma0, max_iter=1000)
        items.append(((w.n,), plan, torch.tensor(w.y.reshape(-1), dtype=torch.float32,
                                                  device="cuda"), p))
        refs.append((prob, ref, eps, gamma0, pp, g))
    got, _ = _run_batch(scg, items, graph=True)
    for i, (prob, ref, eps, gamma0, pp, g) in enumerate(refs):
        x, rep = got[i]
        _, plan, y, p = items[i]
        x_alone, rep_alone, _ = plan.solve(y, p, trace=False)
        assert _same(rep, rep_alone) and torch.equal(x, x_alone)

        def run_gpu(forced, max_iter, plan=plan, y=y, eps=eps, gamma0=gamma0):
            q = plan.params(eps=eps, gamma0=gamma0,
                            max_iter=1000 if max_iter is None else max_iter)
            xs, r, tr = plan.solve(y, q, forced=forced)
            return xs.cpu().numpy().astype(np.float64), r, tr

        def run_oracle(max_iter, prob=prob, g=g, eps=eps, pp=pp):
            return alg.scg(prob, np.zeros(g.J), eps=eps, pp=pp,
                           max_iter=1000 if max_iter is None else max_iter)

        xg, r, ref_c, kinds = c10.compare(f"batch 64x64 seed {i}", run_gpu, run_oracle, eps,
                                          ref=ref)
        rel = c10.rel_l2(xg, ref_c.x)
        print(f"  seed {i}: k={rep.k} ref_k={ref.k} replayed={kinds} rel={rel:.2e}")
        assert rep.status == scg.SCG_OK and rep.f_out <= eps
        assert prob.f(x.cpu().numpy().astype(np.float64)) <= eps * (1 + c10.MARGIN)
        assert r.k == ref_c.k and rel <= 1e-4
    for _, plan, _, _ in items:
        plan.close()
