"""The serving loop (continuous batching on the batch engine) against the
plain one-at-a-time loop on a small Poisson stream of mixed sizes: every
request completes, with the output and report it has alone (bitwise), while
others are resident; admission waits when the arena is full; latencies and
summaries are well formed."""
import numpy as np
import pytest

from synth.workloads import make_serve_item, poisson_arrivals

pytestmark = pytest.mark.gpu

SHAPES = [(32, 45), (48, 64), (64, 90), (96, 128)]


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import serve
    print("[serve] building 24 requests", flush=True)
    cache = serve.PlanCache(shape=(4, 4, 4, 0))
    items = [make_serve_item(i, shapes=SHAPES) for i in range(12)]
    base = [serve.make_request(i, cache, w.y, w.x_true, w.n, w.n_angles, w.n_bins)
            for i, w in enumerate(items)]
    arr = poisson_arrivals(7, 24, 400.0)
    reqs = [serve.Request(i, base[i % 12].plan, base[i % 12].y, base[i % 12].params,
                          float(arr[i])) for i in range(24)]
    yield serve, reqs
    cache.close()


def _same(serve_mod, a, b):
    import torch
    assert set(a.outputs) == set(b.outputs)
    for rid in a.outputs:
        ra, rb = a.reports[rid], b.reports[rid]
        assert (ra.status, ra.k, ra.steps, ra.f_out, ra.tv_out) == \
            (rb.status, rb.k, rb.steps, rb.f_out, rb.tv_out), rid
        assert torch.equal(a.outputs[rid], b.outputs[rid]), rid


def test_served_equals_plain(stream):
    from paper_1709_04912_amd import scg
    serve, reqs = stream
    p = serve.serve_plain(reqs, keep_outputs=True)
    b = serve.serve_batched(reqs, arena_bytes=1 << 30, max_slots=16, iters=2,
                            keep_outputs=True)
    assert len(b.latency_s) == len(p.latency_s) == len(reqs)
    assert all(r.status == scg.SCG_OK for r in b.reports.values())
    _same(serve, p, b)
    for s in (p.summary(), b.summary()):
        assert s["requests"] == len(reqs) and s["recons_per_s"] > 0
        lat = s["latency_ms"]
        assert 0 < lat["p50"] <= lat["p99"] and lat["mean"] > 0
    assert np.all(b.latency_s > 0)


def test_admission_waits_for_room(stream):
    """An arena that holds two of the largest workspaces: requests wait for
    retirements (SCG_EAGAIN inside the loop) and still all complete with
    their plain results."""
    serve, reqs = stream
    need = max(r.plan.workspace_bytes(r.params) for r in reqs)
    p = serve.serve_plain(reqs, keep_outputs=True)
    b = serve.serve_batched(reqs, arena_bytes=2 * need + 4096, max_slots=16, iters=3,
                            keep_outputs=True)
    assert len(b.reports) == len(reqs)
    _same(serve, p, b)


def test_size_aware_engines_and_ls_eps(stream):
    """Requests of the largest size on an engine of their own, stepped in
    alternation with the others, and stopping values eps = 1.05 eps0_hat
    (eps0_hat: f after a run of plain CG): every request still gets its plain
    result, and the ls rule's eps lies above the CG value it came from."""
    from paper_1709_04912_amd import scg
    serve, reqs = stream
    cache = serve.PlanCache(shape=(4, 8, 4, 0, 1))
    items = [make_serve_item(i, shapes=SHAPES) for i in range(8)]
    base = [serve.make_request(i, cache, w.y, w.x_true, w.n, w.n_angles, w.n_bins,
                               eps_rule="ls", ls_steps=60) for i, w in enumerate(items)]
    arr = poisson_arrivals(11, 16, 400.0)
    reqs2 = [serve.Request(i, base[i % 8].plan, base[i % 8].y, base[i % 8].params,
                           float(arr[i])) for i in range(16)]
    for r in base:
        _, rep, _ = r.plan.solve(r.y, r.plan.params(eps=1e-300, gamma0=0.0, variant="CG",
                                                    max_iter=60), trace=False)
        assert abs(r.params.eps - 1.05 * rep.f_out) <= 1e-12 * r.params.eps
    p = serve.serve_plain(reqs2, keep_outputs=True)
    b = serve.serve_batched(reqs2, arena_bytes=1 << 30, max_slots=16, iters=3,
                            keep_outputs=True, large_n=64, large_iters=1)
    assert any(r.n >= 64 for r in reqs2) and any(r.n < 64 for r in reqs2)
    assert len(b.reports) == len(reqs2)
    assert all(r.status == scg.SCG_OK for r in b.reports.values())
    _same(serve, p, b)
    cache.close()


def test_direct_when_idle(stream):
    """The idle path: requests that find nothing resident or waiting are
    solved on their own, the others batched; every request gets its plain
    result bit for bit. Arrivals: eight spaced 0.2 s apart (each finds the
    device idle), then eight at one instant (batched behind the first)."""
    from paper_1709_04912_amd import scg
    serve, reqs = stream
    arr = [0.2 * i for i in range(8)] + [1.8] * 8
    reqs3 = [serve.Request(i, reqs[i].plan, reqs[i].y, reqs[i].params, arr[i])
             for i in range(16)]
    p = serve.serve_plain(reqs3, keep_outputs=True)
    b = serve.serve_batched(reqs3, arena_bytes=1 << 30, max_slots=16, iters=2,
                            keep_outputs=True, direct_when_idle=True)
    assert len(b.reports) == len(reqs3)
    assert all(r.status == scg.SCG_OK for r in b.reports.values())
    # the spaced ones go direct (unless a solve outlasts the spacing); the
    # burst arrives together and is batched
    assert 4 <= b.direct <= 8
    assert b.summary()["solved_directly"] == b.direct
    _same(serve, p, b)
