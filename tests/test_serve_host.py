"""Host logic of the serving loop (paper_1709_04912_amd/serve.py) on the CPU,
with stand-ins for the plan and the batch engine: which requests the idle
path solves on their own, which the engines batch, and that every request
completes once with its own result. No device work runs here; the GPU tests
check the results themselves against scg_solve bit for bit."""
import time
from dataclasses import dataclass

import pytest
import torch

from paper_1709_04912_amd import serve


@dataclass
class FakeReport:
    rid: int
    status: int = 0
    k: int = 0


class FakePlan:
    """A plan whose solve takes `iters` iterations of 0.5 ms each."""

    def __init__(self, n, iters):
        self.n, self.J, self.iters = n, n * n, iters

    def workspace_bytes(self, params):
        return 64

    def workspace(self, params):
        return torch.empty(64, dtype=torch.uint8)

    def solve(self, y, params, out=None, ws=None, trace=False):
        time.sleep(0.0005 * self.iters)
        out.fill_(float(params))
        return out, FakeReport(int(params), 0, self.iters), []


class FakeBatch:
    """An engine whose solves retire after their plan's iteration count."""
    made = []

    def __init__(self, arena_bytes, max_slots=64, graph=False):
        self.max_slots, self.active, self.done, self.next = max_slots, {}, {}, 0
        self.submitted = 0
        FakeBatch.made.append(self)

    def submit(self, plan, y, params, out=None):
        if len(self.active) >= self.max_slots:
            return None
        t = self.next
        self.next += 1
        self.submitted += 1
        self.active[t] = [plan, params, out, plan.iters]
        return t, out

    def step(self, iters=1):
        time.sleep(0.0005 * iters)
        for t in list(self.active):
            rec = self.active[t]
            rec[3] -= iters
            if rec[3] <= 0:
                plan, params, out, _ = self.active.pop(t)
                out.fill_(float(params))
                self.done[t] = FakeReport(int(params), 0, plan.iters)
        return len(self.active)

    def poll(self, t):
        return self.done.pop(t, None)

    def stats(self):
        return {"submitted": self.submitted}

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(serve.torch.cuda, "synchronize", lambda *a: None)
    monkeypatch.setattr(serve.scg, "Batch", FakeBatch)
    FakeBatch.made = []
    return serve


def _requests(arrivals, plans):
    return [serve.Request(i, plans[i % len(plans)], torch.zeros(1), i, a)
            for i, a in enumerate(arrivals)]


def _check_complete(res, reqs):
    assert len(res.latency_s) == len(reqs) and sorted(res.reports) == [r.rid for r in reqs]
    for r in reqs:
        assert res.reports[r.rid].rid == r.rid
        assert bool((res.outputs[r.rid] == float(r.rid)).all())
    assert (res.latency_s > 0).all()


def test_spaced_requests_take_the_idle_path(fake):
    """Requests 20 ms apart, each solved in 2 ms: every one finds the device
    idle and none reaches an engine."""
    plans = [FakePlan(8, 4), FakePlan(16, 4)]
    reqs = _requests([0.02 * i for i in range(10)], plans)
    res = fake.serve_batched(reqs, arena_bytes=1 << 20, keep_outputs=True,
                             direct_when_idle=True)
    _check_complete(res, reqs)
    assert res.direct == 10 and FakeBatch.made[0].submitted == 0


def test_a_burst_is_batched(fake):
    """One request alone, then eight at one instant: the first goes direct,
    the burst to the engine; without the idle path all go to the engine."""
    plans = [FakePlan(8, 6)]
    reqs = _requests([0.0] + [0.05] * 8, plans)
    res = fake.serve_batched(reqs, arena_bytes=1 << 20, keep_outputs=True,
                             direct_when_idle=True)
    _check_complete(res, reqs)
    assert res.direct == 1 and FakeBatch.made[0].submitted == 8
    res = fake.serve_batched(reqs, arena_bytes=1 << 20, keep_outputs=True)
    _check_complete(res, reqs)
    assert res.direct == 0 and FakeBatch.made[-1].submitted == 9


def test_large_requests_stay_on_their_engine(fake):
    """With large_n, requests of the large size never take the idle path,
    even when they find the device idle; the smaller ones do."""
    small, large = FakePlan(8, 2), FakePlan(64, 8)
    reqs = _requests([0.03 * i for i in range(8)], [small, large])
    res = fake.serve_batched(reqs, arena_bytes=1 << 20, keep_outputs=True,
                             direct_when_idle=True, large_n=64, large_slots=1)
    _check_complete(res, reqs)
    assert res.direct == 4
    eng_small, eng_large = FakeBatch.made[-2:]
    assert eng_small.submitted == 0 and eng_large.submitted == 4
