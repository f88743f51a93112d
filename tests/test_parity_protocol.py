"""The decision-checked comparison of FP32 solves with the oracle (host
logic of tests/parity_c10.py), driven by made-up traces: identical traces
pass untouched; a trial flip at a margin within FP32 rounding is replayed
with the oracle's decisions and counted; a flip at a larger margin fails; a
stop that flips at a tiny margin is compared at the same step count."""
from dataclasses import dataclass, field

import numpy as np
import pytest

import parity_c10 as c10


@pytest.fixture(autouse=True)
def _own_tally():
    """The made-up cases stay out of the session's list of replayed cases."""
    saved = (list(c10.FORCED), list(c10.CHECKED))
    yield
    c10.FORCED[:], c10.CHECKED[:] = saved


@dataclass
class Rep:
    steps: int


@dataclass
class Res:
    x: np.ndarray
    steps: int
    trace: list = field(default_factory=list)


def _entry(trials, accepted, margins, tv_x=100.0, f_half=10.0):
    return {"trials": trials, "accepted": accepted, "margins": margins, "tv_x": tv_x,
            "f_half": f_half}


def _ref(steps=3, f_last=0.9):
    tr = [_entry(2, 1, [5.0, -3.0]) for _ in range(steps)]
    tr[-1]["f_half"] = f_last
    return Res(np.ones(4), steps, tr)


def test_identical_traces_pass():
    ref = _ref()
    calls = []

    def run_gpu(forced, max_iter):
        calls.append((forced, max_iter))
        return np.ones(4), Rep(3), [dict(e) for e in ref.trace]

    x, rep, r, kinds = c10.compare("same", run_gpu, lambda m: ref, 1.0, ref=ref)
    assert kinds == [] and calls == [(None, None)] and r is ref


def test_small_margin_trial_flip_is_replayed():
    ref = _ref()
    ref.trace[1]["margins"] = [1e-4, -3.0]       # trial 0 rejected by 1e-6 relative
    gpu = [dict(e) for e in ref.trace]
    gpu[1] = _entry(1, 0, [])                    # the GPU accepted trial 0
    calls = []

    def run_gpu(forced, max_iter):
        calls.append(forced)
        return (np.ones(4), Rep(3), gpu if forced is None else [dict(e) for e in ref.trace])

    n0 = len(c10.FORCED)
    x, rep, r, kinds = c10.compare("flip", run_gpu, lambda m: ref, 1.0, ref=ref)
    assert kinds == ["trial"] and calls[1] == c10.decisions(ref.trace)
    assert c10.FORCED[n0][:3] == ("flip", "trial", 2)


def test_large_margin_trial_flip_fails():
    ref = _ref()
    gpu = [dict(e) for e in ref.trace]
    gpu[0] = _entry(1, 0, [])                    # oracle rejected trial 0 by 5 %

    def run_gpu(forced, max_iter):
        return np.ones(4), Rep(3), gpu

    with pytest.raises(AssertionError, match="margin"):
        c10.compare("bug", run_gpu, lambda m: ref, 1.0, ref=ref)


def test_stop_flip_within_rounding():
    # the oracle stops after 3 steps with f = eps (1 - 1e-7); the GPU goes on
    ref = _ref(f_last=1.0 - 1e-7)
    calls = []

    def run_gpu(forced, max_iter):
        calls.append(max_iter)
        steps = 4 if max_iter is None else max_iter
        return np.ones(4), Rep(steps), [dict(e) for e in ref.trace] + [_entry(2, 1, [5, -3])]

    x, rep, r, kinds = c10.compare("stop", run_gpu, lambda m: ref, 1.0, ref=ref)
    assert kinds == ["stop"] and calls == [None, 3] and rep.steps == 3
    # the GPU stops one step early where the oracle's f exceeds eps by 1e-7
    ref2 = _ref(steps=4, f_last=0.5)
    ref2.trace[2]["f_half"] = 1.0 + 1e-7
    shorter = Res(np.zeros(4), 3, ref2.trace[:3])

    def run_gpu2(forced, max_iter):
        return np.ones(4), Rep(3), ref2.trace[:3]

    x, rep, r, kinds = c10.compare("stop2", run_gpu2, lambda m: shorter if m == 3 else ref2,
                                   1.0, ref=ref2)
    assert kinds == ["stop"] and r is shorter


def test_stop_flip_with_large_margin_fails():
    ref = _ref(f_last=0.5)

    def run_gpu(forced, max_iter):
        return np.ones(4), Rep(4), ref.trace + [_entry(2, 1, [5, -3])]

    with pytest.raises(AssertionError, match="stop margin"):
        c10.compare("stopbug", run_gpu, lambda m: ref, 1.0, ref=ref)
