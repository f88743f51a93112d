"""Decision-checked parity of FP32 GPU solves against the FP64 oracle.

The accept test TV(x + gamma v) <= TV(x) of perturbed() (eq.
superiorization) and the loop test f(x_{k-1/2}) > eps of the superiorized
algorithms are discontinuous, and the paper says nothing about rounding.
Reading used by these tests: an FP32 solve may take the other branch of
such a test only where the oracle's FP64 margin lies within FP32 rounding of
the threshold, |TV(z) - TV(x)| <= MARGIN * TV(x) for a trial and
|f - eps| <= MARGIN * eps for the stop. Before the first differing decision
both sides took the same branches, so their states differ by rounding only
and the first flip is the one whose margin decides. Where it is that small,
the GPU solve is run again with the oracle's decisions (scg_solve's
`forced` argument), or both sides are taken to the same step count for a
stop that flipped, and the images are compared there; every such case is
counted and listed at the end of the session. A flip at a larger margin
fails the test: that is a bug, not rounding.
"""
from __future__ import annotations

import math

import numpy as np

# FP32 terms (unit roundoff 6e-8) summed over up to ~1e6 pixels or rays, on a
# trajectory that has drifted from the FP64 one by rounding: 1e-5 relative
MARGIN = 1e-5

FORCED: list = []     # (label, kind, step, relative margin)
CHECKED: list = []    # labels of every comparison made


def fp32_data(y):
    """The values an FP32 solve receives: y rounded to FP32, held exactly in
    FP64. FP32 parity runs the oracle on these, so both sides solve the same
    problem and only arithmetic differs (at 512 x 512 the rounding of y
    alone moves the oracle's own output by 3.5e-5)."""
    return np.asarray(y, dtype=np.float32).astype(np.float64)


def decisions(trace):
    return [(t["trials"], t["accepted"]) for t in trace]


def _decided_at(e) -> int:
    # trial index at which the step's search ended (accepted or exhausted)
    return e["accepted"] if e["accepted"] >= 0 else e["trials"]


def first_flip(ref_trace, gpu_trace):
    """(step index, relative FP64 margin) of the first step whose trial
    decision differs, or (None, 0.0)."""
    for i, (r, g) in enumerate(zip(ref_trace, gpu_trace)):
        if "trials" not in r:
            return None, 0.0
        if (r["trials"], r["accepted"]) != (g["trials"], g["accepted"]):
            m = min(_decided_at(r), _decided_at(g))
            margins = r.get("margins", [])
            if m >= len(margins) or r["tv_x"] == 0.0:
                return i, math.inf
            return i, abs(margins[m]) / abs(r["tv_x"])
    return None, 0.0


def _f_of(entry) -> float:
    return entry["f_half"] if "f_half" in entry else entry["f"]


def stop_margin(ref, steps_gpu: int, eps: float) -> float:
    """Relative FP64 margin of the oracle's loop test at the step where the
    two sides stopped differently."""
    s_r = ref.steps
    if steps_gpu < s_r:
        # the GPU stopped after steps_gpu steps, the oracle went on
        if steps_gpu < 1:
            return math.inf
        return (_f_of(ref.trace[steps_gpu - 1]) - eps) / eps
    if s_r < 1:
        return math.inf
    return (eps - _f_of(ref.trace[s_r - 1])) / eps


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def compare(label, run_gpu, run_oracle, eps, ref=None, margin=MARGIN):
    """run_gpu(forced, max_iter) -> (x, report, trace) with x on the host in
    FP64 (forced: list of (trials, accepted) or None; max_iter None: the
    case's own cap); run_oracle(max_iter) -> oracle Result. Returns
    (x_gpu, report, oracle result, forced kinds) with both sides at the same
    step count and with the same decisions."""
    CHECKED.append(label)
    if ref is None:
        ref = run_oracle(None)
    x, rep, tr = run_gpu(None, None)
    kinds = []
    forced = None
    i, rel = first_flip(ref.trace, tr)
    if i is not None:
        assert rel <= margin, (f"{label}: the trial decision of step {i + 1} differs from the "
                               f"oracle's at FP64 margin {rel:.3e} (> {margin:g})")
        forced = decisions(ref.trace)
        FORCED.append((label, "trial", i + 1, rel))
        kinds.append("trial")
        x, rep, tr = run_gpu(forced, None)
        n = min(len(tr), len(ref.trace))
        assert decisions(tr)[:n] == forced[:n]
    if rep.steps != ref.steps:
        rel = stop_margin(ref, rep.steps, eps)
        assert 0.0 <= rel <= margin, (f"{label}: stopped after {rep.steps} steps, the oracle "
                                      f"after {ref.steps}, FP64 stop margin {rel:.3e}")
        FORCED.append((label, "stop", min(rep.steps, ref.steps), rel))
        kinds.append("stop")
        if rep.steps < ref.steps:
            ref = run_oracle(rep.steps)
        else:
            x, rep, tr = run_gpu(forced, ref.steps)
        assert rep.steps == ref.steps
    return x, rep, ref, kinds


def summary_lines():
    lines = [f"FP32 decision checks: {len(CHECKED)} comparisons, {len(FORCED)} replayed "
             f"(margin bound {MARGIN:g})"]
    for label, kind, step, rel in FORCED:
        lines.append(f"  replayed {kind} decision of step {step} in {label}: "
                     f"FP64 margin {rel:.3e}")
    return lines
