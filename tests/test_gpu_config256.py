"""S-CG and S-PCG at 256 x 256 (360 angles, 367 bins, 20 ellipses, 2 %
Gaussian noise) solved to the stop against the FP64 oracle: the FP64 GPU
path with identical decisions, stop and image within 1e-8, and the FP32
path (FP32 operators, TV and vector updates, FP64 CG scalars and eps test)
within relative L2 1e-4 with the eps test met, its decisions checked
against the oracle's FP64 margins (tests/parity_c10.py).

eps = 1.05 eps0_hat, eps0_hat an upper bound of the least-squares floor from
the oracle's CG run to ||g|| <= 1e-10 ||g_0|| (tests/golden/eps.json).
"""
import json
import os

import numpy as np
import pytest

import parity_c10 as c10
from oracle import algorithms as alg
from synth import make_workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = {"S_CG": alg.scg, "S_PCG": alg.spcg}
_REFS = {}


@pytest.fixture(scope="module")
def scg():
    from paper_1709_04912_amd import scg as mod
    return mod


@pytest.fixture(scope="module")
def case256(oracle_lib):
    import torch
    assert torch.cuda.is_available()
    gd = json.load(open(os.path.join(HERE, "golden", "eps.json")))["cfg2_s0"]
    w = make_workload(2, 0, supersample=2)
    g = oracle_lib.Geometry(w.n, w.n_angles, w.n_bins)
    return w, g, alg.Problem(g, w.y), 1.05 * gd["eps0"], 0.05 * gd["x1_norm"]


def _oracle(case256, variant, max_iter=None, fp32_data=False):
    """The oracle's solve on y, or on y rounded to FP32 (the FP32 solve's
    input)."""
    w, g, prob, eps, gamma0 = case256
    key = (variant, max_iter, fp32_data)
    if key not in _REFS:
        print(f"  oracle {variant} 256x256 max_iter={max_iter} fp32 data={fp32_data}",
              flush=True)
        if fp32_data:
            prob = alg.Problem(g, c10.fp32_data(w.y))
        _REFS[key] = ORACLE[variant](prob, np.zeros(g.J), eps=eps,
                                     pp=alg.PerturbParams(gamma0),
                                     max_iter=400 if max_iter is None else max_iter)
    return _REFS[key]


@pytest.mark.parametrize("variant", ["S_CG", "S_PCG"])
def test_fp64_to_the_stop(scg, case256, variant):
    import torch
    w, g, prob, eps, gamma0 = case256
    print(f"[256 fp64] variant={variant} eps={eps:.6g}", flush=True)
    ref = _oracle(case256, variant)
    assert ref.status == "ok"
    y64 = torch.tensor(w.y.reshape(-1), dtype=torch.float64, device="cuda")
    with scg.Plan(w.n, w.n_angles, w.n_bins) as plan:
        x, rep, trace = plan.solve(y64, plan.params(eps=eps, gamma0=gamma0, variant=variant,
                                                    prec=scg.SCG_F64, max_iter=400))
    rel = c10.rel_l2(x.cpu().numpy(), ref.x)
    print(f"  k={rep.k} ref_k={ref.k} rel={rel:.2e}")
    assert rep.status == scg.SCG_OK and rep.k == ref.k
    assert c10.decisions(trace) == c10.decisions(ref.trace)
    assert rep.f_out <= eps and abs(rep.f_out - ref.f_out) <= 1e-9 * ref.f_out
    assert rel <= 1e-8


@pytest.mark.parametrize("variant", ["S_CG", "S_PCG"])
def test_fp32_to_the_stop(scg, case256, variant):
    import torch
    w, g, prob, eps, gamma0 = case256
    print(f"[256 fp32] variant={variant} eps={eps:.6g}", flush=True)
    y32 = torch.tensor(w.y.reshape(-1), dtype=torch.float32, device="cuda")
    with scg.Plan(w.n, w.n_angles, w.n_bins) as plan:
        def run_gpu(forced, max_iter):
            p = plan.params(eps=eps, gamma0=gamma0, variant=variant, prec=scg.SCG_F32,
                            max_iter=400 if max_iter is None else max_iter)
            x, rep, trace = plan.solve(y32, p, forced=forced)
            return x.cpu().numpy().astype(np.float64), rep, trace

        xg, rep, ref, kinds = c10.compare(f"256x256 {variant}", run_gpu,
                                          lambda m: _oracle(case256, variant, m, True), eps,
                                          ref=_oracle(case256, variant, None, True))
    rel = c10.rel_l2(xg, ref.x)
    prob = alg.Problem(g, c10.fp32_data(w.y))
    print(f"  k={rep.k} ref_k={ref.k} replayed={kinds} rel={rel:.2e} f={rep.f_out:.8g}")
    assert rep.k == ref.k and rel <= 1e-4
    if "stop" not in kinds:
        assert rep.status == scg.SCG_OK and rep.f_out <= eps
    assert prob.f(xg) <= eps * (1 + c10.MARGIN)
