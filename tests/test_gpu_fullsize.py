"""S-CG at the benchmark's size in its launch configuration (512 x 512, 720
angles, 729 bins, autotuned launch shapes, FP32 operators with FP64 scalars,
eps = f(x_true), gamma0 = 0.05 ||x_1||): the first step against the FP64
oracle, and the solve to the stop checked with properties that hold at any
size - the oracle's FP64 f of the output meets eps, and the output's TV is
below unsuperiorized CG's at the same eps."""
import numpy as np
import pytest

from oracle import algorithms as alg
from synth import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(oracle_lib):
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import scg
    print("[full size] generating the 512x512 workload", flush=True)
    w = make_workload(3, 0)
    g = oracle_lib.Geometry(w.n, w.n_angles, w.n_bins)
    prob = alg.Problem(g, w.y)
    eps = prob.f(w.x_true)
    plan = scg.Plan(w.n, w.n_angles, w.n_bins)
    plan.autotune(scg.SCG_F32)
    y64 = torch.tensor(w.y.reshape(-1), dtype=torch.float64, device="cuda")
    x1, _, _ = plan.solve(y64, plan.params(eps=1e-300, gamma0=0.0, variant="CG",
                                           prec=scg.SCG_F64, max_iter=1), trace=False)
    gamma0 = 0.05 * float(torch.linalg.vector_norm(x1))
    y32 = y64.float()
    yield scg, plan, w, g, prob, eps, gamma0, y32
    plan.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_first_step(case):
    scg, plan, w, g, prob, eps, gamma0, y32 = case
    print("[full size] first S-CG step against the oracle", flush=True)
    ref = alg.scg(prob, np.zeros(g.J), eps=eps, pp=alg.PerturbParams(gamma0), max_iter=1)
    dec = [(t["trials"], t["accepted"]) for t in ref.trace]
    x, rep, trace = plan.solve(y32, plan.params(eps=eps, gamma0=gamma0, prec=scg.SCG_F32,
                                                max_iter=1))
    if [(t["trials"], t["accepted"]) for t in trace] != dec:
        x, rep, trace = plan.solve(y32, plan.params(eps=eps, gamma0=gamma0, prec=scg.SCG_F32,
                                                    max_iter=1), forced=dec)
    rel = _rel(x.cpu().numpy().astype(np.float64), ref.x)
    print(f"  k={rep.k} ref_k={ref.k} rel={rel:.2e} f={rep.f_out:.8g} ref_f={ref.f_out:.8g}")
    assert rep.status == scg.SCG_ENOCONV and ref.status == "noconv" and rep.k == ref.k == 2
    assert rel <= 1e-4
    assert abs(rep.f_out - ref.f_out) <= 1e-5 * ref.f_out


def test_solve_to_the_stop(case):
    import torch
    scg, plan, w, g, prob, eps, gamma0, y32 = case
    print("[full size] S-CG and CG to the stop", flush=True)
    x, rep, _ = plan.solve(y32, plan.params(eps=eps, gamma0=gamma0, prec=scg.SCG_F32,
                                            max_iter=2000), trace=False)
    xc, repc, _ = plan.solve(y32, plan.params(eps=eps, gamma0=0.0, variant="CG",
                                              prec=scg.SCG_F32, max_iter=2000), trace=False)
    xg = x.cpu().numpy().astype(np.float64)
    f_oracle = prob.f(xg)
    print(f"  S-CG k={rep.k} f={rep.f_out:.8g} oracle f={f_oracle:.8g} eps={eps:.8g}; "
          f"TV {rep.tv_out:.6g} vs CG {repc.tv_out:.6g} (k={repc.k})")
    assert rep.status == scg.SCG_OK and rep.f_out <= eps
    assert abs(f_oracle - rep.f_out) <= 1e-5 * rep.f_out
    assert f_oracle <= eps * (1 + 1e-5)
    assert repc.status == scg.SCG_OK and rep.tv_out < repc.tv_out
    tv_oracle = g.tv(xg)
    assert abs(tv_oracle - rep.tv_out) <= 1e-4 * tv_oracle
