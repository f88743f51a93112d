"""Per-iteration curves (error, f, TV against time, past the stop) on the
64 x 64 workload: the structure of the result and the behaviour the paper's
experimental section describes that holds on any such run - CG's f never
increases; past its stop S-CG's f keeps falling toward the least-squares
floor (superiorization does not regularize the limit); at the stop S-CG's
TV is at or below CG's, and its stop iterate meets eps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def result():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import curves, scg
    print("[curves] 64x64, CG / S_CG / S_PCG_K", flush=True)
    return curves.run(config=1, seed=0, variants=["CG", "S_CG", "S_PCG_K"], prec=scg.SCG_F64,
                      k_max=80, rho_grid=(0.02, 0.05))


@pytest.fixture(scope="module")
def oracle_case(oracle_lib):
    """The 64 x 64 curve workload with eps = f(x_true) and ||x_1|| from the
    oracle, so every input of the comparison below is the oracle's."""
    from oracle import algorithms as alg
    from synth import make_workload
    w = make_workload(1, 0)
    g = oracle_lib.Geometry(w.n, w.n_angles, w.n_bins)
    prob = alg.Problem(g, w.y)
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    return g, prob, prob.f(w.x_true.reshape(-1)), float(np.linalg.norm(x1))


@pytest.mark.parametrize("variant", ["S_CG", "S_CG_K"])
def test_points_match_oracle(oracle_case, variant):
    """Every point of an FP64 curve (f and TV of the output after m steps or
    passes) equals the oracle's at the same m, to 1e-9 relative: the points
    are the solver's own iterates, continued past the stop."""
    from oracle import algorithms as alg
    from paper_1709_04912_amd import curves, scg
    g, prob, eps, x1_norm = oracle_case
    rho = 0.05
    res = curves.run(config=1, seed=0, variants=[variant], prec=scg.SCG_F64, k_max=40,
                     eps=eps, x1_norm=x1_norm, rho=rho)
    c = res["curves"][0]
    pts = c["points"]
    pp = alg.PerturbParams(rho * x1_norm)
    fn = alg.scg if variant == "S_CG" else alg.scg_k
    ref = fn(prob, np.zeros(g.J), 1e-300, pp, max_iter=len(pts), record=True)
    assert len(ref.trace) == len(pts) and len(pts) > c["stop"]["steps"]
    print(f"[curves vs oracle] {variant}: {len(pts)} points, stop at {c['stop']['steps']}")
    for p, t, rec in zip(pts, ref.trace, ref.records):
        assert abs(p["f"] - t["f_half"]) <= 1e-9 * t["f_half"], (variant, p["steps"])
        tv = g.tv(rec["x_half"])
        assert abs(p["tv"] - tv) <= 1e-9 * tv, (variant, p["steps"])
    # the stop: the first m whose f meets eps, as the oracle's loop decides it
    stop_ref = fn(prob, np.zeros(g.J), eps, pp, max_iter=40)
    assert stop_ref.status == "ok" and c["stop"]["k"] == stop_ref.k


def _curve(result, v):
    return next(c for c in result["curves"] if c["variant"] == v)


def test_structure(result):
    from paper_1709_04912_amd import curves
    assert result["eps"] > 0 and result["tv_phantom"] > 0
    for c in result["curves"]:
        ms = [p["steps"] for p in c["points"]]
        assert ms == list(range(1, len(ms) + 1))
        assert len(ms) >= c["stop"]["steps"]
        for p in c["points"]:
            assert p["time_s"] > 0 and np.isfinite(p["f"]) and np.isfinite(p["error"])
    print(curves.summary(result))


def test_cg_f_nonincreasing(result):
    f = [p["f"] for p in _curve(result, "CG")["points"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(f, f[1:]))


def test_scg_past_the_stop(result):
    from paper_1709_04912_amd import scg
    c = _curve(result, "S_CG")
    s = c["stop"]
    assert s["status"] == scg.SCG_OK and s["f"] <= result["eps"]
    # the stop's output is the point after as many steps
    p = c["points"][s["steps"] - 1]
    assert p["k"] == s["k"]
    assert abs(p["f"] - s["f"]) <= 1e-6 * s["f"]
    past = [q["f"] for q in c["points"][s["steps"]:]]
    assert past and min(past) < s["f"]
    assert s["tv"] <= _curve(result, "CG")["stop"]["tv"] * (1 + 1e-9)
