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
