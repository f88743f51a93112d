"""scg_solve_static (the entry point for callers that cannot allocate device
memory) against scg_solve through the C-ABI: two calls in a row on the same
device-wide static workspace, the second with a smaller problem, each
bitwise equal to scg_solve's output and report on the same inputs; the
static workspace's size limit is reported as SCG_ENOMEM."""
import numpy as np
import pytest

from synth import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scg():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import scg as mod
    return mod


def _same(a, b):
    return (a.status, a.k, a.steps, a.trials_total, a.ell, a.f_out, a.tv_out) == \
        (b.status, b.k, b.steps, b.trials_total, b.ell, b.f_out, b.tv_out)


def _case(scg, n, na, nb, seed, prec, variant):
    import torch
    w = make_workload(1, seed, n=n, n_angles=na, n_bins=nb, supersample=2)
    dt = torch.float32 if prec == scg.SCG_F32 else torch.float64
    y = torch.tensor(w.y.reshape(-1), dtype=dt, device="cuda")
    plan = scg.Plan(n, na, nb)
    f0 = 0.5 * float(np.sum(w.y ** 2))
    p = plan.params(eps=2e-3 * f0, gamma0=0.05 * float(np.abs(w.y).max()) / n, variant=variant,
                    prec=prec, max_iter=300)
    return plan, y, p


@pytest.mark.parametrize("variant", ["S_CG", "S_PCG"])
def test_static_equals_solve(scg, variant):
    import torch
    print(f"[no-alloc] {variant}", flush=True)
    assert scg.static_workspace_bytes() == 32 << 20
    # two calls in a row, the second smaller: the array keeps the first
    # call's contents, which must not leak into the second result
    for n, na, nb, seed, prec in ((96, 120, 139, 0, scg.SCG_F32), (40, 60, 61, 1, scg.SCG_F64),
                                  (24, 30, 37, 2, scg.SCG_F32)):
        plan, y, p = _case(scg, n, na, nb, seed, prec, variant)
        assert plan.workspace_bytes(p) <= scg.static_workspace_bytes()
        x_ref, rep_ref, tr_ref = plan.solve(y, p)
        out = torch.full_like(x_ref, float("nan"))
        x_st, rep_st, tr_st = plan.solve_static(y, p, out=out)
        print(f"  {n}x{n} prec={prec}: k={rep_st.k} status={rep_st.status}", flush=True)
        assert rep_ref.status in (scg.SCG_OK, scg.SCG_ENOCONV) and rep_ref.steps > 0
        assert _same(rep_ref, rep_st) and torch.equal(x_ref, x_st) and tr_ref == tr_st
        plan.close()


def test_static_limit(scg):
    import torch
    # FP64 at 1024 x 1024 needs far more than 32 MiB
    plan = scg.Plan(1024, 8, 1450)
    p = plan.params(eps=1.0, gamma0=0.0, prec=scg.SCG_F64, max_iter=1)
    assert plan.workspace_bytes(p) > scg.static_workspace_bytes()
    y = torch.zeros(8 * 1450, dtype=torch.float64, device="cuda")
    with pytest.raises(scg.ScgError) as e:
        plan.solve_static(y, p)
    assert e.value.status == scg.SCG_ENOMEM
    plan.close()
