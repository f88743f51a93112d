"""The smallest problems the library accepts, against the FP64 oracle: images
of 2 x 2, 3 x 3 and 5 x 5 pixels (one, four and sixteen TV terms), a single
angle, a single bin, more bins than the image is wide and fewer, through
every solver variant in FP64, to the stop (or to the iteration cap where the
stopping value is not reached): the oracle's status, k and trial decisions,
and its image within 1e-8 relative, or within 10 times the oracle's own
amplification of a relative change of y applied to FP64's unit roundoff if
that is larger. eps lies 1 % of the way from the least-squares floor to
f(0): closer to the floor, plain CG on the 5 x 5 image with 63 rays runs 15
steps and amplifies such a change 1.4e10-fold, which no bound on the image
survives. Launches here have one block per phase and partial sums of a
handful of blocks. The operators alone are checked at the same geometries."""
import numpy as np
import pytest

from oracle import algorithms as alg

pytestmark = pytest.mark.gpu

# (N, angles, bins)
CASES = [(2, 1, 3), (2, 4, 1), (3, 2, 5), (3, 5, 2), (5, 3, 4), (5, 7, 9)]
ORACLE = {
    "CG": lambda p, x0, eps, pp, m: alg.cg(p, x0, eps, max_iter=m),
    "PCG": lambda p, x0, eps, pp, m: alg.pcg(p, x0, eps, max_iter=m),
    "S_CG": lambda p, x0, eps, pp, m: alg.scg(p, x0, eps, pp, max_iter=m),
    "S_CG_CD": lambda p, x0, eps, pp, m: alg.scg_cd(p, x0, eps, pp, max_iter=m),
    "S_PCG": lambda p, x0, eps, pp, m: alg.spcg(p, x0, eps, pp, max_iter=m),
    "S_CG_K": lambda p, x0, eps, pp, m: alg.scg_k(p, x0, eps, pp, K=2, max_iter=m),
    "S_PCG_K": lambda p, x0, eps, pp, m: alg.spcg_k(p, x0, eps, pp, K=2, max_iter=m),
    "S_CG_3OP": lambda p, x0, eps, pp, m: alg.scg_3op(p, x0, eps, pp, max_iter=m),
}
MAX_ITER = 30


def _problem(oracle_lib, case):
    n, na, nb = case
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(100 * n + 10 * na + nb)
    y = rng.uniform(0.5, 1.5, na * nb)
    prob = alg.Problem(g, y)
    floor, _ = alg.ls_floor_dense(g, y)
    eps = floor + 1e-2 * (0.5 * float(y @ y) - floor)
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    gamma0 = 0.05 * float(np.linalg.norm(x1))
    return g, y, prob, eps, gamma0


@pytest.mark.parametrize("variant", list(ORACLE) + ["S_CG/mirrored", "S_CG_K/mirrored"])
@pytest.mark.parametrize("case", CASES)
def test_tiny_problem(oracle_lib, case, variant):
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import scg
    g, y, prob, eps, gamma0 = _problem(oracle_lib, case)
    print(f"[tiny] {case} {variant} eps={eps:.4g}", flush=True)
    variant, _, mirrored = variant.partition("/")
    pp = alg.PerturbParams(gamma0)
    ref = ORACLE[variant](prob, np.zeros(g.J), eps, pp, MAX_ITER)
    alt = ORACLE[variant](alg.Problem(g, y * (1 + 1e-13)), np.zeros(g.J), eps, pp, ref.steps)
    nrm = float(np.linalg.norm(ref.x))
    amp = float(np.linalg.norm(alt.x - ref.x)) / max(nrm, 1e-300) / 1e-13
    tol = max(1e-8, 10 * amp * 2.0 ** -52)
    n, na, nb = case
    with scg.Plan(n, na, nb) as plan:
        if mirrored:   # both mirrored operators
            plan.set_tuning(scg.SCG_F64, 4, 8, 8, 0, 1, 1)
        p = plan.params(eps=eps, gamma0=gamma0, variant=variant, prec=scg.SCG_F64,
                        max_iter=MAX_ITER)
        x, rep, trace = plan.solve(torch.tensor(y, dtype=torch.float64, device="cuda"), p)
    xg = x.cpu().numpy()
    want = scg.SCG_OK if ref.status == "ok" else scg.SCG_ENOCONV
    err = float(np.linalg.norm(xg - ref.x))
    print(f"  status {rep.status}/{ref.status} k {rep.k}/{ref.k} err {err:.2e} of {nrm:.3g} "
          f"(amplification {amp:.3g}, tolerance {tol:.2e})", flush=True)
    assert rep.status == want and rep.k == ref.k
    if variant.startswith("S_"):
        assert [(t["trials"], t["accepted"]) for t in trace] == \
            [(t["trials"], t["accepted"]) for t in ref.trace]
    assert err <= max(tol * nrm, 1e-12), (err, nrm)
    if ref.status == "ok":
        assert rep.f_out <= eps


@pytest.mark.parametrize("case", CASES)
def test_tiny_operators(oracle_lib, case):
    """A, A^T (both also mirrored), the ramp filter, TV and its subgradient at the
    same geometries against the oracle (FP32 within 1e-5, TV's value 1e-6;
    FP64 within 1e-12), and on a flat image, whose TV and subgradient are
    exactly zero."""
    import torch
    assert torch.cuda.is_available()
    from paper_1709_04912_amd import scg
    n, na, nb = case
    print(f"[tiny operators] {case}", flush=True)
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(7 * n + na + 3 * nb)
    x = rng.uniform(-1, 1, n * n)
    y = rng.uniform(-1, 1, na * nb)
    refs = (g.project(x), g.backproject(y), g.filter(y), g.tv_subgrad(x))
    tv_ref = g.tv(x)
    with scg.Plan(n, na, nb) as plan:
        for prec, dt, tol, tol_tv in ((scg.SCG_F32, torch.float32, 1e-5, 1e-6),
                                      (scg.SCG_F64, torch.float64, 1e-12, 1e-12)):
            xd = torch.tensor(x, dtype=dt, device="cuda")
            yd = torch.tensor(y, dtype=dt, device="cuda")
            tv, s = plan.tv(xd, subgrad=True)
            got = [plan.project(xd), plan.backproject(yd), plan.filter(yd), s]
            plan.set_tuning(prec, 4, 8, 8, 0, 1, 1)    # both mirrored operators
            got.append(plan.backproject(yd))
            got.append(plan.project(xd))
            for out, ref in zip(got, refs + (refs[1], refs[0])):
                out = out.cpu().numpy()
                assert np.linalg.norm(out - ref) <= tol * np.linalg.norm(ref), dt
            assert abs(tv - tv_ref) <= tol_tv * tv_ref, dt
            flat = torch.full((n * n,), 0.75, dtype=dt, device="cuda")
            tv0, s0 = plan.tv(flat, subgrad=True)
            assert tv0 == 0.0 and not s0.any(), dt
    assert g.tv(np.full(n * n, 0.75)) == 0.0 and not g.tv_subgrad(np.full(n * n, 0.75)).any()
