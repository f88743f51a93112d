"""Pins of the oracle's CG family against dense linear algebra.

* CG's k-th iterate minimises f over x0 + span{g0, H g0, ..., H^{k-1} g0},
  H = A^T A (the Krylov property of CG); the reference minimiser comes from a
  dense QR basis of that Krylov space and a dense least-squares solve.
* Run to convergence, CG reaches the dense least-squares solution.
* S-CG with gamma0 = 0 (no perturbation) produces CG's iterates: the
  perturbation-resilient step reproduces CG in exact arithmetic.
"""
import numpy as np
import pytest

from oracle import algorithms as alg


def _small_problem(oracle_lib, n=6, na=16, nb=9, seed=0):
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(seed)
    A = g.dense()
    y = A @ rng.uniform(0, 1, g.J) + 0.05 * rng.standard_normal(g.L)
    return g, A, y


def test_cg_krylov_minimisers(oracle_lib):
    g, A, y = _small_problem(oracle_lib)
    prob = alg.Problem(g, y)
    x0 = np.zeros(g.J)
    H = A.T @ A
    g0 = A.T @ (A @ x0 - y)
    # iterates of CG with eps = 0 (runs max_iter steps)
    iters = []
    x = x0.copy()
    for k in range(1, 7):
        res = alg.cg(prob, x0, eps=0.0, max_iter=k)
        iters.append(res.x)
    for k, xk in enumerate(iters, start=1):
        K = np.empty((g.J, k))
        v = g0.copy()
        for col in range(k):
            K[:, col] = v
            v = H @ v
        Q, _ = np.linalg.qr(K)
        c, *_ = np.linalg.lstsq(A @ Q, y - A @ x0, rcond=None)
        xref = x0 + Q @ c
        assert np.linalg.norm(xk - xref) <= 1e-8 * np.linalg.norm(xref), k


def test_cg_reaches_least_squares(oracle_lib):
    g, A, y = _small_problem(oracle_lib, seed=2)
    prob = alg.Problem(g, y)
    eps0, xls = alg.ls_floor_dense(g, y)
    res = alg.cg(prob, np.zeros(g.J), eps=eps0 * (1 + 1e-13), max_iter=500)
    assert np.linalg.norm(res.x - xls) <= 1e-6 * np.linalg.norm(xls)
    assert res.f_out <= eps0 * (1 + 1e-13)


def test_pcg_reaches_least_squares_consistent(oracle_lib):
    """With consistent data (y in the range of A) the filtered-residual
    preconditioner still leads PCG to the least-squares solution, f -> 0."""
    g = oracle_lib.Geometry(6, 16, 9)
    rng = np.random.default_rng(3)
    A = g.dense()
    xt = rng.uniform(0, 1, g.J)
    y = A @ xt
    prob = alg.Problem(g, y)
    res = alg.pcg(prob, np.zeros(g.J), eps=1e-20 * float(y @ y), max_iter=500)
    assert res.status == "ok"
    assert np.linalg.norm(res.x - xt) <= 1e-6 * np.linalg.norm(xt)


def test_scg_without_perturbation_is_cg(oracle_lib):
    g, A, y = _small_problem(oracle_lib, n=8, na=20, nb=13, seed=4)
    prob = alg.Problem(g, y)
    x0 = np.zeros(g.J)
    pp = alg.PerturbParams(gamma0=0.0)
    for k in range(1, 9):
        ref = alg.cg(prob, x0, eps=0.0, max_iter=k).x
        res = alg.scg(prob, x0, eps=0.0, pp=pp, max_iter=k - 1, record=True)
        # after k-1 PR steps the last x_{k} is records[-1]['x_next'] (x1 when k = 1)
        xk = res.records[-1]["x_next"] if res.records else None
        if xk is None:
            continue
        assert np.linalg.norm(xk - ref) <= 1e-9 * np.linalg.norm(ref), k


def test_pcg_k_and_cg_k_steps(oracle_lib):
    """CG-K from x0 with K steps equals K iterations of CG."""
    g, A, y = _small_problem(oracle_lib, seed=5)
    prob = alg.Problem(g, y)
    x0 = np.zeros(g.J)
    for K in (1, 2, 3):
        xk, f0 = alg.cg_k(prob, x0, K)
        ref = alg.cg(prob, x0, eps=0.0, max_iter=K).x
        assert np.allclose(xk, ref, rtol=0, atol=1e-12 * np.linalg.norm(ref))
        assert f0 == pytest.approx(prob.f(x0))


def test_scg_1_without_perturbation_is_steepest_descent(oracle_lib):
    """S-CG-K with K = 1 and gamma0 = 0 restarts CG after every step: each
    pass is one exact line search along -g, x' = x - (g^T g / ||A g||^2) g
    (written here with the dense matrix). The loop tests f of the pass's
    input, so the output after m passes is the (m-1)-th iterate."""
    g, A, y = _small_problem(oracle_lib, n=6, na=12, nb=9, seed=6)
    prob = alg.Problem(g, y)
    x = np.zeros(g.J)
    sd = [x.copy()]
    for _ in range(8):
        gr = A.T @ (A @ x - y)
        Ag = A @ gr
        x = x - (gr @ gr) / (Ag @ Ag) * gr
        sd.append(x.copy())
    f = [0.5 * float(np.sum((A @ v - y) ** 2)) for v in sd]
    for m in range(1, 7):
        # eps between f of the (m-1)-th and the (m-2)-th iterate: m passes
        eps = 0.5 * (f[m - 1] + f[m - 2]) if m >= 2 else 1.5 * f[0]
        res = alg.scg_k(prob, np.zeros(g.J), eps=eps, pp=alg.PerturbParams(0.0), K=1)
        want_k = m if m >= 2 else 0
        assert res.k == want_k, (m, res.k)
        ref = sd[max(want_k - 1, 0)]
        assert np.linalg.norm(res.x - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-30)
        assert res.f_out <= eps


def test_scg_k_passes_are_krylov_minimisers(oracle_lib):
    """With gamma0 = 0, every S-CG-2 pass minimises f over x + span{g, H g}
    (H = A^T A) from the pass's input x: a dense QR of that Krylov space."""
    g, A, y = _small_problem(oracle_lib, n=6, na=14, nb=9, seed=7)
    prob = alg.Problem(g, y)
    H = A.T @ A
    x = np.zeros(g.J)
    xs = [x.copy()]
    for _ in range(5):
        gr = A.T @ (A @ x - y)
        Kb = np.stack([gr, H @ gr], axis=1)
        Q, _ = np.linalg.qr(Kb)
        c, *_ = np.linalg.lstsq(A @ Q, y - A @ x, rcond=None)
        x = x + Q @ c
        xs.append(x.copy())
    f = [0.5 * float(np.sum((A @ v - y) ** 2)) for v in xs]
    for m in (2, 3, 4, 5):
        eps = 0.5 * (f[m - 1] + f[m - 2])
        res = alg.scg_k(prob, np.zeros(g.J), eps=eps, pp=alg.PerturbParams(0.0), K=2)
        assert res.k == m
        assert np.linalg.norm(res.x - xs[m - 1]) <= 1e-9 * np.linalg.norm(xs[m - 1])


def test_scg_k_terminates_below_eps(oracle_lib):
    """With perturbations (gamma0 > 0) S-CG-2 stops with f(output) <= eps for
    eps above the least-squares floor, and f(x0) <= eps returns x0 at k = 0."""
    g, A, y = _small_problem(oracle_lib, n=8, na=20, nb=13, seed=8)
    prob = alg.Problem(g, y)
    eps0, _ = alg.ls_floor_dense(g, y)
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    pp = alg.PerturbParams(gamma0=0.05 * float(np.linalg.norm(x1)))
    res = alg.scg_k(prob, np.zeros(g.J), eps=1.1 * eps0, pp=pp, K=2, max_iter=2000)
    assert res.status == "ok" and res.f_out <= 1.1 * eps0
    assert prob.f(res.x) == pytest.approx(res.f_out, rel=1e-12)
    x0 = np.full(g.J, 0.3)
    big = 2 * prob.f(x0)
    res0 = alg.scg_k(prob, x0, eps=big, pp=pp, K=2)
    assert res0.k == 0 and np.array_equal(res0.x, x0)


def test_spcg_1_without_perturbation_is_preconditioned_descent(oracle_lib):
    """S-PCG-K with K = 1 and gamma0 = 0: each pass is one exact line search
    along -z, z = A^T K (A x - y) the filtered-residual direction,
    x' = x - (g^T z / ||A z||^2) z with g = A^T (A x - y) (written with the
    dense A and the filter as a dense matrix). The loop tests f of the pass's
    input, so the output after m passes is the (m-1)-th iterate."""
    g, A, y = _small_problem(oracle_lib, n=6, na=12, nb=9, seed=8)
    prob = alg.Problem(g, y)
    Kd = np.stack([prob.K(e) for e in np.eye(g.L)], axis=1)
    x = np.zeros(g.J)
    it = [x.copy()]
    for _ in range(8):
        r = A @ x - y
        gr = A.T @ r
        z = A.T @ (Kd @ r)
        Az = A @ z
        x = x - (gr @ z) / (Az @ Az) * z
        it.append(x.copy())
    f = [0.5 * float(np.sum((A @ v - y) ** 2)) for v in it]
    assert all(f[i + 1] < f[i] for i in range(len(f) - 1))
    for m in range(2, 7):
        eps = 0.5 * (f[m - 1] + f[m - 2])
        res = alg.spcg_k(prob, np.zeros(g.J), eps=eps, pp=alg.PerturbParams(0.0), K=1)
        assert res.k == m, (m, res.k)
        ref = it[m - 1]
        assert np.linalg.norm(res.x - ref) <= 1e-10 * np.linalg.norm(ref)
        assert res.f_out <= eps


def test_pcg_k_equals_pcg(oracle_lib):
    """PCG-K from x0 with K steps is K iterations of PCG."""
    g, A, y = _small_problem(oracle_lib, seed=9)
    prob = alg.Problem(g, y)
    x0 = np.zeros(g.J)
    for K in (1, 2, 4):
        xk, f0 = alg.pcg_k(prob, x0, K)
        ref = alg.pcg(prob, x0, eps=0.0, max_iter=K).x
        assert np.linalg.norm(xk - ref) <= 1e-12 * np.linalg.norm(ref)
        assert f0 == pytest.approx(prob.f(x0))
