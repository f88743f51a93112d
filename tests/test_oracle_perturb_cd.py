"""Pins of the oracle's perturbed() (eq. superiorization with the step sizes
of eq. gamma_sequence) and of its S-CG-CD (Alg. S-CG-CD with CG-CD-STEP).

perturbed():
  * On a stand-in "TV" phi(x) = x_0^2 (subgradient 2 x_0 e_0) the accept
    test phi(x + gamma v) <= phi(x) reads gamma <= 2 |x_0|, so the first
    accepted counter value l is known in closed form. Step sizes that are
    powers of two make every comparison exact, which pins: the counter
    starts where the previous call left it and advances by one per trial
    (accepted or not); gamma = gamma0 a^l, not gamma0 a^(l+1); acceptance
    at equality (the test is non-strict); exhaustion of max_trials leaves x
    unchanged while l still advances; a zero subgradient changes nothing.
  * On the real isotropic TV, a single bright pixel: its subgradient, its
    norm 1 + 2 sqrt(2) and TV along -s/||s|| are worked out by hand below,
    which fixes the accepted trial and the returned image. A straight edge:
    TV rises along -s/||s|| for every step up to ||s||/2 (worked out below),
    so every trial is rejected.
S-CG-CD:
  * gamma0 = 0: CG-CD-STEP's beta = -||g'||^2/g^T p equals CG's
    ||g'||^2/||g||^2 under exact line searches on a quadratic, so the output
    after m steps is the minimiser of f over x0 + span{g0, H g0, ...,
    H^(m-1) g0} (H = A^T A), taken here from a dense QR basis; the
    successive steps x_{k+1} - x_k are A^T A-conjugate.
  * With perturbations: each step's exact line search lowers f, and the
    solve stops with f <= eps for eps above the least-squares floor.
"""
import math

import numpy as np
import pytest

from oracle import algorithms as alg

SQ2 = math.sqrt(2.0)


class QuadraticStandIn:
    """phi(x) = x_0^2 in place of TV (the perturbation logic only calls
    tv() and tv_subgrad())."""

    def tv(self, x, kappa=0.0):
        return float(x[0] * x[0])

    def tv_subgrad(self, x, kappa=0.0):
        s = np.zeros_like(x)
        s[0] = 2.0 * x[0]
        return s


def _x(d, n=5):
    x = np.zeros(n)
    x[0] = d
    return x


def test_perturbed_first_accepted_closed_form():
    g = QuadraticStandIn()
    # gamma_l = 2^-l: accepted at the first l with 2^-l <= 2 d
    for d, l_star in ((0.1, 3), (0.3, 1), (0.7, 0), (0.01, 6)):
        pp = alg.PerturbParams(gamma0=1.0, a=0.5, max_trials=50)
        z, ell, info = alg.perturbed(g, _x(d), 0, pp)
        assert info.accepted == l_star and info.trials == l_star + 1 and ell == l_star + 1
        assert info.gamma == 2.0 ** -l_star
        assert z[0] == d - 2.0 ** -l_star and not z[1:].any()
        assert len(info.margins) == l_star + 1 and info.margins[-1] <= 0.0
        assert all(m > 0.0 for m in info.margins[:-1])
    # a = 0.975 (the paper's value): d midway between two thresholds
    a, gamma0 = 0.975, 2.0
    for l_star in (0, 5, 40):
        d = 0.5 * gamma0 * a ** (l_star - 0.5) if l_star else 2.0 * gamma0
        pp = alg.PerturbParams(gamma0=gamma0, a=a, max_trials=100)
        z, ell, info = alg.perturbed(g, _x(d), 0, pp)
        assert info.accepted == l_star and ell == l_star + 1


def test_perturbed_counter_is_global():
    """Counter values run on across calls: l = 0..3 in the first call (the
    fourth trial is accepted), l = 4, 5 in the second. Dyadic values keep
    every sum exact."""
    g = QuadraticStandIn()
    pp = alg.PerturbParams(gamma0=1.0, a=0.5, max_trials=50)
    z1, ell, info1 = alg.perturbed(g, _x(13 / 128), 0, pp)     # 2 d = 0.203125
    assert (ell, info1.accepted, info1.gamma) == (4, 3, 0.125)
    assert z1[0] == -3 / 128
    z2, ell, info2 = alg.perturbed(g, z1, ell, pp)
    # 2^-4 > 2 * 3/128 is rejected, 2^-5 accepted; v = +e_0 now
    assert (ell, info2.accepted, info2.trials, info2.gamma) == (6, 1, 2, 2.0 ** -5)
    assert z2[0] == 1 / 128
    # a call that starts at l = 6 takes gamma0 a^6 first
    z3, ell3, info3 = alg.perturbed(g, _x(1.0), 6, pp)
    assert info3.accepted == 0 and info3.gamma == 2.0 ** -6 and ell3 == 7


def test_perturbed_accepts_at_equality():
    # gamma_2 = 1/4 = 2 d exactly: phi(x + gamma v) = (d - 2d)^2 = d^2 = phi(x)
    g = QuadraticStandIn()
    pp = alg.PerturbParams(gamma0=1.0, a=0.5, max_trials=50)
    z, ell, info = alg.perturbed(g, _x(0.125), 0, pp)
    assert info.accepted == 2 and ell == 3 and info.margins[-1] == 0.0
    assert z[0] == -0.125


def test_perturbed_exhaustion_and_zero_subgradient():
    g = QuadraticStandIn()
    pp = alg.PerturbParams(gamma0=1.0, a=0.5, max_trials=3)
    x = _x(0.01)
    z, ell, info = alg.perturbed(g, x, 10, pp)      # 2^-10 <= 0.02: accepted at once
    assert info.accepted == 0
    z, ell, info = alg.perturbed(g, x, 0, pp)       # 1, 1/2, 1/4 all > 0.02
    assert info.accepted == -1 and info.trials == 3 and ell == 3 and info.gamma == 0.0
    assert np.array_equal(z, x) and z is not x
    z, ell, info = alg.perturbed(g, np.zeros(5), 7, pp)
    assert ell == 7 and info.trials == 0 and info.accepted == -1 and np.array_equal(z, 0 * z)


def _spike(n=7, i0=3, j0=3, h=1.0):
    x = np.zeros((n, n))
    x[i0, j0] = h
    return x


def _spike_subgradient(n=7, i0=3, j0=3):
    # the bright pixel's own term (a = b = -h, t = sqrt(2) h) and the terms
    # of the pixels above and left of it (t = h), differentiated; terms with
    # t = 0 contribute nothing
    s = np.zeros((n, n))
    s[i0, j0] = 2.0 + SQ2
    s[i0 - 1, j0] = -1.0
    s[i0, j0 - 1] = -1.0
    s[i0 + 1, j0] = -1.0 / SQ2
    s[i0, j0 + 1] = -1.0 / SQ2
    return s


def _spike_tv_along(c, h=1.0):
    """TV of the spike moved by gamma v, c = gamma / ||s||: the centre becomes
    p = h - (2 + sqrt 2) c, the pixels above and left u = c, below and right
    w = c / sqrt 2; the ten terms that touch them are summed by hand."""
    p, u, w = h - (2.0 + SQ2) * c, c, c / SQ2
    return (SQ2 * abs(p - w) + 2.0 * math.hypot(p - u, u) + 2.0 * w + 2.0 * SQ2 * w
            + 2.0 * u + SQ2 * u)


def test_perturbed_real_tv_spike(oracle_lib):
    n = 7
    geo = oracle_lib.Geometry(n, 4, 11)
    x = _spike(n)
    s = _spike_subgradient(n)
    assert np.allclose(geo.tv_subgrad(x.reshape(-1)), s.reshape(-1), rtol=0, atol=1e-14)
    snorm = 1.0 + 2.0 * SQ2                         # sqrt(9 + 4 sqrt 2)
    assert abs(np.linalg.norm(s) - snorm) <= 1e-14
    tv_x = 2.0 + SQ2
    assert abs(_spike_tv_along(0.0) - tv_x) <= 1e-14
    # gamma0 large enough to overshoot: the first trials raise TV
    for gamma0, a in ((3.0 * snorm, 0.8), (0.9 * snorm, 0.975), (0.05, 0.975)):
        expect = next(l for l in range(200)
                      if _spike_tv_along(gamma0 * a ** l / snorm) <= tv_x)
        c_hit = gamma0 * a ** expect / snorm
        # keep clear of the threshold: the two neighbouring trials are decided
        # by a margin far above rounding
        assert _spike_tv_along(c_hit) - tv_x < -1e-9
        if expect:
            assert _spike_tv_along(gamma0 * a ** (expect - 1) / snorm) - tv_x > 1e-9
        pp = alg.PerturbParams(gamma0=gamma0, a=a, max_trials=200)
        z, ell, info = alg.perturbed(geo, x.reshape(-1), 0, pp)
        assert info.accepted == expect and ell == expect + 1
        zref = x - c_hit * s
        assert np.max(np.abs(z - zref.reshape(-1))) <= 1e-13
        assert abs(geo.tv(z) - _spike_tv_along(c_hit)) <= 1e-12


def test_perturbed_real_tv_edge_rejects(oracle_lib):
    """x = 0 left of column N/2, 1 from it on. s = -1 on column N/2 - 1 and
    +1 on column N/2 (rows 0..N-2), ||s|| = sqrt(2 (N-1)); with c = gamma/||s||
    TV(x + gamma v) - TV(x) = (1 + sqrt 2) c + sqrt((1 - 2c)^2 + c^2) - 1 > 0
    for 0 < c <= 1/2, so no trial is accepted, x is returned unchanged and l
    advances by max_trials."""
    n = 8
    geo = oracle_lib.Geometry(n, 4, 13)
    x = np.zeros((n, n))
    x[:, n // 2:] = 1.0
    s = geo.tv_subgrad(x.reshape(-1)).reshape(n, n)
    sref = np.zeros((n, n))
    sref[: n - 1, n // 2 - 1] = -1.0
    sref[: n - 1, n // 2] = 1.0
    assert np.array_equal(s, sref)
    snorm = math.sqrt(2.0 * (n - 1))
    for c in (1e-3, 0.1, 0.3, 0.5):
        delta = (1 + SQ2) * c + math.hypot(1 - 2 * c, c) - 1
        assert delta > 0
        z = x.reshape(-1) - c * snorm * s.reshape(-1) / snorm
        assert abs(geo.tv(z) - geo.tv(x.reshape(-1)) - delta) <= 1e-12
    pp = alg.PerturbParams(gamma0=0.5 * snorm, a=0.975, max_trials=30)
    z, ell, info = alg.perturbed(geo, x.reshape(-1), 4, pp)
    assert info.accepted == -1 and info.trials == 30 and ell == 34
    assert np.array_equal(z, x.reshape(-1))
    assert all(m > 0 for m in info.margins)


# ---------------------------------------------------------------------------
# S-CG-CD
# ---------------------------------------------------------------------------

def _small_problem(oracle_lib, n=6, na=16, nb=9, seed=0):
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(seed)
    A = g.dense()
    y = A @ rng.uniform(0, 1, g.J) + 0.05 * rng.standard_normal(g.L)
    return g, A, y


def _krylov_minimiser(A, y, x0, m):
    H = A.T @ A
    g0 = A.T @ (A @ x0 - y)
    K = np.empty((A.shape[1], m))
    v = g0.copy()
    for col in range(m):
        K[:, col] = v
        v = H @ v
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(A @ Q, y - A @ x0, rcond=None)
    return x0 + Q @ c


@pytest.mark.parametrize("seed", [0, 1])
def test_scg_cd_unperturbed_is_krylov(oracle_lib, seed):
    g, A, y = _small_problem(oracle_lib, seed=seed)
    prob = alg.Problem(g, y)
    x0 = np.zeros(g.J)
    pp = alg.PerturbParams(gamma0=0.0)
    outs = []
    for m in range(0, 9):
        res = alg.scg_cd(prob, x0, eps=0.0, pp=pp, max_iter=m)
        assert res.status == "noconv" and res.steps == m and res.k == m + 1
        outs.append(res.x)
    assert np.array_equal(outs[0], x0)              # x_{1/2} = x0
    for m in range(1, 9):
        xref = _krylov_minimiser(A, y, x0, m)
        assert np.linalg.norm(outs[m] - xref) <= 1e-9 * np.linalg.norm(xref), m
    # steps x_{k+1} - x_k are conjugate: <A d_i, A d_j> = 0, i != j
    d = [outs[m + 1] - outs[m] for m in range(8)]
    Ad = [A @ v for v in d]
    for i in range(8):
        for j in range(i):
            cos = abs(Ad[i] @ Ad[j]) / (np.linalg.norm(Ad[i]) * np.linalg.norm(Ad[j]))
            assert cos <= 1e-8, (i, j, cos)


def test_scg_cd_unperturbed_equals_cg_and_scg(oracle_lib):
    g, A, y = _small_problem(oracle_lib, n=8, na=20, nb=13, seed=4)
    prob = alg.Problem(g, y)
    pp = alg.PerturbParams(gamma0=0.0)
    for m in (3, 10):
        cd = alg.scg_cd(prob, np.zeros(g.J), eps=0.0, pp=pp, max_iter=m).x
        cg = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=m).x
        assert np.linalg.norm(cd - cg) <= 1e-9 * np.linalg.norm(cg)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_scg_cd_perturbed_decrease_and_termination(oracle_lib, seed):
    g, A, y = _small_problem(oracle_lib, n=10, na=24, nb=15, seed=seed)
    prob = alg.Problem(g, y)
    eps0, _ = alg.ls_floor_dense(g, y)
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    pp = alg.PerturbParams(gamma0=0.2 * float(np.linalg.norm(x1)))
    res = alg.scg_cd(prob, np.zeros(g.J), eps=1.1 * eps0, pp=pp, max_iter=2000, record=True)
    assert res.status == "ok" and res.f_out <= 1.1 * eps0
    assert abs(prob.f(res.x) - res.f_out) <= 1e-10 * res.f_out
    moved = 0
    for rec in res.records:
        assert prob.f(rec["x_next"]) <= prob.f(rec["x_half"]) * (1 + 1e-12)
        # the exact line search: the gradient at x_{k+1} is orthogonal to p_k
        gn = A.T @ (A @ rec["x_next"] - y)
        assert abs(gn @ rec["p"]) <= 1e-8 * np.linalg.norm(gn) * np.linalg.norm(rec["p"])
        moved += np.linalg.norm(rec["x_half"] - rec["x_k"]) > 0
    assert moved >= 2


@pytest.mark.parametrize("fn", [alg.scg, alg.scg_cd, alg.spcg, alg.scg_3op])
def test_counter_runs_across_steps(oracle_lib, fn):
    """The solvers hand perturbed() the counter where the previous step left
    it: after each step l equals the running total of trials (one global
    sequence gamma0 a^l, never restarted)."""
    g, A, y = _small_problem(oracle_lib, n=10, na=24, nb=15, seed=5)
    prob = alg.Problem(g, y)
    x1 = alg.cg(prob, np.zeros(g.J), eps=0.0, max_iter=1).x
    pp = alg.PerturbParams(gamma0=0.5 * float(np.linalg.norm(x1)))
    res = fn(prob, np.zeros(g.J), 0.0, pp, max_iter=12)
    total = 0
    for t in res.trace:
        total += t["trials"]
        assert t["ell"] == total
        assert len(t["margins"]) == t["trials"]
    assert total > len(res.trace)          # some steps rejected trials
    assert res.ell == total
