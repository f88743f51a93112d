"""Pins of the oracle's preconditioning filter F^T C F (Filters for
Preconditioning section) and of S-PCG's invariance to its scale.

* The direct convolution with k = IDFT(c) equals the FFT route (numpy's FFT):
  zero-pad each projection to P, multiply its DFT by c(w_m), inverse DFT,
  keep the first n_bins samples.
* The filter is symmetric positive definite (c > 0).
* Multiplying c by any s > 0 leaves every S-PCG iterate unchanged: p, h, z
  scale by s, beta is unchanged and alpha scales by 1/s.
"""
import numpy as np
import pytest

from oracle import algorithms as alg


def _fft_filter(r2d, P, mu):
    m = np.fft.fftfreq(P) * P                       # 0..P/2-1, -P/2..-1
    w = 2 * np.pi * m / P
    c = (np.abs(w) + mu) * (0.54 + 0.46 * np.cos(w))
    pad = np.zeros((r2d.shape[0], P))
    pad[:, :r2d.shape[1]] = r2d
    out = np.fft.ifft(np.fft.fft(pad, axis=1) * c[None, :], axis=1)
    return out.real[:, :r2d.shape[1]]


@pytest.mark.parametrize("na,nb", [(5, 7), (3, 95), (4, 129)])
def test_filter_equals_fft(oracle_lib, na, nb):
    g = oracle_lib.Geometry(8, na, nb)
    rng = np.random.default_rng(nb)
    r = rng.standard_normal(g.L)
    P = g.filter_pad()
    assert P >= 2 * nb
    mu = g.default_mu()
    ref = _fft_filter(r.reshape(na, nb), P, mu).reshape(-1)
    got = g.filter(r, mu)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_filter_spd(oracle_lib):
    g = oracle_lib.Geometry(8, 2, 21)
    rng = np.random.default_rng(0)
    for _ in range(10):
        r = rng.standard_normal(g.L)
        s = rng.standard_normal(g.L)
        Kr, Ks = g.filter(r), g.filter(s)
        assert r @ Kr > 0
        assert abs(s @ Kr - r @ Ks) <= 1e-12 * (abs(s @ Kr) + 1e-30)


def test_spcg_scale_invariance(oracle_lib):
    g = oracle_lib.Geometry(12, 18, 19)
    rng = np.random.default_rng(3)
    xt = np.zeros((12, 12))
    xt[3:9, 2:8] = 1.0
    y = g.project(xt) + 0.02 * rng.standard_normal(g.L)
    prob1 = alg.Problem(g, y)
    prob2 = alg.Problem(g, y)
    k = g.filter_kernel()
    prob2._kernel = 7.5 * k
    pp = alg.PerturbParams(gamma0=0.5)
    a = alg.spcg(prob1, np.zeros(g.J), eps=0.0, pp=pp, max_iter=8)
    b = alg.spcg(prob2, np.zeros(g.J), eps=0.0, pp=pp, max_iter=8)
    assert [t["accepted"] for t in a.trace] == [t["accepted"] for t in b.trace]
    assert np.linalg.norm(a.x - b.x) <= 1e-10 * np.linalg.norm(a.x)


def test_spcg_each_step_decreases_f(oracle_lib):
    """Exact line search along any direction: without perturbation
    f(x_{k+3/2}) = f(x_{k+1}) = f(x_{k+1/2}) - (g'^T p')^2 / (2 ||A p'||^2)."""
    g = oracle_lib.Geometry(12, 18, 19)
    rng = np.random.default_rng(4)
    y = rng.uniform(0, 5, g.L)
    prob = alg.Problem(g, y)
    res = alg.spcg(prob, np.zeros(g.J), eps=0.0, pp=alg.PerturbParams(0.0), max_iter=10)
    tr = res.trace
    assert len(tr) == 10
    for a, b in zip(tr[:-1], tr[1:]):
        assert b["f_half"] <= a["f_half"]
        expect = a["f_half"] - 0.5 * a["gp"] ** 2 / a["qq"]
        assert abs(b["f_half"] - expect) <= 1e-10 * a["f_half"]
