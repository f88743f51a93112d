"""Pins of the oracle's total variation and its subgradient.

Closed forms: constant image, linear ramp, checkerboard and an isolated
spike; convexity through the subgradient inequality; central finite
differences where TV is differentiable; homogeneity and shift invariance."""
import math

import numpy as np
import pytest


def test_constant_is_zero(oracle_lib):
    g = oracle_lib.Geometry(9, 4, 13)
    assert g.tv(np.full(81, 3.25)) == 0.0
    assert np.all(g.tv_subgrad(np.full(81, 3.25)) == 0.0)


@pytest.mark.parametrize("alpha,beta", [(0.3, -1.1), (2.0, 0.0), (0.0, -0.5)])
def test_ramp(oracle_lib, alpha, beta):
    n = 11
    g = oracle_lib.Geometry(n, 4, 17)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = alpha * i + beta * j
    ref = (n - 1) ** 2 * math.hypot(alpha, beta)
    assert abs(g.tv(x) - ref) <= 1e-12 * ref


def test_checkerboard(oracle_lib):
    n = 10
    g = oracle_lib.Geometry(n, 4, 15)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = (-1.0) ** (i + j)
    ref = (n - 1) ** 2 * 2 * math.sqrt(2)
    assert abs(g.tv(x) - ref) <= 1e-12 * ref


def test_spike(oracle_lib):
    """A spike of height h at an interior pixel enters three terms: its own
    (a = b = -h), the one above (a = h) and the one to the left (b = h)."""
    n, h = 7, 1.7
    g = oracle_lib.Geometry(n, 4, 11)
    x = np.zeros((n, n))
    x[3, 4] = h
    assert abs(g.tv(x) - h * (2 + math.sqrt(2))) <= 1e-14
    s = g.tv_subgrad(x).reshape(n, n)
    # d/dx of: own term sqrt(2) h -> 2/sqrt2 = sqrt2; above (3-1,4): 1; left (3,3): 1
    assert abs(s[3, 4] - (math.sqrt(2) + 2.0)) <= 1e-14
    assert abs(s[4, 4] - (-1 / math.sqrt(2))) <= 1e-14   # own term's a-neighbour
    assert abs(s[3, 5] - (-1 / math.sqrt(2))) <= 1e-14   # own term's b-neighbour
    assert abs(s[2, 4] - (-1.0)) <= 1e-14                # base of the term above
    assert abs(s[3, 3] - (-1.0)) <= 1e-14                # base of the term to the left


def test_boundary_terms(oracle_lib):
    """Only the (N-1)^2 interior forward-difference terms count: a spike in
    the last row or column enters the single term whose difference it ends."""
    n = 5
    g = oracle_lib.Geometry(n, 4, 9)
    x = np.zeros((n, n))
    x[n - 1, n - 1] = 1.0
    assert g.tv(x) == 0.0
    x = np.zeros((n, n))
    x[n - 1, 2] = 1.0
    assert abs(g.tv(x) - 1.0) <= 1e-15


def test_subgradient_inequality(oracle_lib):
    n = 12
    g = oracle_lib.Geometry(n, 4, 19)
    rng = np.random.default_rng(7)
    for _ in range(20):
        x = rng.standard_normal(n * n)
        x[rng.random(n * n) < 0.3] = 0.0
        x = np.round(x, 1)          # creates flat regions (t = 0 terms)
        s = g.tv_subgrad(x)
        tvx = g.tv(x)
        for _ in range(10):
            z = x + rng.standard_normal(n * n) * rng.uniform(0.01, 2.0)
            assert g.tv(z) >= tvx + s @ (z - x) - 1e-12 * (1 + abs(tvx))


def test_finite_differences(oracle_lib):
    n = 8
    g = oracle_lib.Geometry(n, 4, 13)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n * n)
    s = g.tv_subgrad(x)
    eps = 1e-6
    fd = np.empty_like(x)
    for k in range(x.size):
        e = np.zeros_like(x)
        e[k] = eps
        fd[k] = (g.tv(x + e) - g.tv(x - e)) / (2 * eps)
    assert np.max(np.abs(fd - s)) <= 1e-7


def test_homogeneity_and_shift(oracle_lib):
    n = 16
    g = oracle_lib.Geometry(n, 4, 23)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(n * n)
    assert abs(g.tv(-2.5 * x) - 2.5 * g.tv(x)) <= 1e-12 * g.tv(x)
    assert abs(g.tv(x + 7.0) - g.tv(x)) <= 1e-11 * g.tv(x)


def test_kappa_smoothing(oracle_lib):
    n = 6
    g = oracle_lib.Geometry(n, 4, 9)
    kappa = 0.3
    assert abs(g.tv(np.zeros(n * n), kappa) - (n - 1) ** 2 * kappa) <= 1e-14
