"""Pins of the oracle's system matrix A against closed forms.

The oracle builds A by Siddon traversal (ray-driven) and A^T by clipping
each candidate line against a pixel square (pixel-driven). Neither uses the
closed-form chord of a line through a square, which these tests write out
from elementary geometry: for a line with unit normal (c, s) at signed
distance tau from a square's centre, with m = max(|c|,|s|), n = min(|c|,|s|),
the chord is the trapezoid min(1/m, max(0, ((m+n)/2 - |tau|)/(m n))) for
n > 0 and, for an axis-aligned line (n = 0), 1 inside, 1/2 on an edge (the
reading for a ray lying on a pixel edge) and 0 outside.
"""
import math

import numpy as np
import pytest

from synth import bin_centres


def chord_closed_form(c, s, tau, size=1.0):
    """Chord of the line {p.(c,s) = tau} through a square of side `size`
    centred at the origin."""
    m, n = max(abs(c), abs(s)), min(abs(c), abs(s))
    t = abs(tau) / size
    if n == 0.0:
        w = 1.0 if t < 0.5 else (0.5 if t == 0.5 else 0.0)
    else:
        w = min(1.0 / m, max(0.0, ((m + n) / 2.0 - t) / (m * n)))
    return w * size


def dense_closed_form(g):
    n = g.n
    h = 0.5 * (n - 1)
    t = bin_centres(g.n_bins)
    A = np.zeros((g.L, g.J))
    for a in range(g.n_angles):
        c, s = g.cos[a], g.sin[a]
        for b in range(g.n_bins):
            for i in range(n):
                for j in range(n):
                    tau = t[b] - ((j - h) * c + (h - i) * s)
                    A[a * g.n_bins + b, i * n + j] = chord_closed_form(c, s, tau)
    return A


@pytest.mark.parametrize("n,na,nb", [(4, 8, 7), (5, 12, 8), (8, 16, 15), (6, 30, 11)])
def test_siddon_equals_trapezoid(oracle_lib, n, na, nb):
    g = oracle_lib.Geometry(n, na, nb)
    A = g.dense()
    B = dense_closed_form(g)
    assert np.max(np.abs(A - B)) <= 1e-12


def test_trig_table_snaps_axes(oracle_lib):
    g = oracle_lib.Geometry(8, 180, 13)
    assert g.cos[0] == 1.0 and g.sin[0] == 0.0
    assert g.cos[90] == 0.0 and g.sin[90] == 1.0
    assert abs(g.cos[45] - math.sqrt(0.5)) < 1e-15


@pytest.mark.parametrize("n,na,nb", [(16, 24, 25), (15, 20, 23), (32, 45, 47)])
def test_constant_image(oracle_lib, n, na, nb):
    """A applied to the all-ones image is the chord through the whole N x N
    square, i.e. N times the unit-square chord at tau/N."""
    g = oracle_lib.Geometry(n, na, nb)
    y = g.project(np.ones(g.J)).reshape(na, nb)
    t = bin_centres(nb)
    for a in range(na):
        for b in range(nb):
            ref = chord_closed_form(g.cos[a], g.sin[a], t[b], size=float(n))
            assert abs(y[a, b] - ref) <= 1e-11, (a, b, y[a, b], ref)


@pytest.mark.parametrize("blk,i0,j0", [(3, 2, 5), (4, 7, 1), (1, 5, 5)])
def test_aligned_block(oracle_lib, blk, i0, j0):
    """An s x s block of ones aligned with the pixel grid projects to
    s times the unit-square chord at (t - proj(block centre))/s."""
    n, na, nb = 12, 30, 19
    g = oracle_lib.Geometry(n, na, nb)
    x = np.zeros((n, n))
    x[i0:i0 + blk, j0:j0 + blk] = 1.0
    y = g.project(x).reshape(na, nb)
    h = 0.5 * (n - 1)
    xc = (j0 + 0.5 * (blk - 1)) - h
    yc = h - (i0 + 0.5 * (blk - 1))
    t = bin_centres(nb)
    for a in range(na):
        c, s = g.cos[a], g.sin[a]
        for b in range(nb):
            ref = chord_closed_form(c, s, t[b] - (xc * c + yc * s), size=float(blk))
            assert abs(y[a, b] - ref) <= 1e-11


@pytest.mark.parametrize("n,nb", [(16, 25), (16, 24), (15, 23)])
def test_axis_angles_conserve_mass(oracle_lib, n, nb):
    """At 0 and 90 degrees every pixel's unit chord splits over the bins
    without loss, so the projection sums to the image sum."""
    g = oracle_lib.Geometry(n, 4, nb)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, g.J)
    y = g.project(x).reshape(4, nb)
    assert abs(y[0].sum() - x.sum()) <= 1e-12 * g.J
    assert abs(y[2].sum() - x.sum()) <= 1e-12 * g.J


def test_edge_ray_halves(oracle_lib):
    """Even N, odd n_b: every 0-degree ray lies on a column edge, so a single
    bright pixel is seen at half weight by the two rays along its edges."""
    n, nb = 8, 9
    g = oracle_lib.Geometry(n, 2, nb)
    x = np.zeros((n, n))
    x[3, 4] = 1.0
    y = g.project(x).reshape(2, nb)
    nz = np.nonzero(y[0])[0]
    assert list(y[0][nz]) == [0.5, 0.5]
    # The same pixel back-projects consistently (adjoint at the tie).
    r = np.zeros((2, nb))
    r[0, nz[0]] = 1.0
    bp = g.backproject(r).reshape(n, n)
    assert bp[3, 4] == 0.5 and bp[3, 3] == 0.5


@pytest.mark.parametrize("geom", [(7, 9, 11), (8, 12, 10), (33, 45, 49), (64, 90, 95),
                                  (5, 1, 8), (20, 7, 12)])
def test_mirror_symmetry(oracle_lib, geom):
    """The symmetry the mirrored backprojector relies on: mirroring the image
    about its vertical axis maps the ray at angle theta_a and bin b to the ray
    at angle theta_{n_a - a} and the same bin (a >= 1), and angle 0's rays to
    the reversed bins of angle 0. So A^T of the sinogram with its rows
    mirrored that way is A^T y mirrored, and A of the mirrored image is A x
    with its rows mirrored, up to the rounding of the trig table."""
    n, na, nb = geom
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(n + na)
    x = rng.uniform(-1, 1, (n, n))
    y = rng.uniform(-1, 1, (na, nb))

    def mirror_rows(s):
        m = np.empty_like(s)
        m[0] = s[0, ::-1]
        m[1:] = s[:0:-1]
        return m

    aty = g.backproject(y.reshape(-1)).reshape(n, n)
    aty_m = g.backproject(mirror_rows(y).reshape(-1)).reshape(n, n)
    assert np.linalg.norm(aty_m - aty[:, ::-1]) <= 1e-13 * np.linalg.norm(aty)
    ax = g.project(x.reshape(-1)).reshape(na, nb)
    ax_m = g.project(x[:, ::-1].reshape(-1)).reshape(na, nb)
    assert np.linalg.norm(ax_m - mirror_rows(ax)) <= 1e-13 * np.linalg.norm(ax)
    # a plausible mistake fails: pairing angle a with n_a - 1 - a instead
    if na > 2:
        wrong = y[::-1]
        aty_w = g.backproject(wrong.reshape(-1)).reshape(n, n)
        assert np.linalg.norm(aty_w - aty[:, ::-1]) > 1e-3 * np.linalg.norm(aty)
