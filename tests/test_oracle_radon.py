"""The oracle's A against the closed-form Radon transform of ellipses.

A applied to the pixel-averaged phantom approximates the exact line
integrals; the discrepancy is discretisation error, small and shrinking as
the grid is refined at fixed physical phantom."""
import numpy as np
import pytest

from synth import analytic_sinogram, random_ellipses, rasterize


def _rel_err(oracle_lib, ells, n, na, nb, ss=8):
    g = oracle_lib.Geometry(n, na, nb, threads=0)
    x = rasterize(ells, n, supersample=ss)
    y = analytic_sinogram(ells, n, na, nb)
    # pixel units scale with n: compare in normalised units
    ya = g.project(x)
    return np.linalg.norm(ya - y.reshape(-1)) / np.linalg.norm(y)


@pytest.mark.slow
def test_ellipse_projection_converges(oracle_lib):
    rng = np.random.default_rng(1001)
    ells = random_ellipses(rng, 10)
    errs = []
    for n in (32, 64, 128):
        na = 45
        nb = int(np.ceil(np.sqrt(2) * n)) + 4
        errs.append(_rel_err(oracle_lib, ells, n, na, nb))
    assert errs[1] < 0.05
    assert errs[2] < errs[1] < errs[0]
    # at least ~linear decrease as the grid is refined
    assert errs[2] < 0.75 * errs[1]


def test_single_disk_mass(oracle_lib):
    """The projection of a centred disk keeps the disk's mass at every angle
    (up to the rasterisation's area error)."""
    from synth.phantom import Ellipse
    n = 64
    ells = [Ellipse(0.0, 0.0, 0.5, 0.5, 0.0, 1.0)]
    g = oracle_lib.Geometry(n, 12, 95)
    x = rasterize(ells, n, supersample=16)
    y = g.project(x).reshape(12, 95)
    area = np.pi * (0.5 * 32) ** 2
    for a in (0, 6):
        assert abs(y[a].sum() - x.sum()) <= 1e-9 * area
    assert abs(x.sum() - area) / area < 2e-3
    ya = analytic_sinogram(ells, n, 12, 95)
    assert np.linalg.norm(y - ya) / np.linalg.norm(ya) < 0.05
