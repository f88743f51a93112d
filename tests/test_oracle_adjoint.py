"""Adjoint identity of the oracle's independent ray-driven A and pixel-driven
A^T: <A x, y> = <x, A^T y> to 1e-12 relative."""
import numpy as np
import pytest


@pytest.mark.parametrize("n,na,nb", [(8, 16, 15), (9, 13, 14), (33, 50, 49), (64, 90, 95),
                                     (40, 7, 30), (16, 180, 25)])
def test_adjoint_identity(oracle_lib, n, na, nb):
    g = oracle_lib.Geometry(n, na, nb)
    rng = np.random.default_rng(n * 1000 + na)
    for _ in range(3):
        x = rng.uniform(-1, 1, g.J)
        y = rng.uniform(-1, 1, g.L)
        lhs = float(g.project(x) @ y)
        rhs = float(x @ g.backproject(y))
        scale = float(np.abs(g.project(np.abs(x))) @ np.abs(y))
        assert abs(lhs - rhs) <= 1e-12 * scale


def test_dense_transpose(oracle_lib):
    g = oracle_lib.Geometry(10, 17, 16)
    A = g.dense()
    rng = np.random.default_rng(1)
    y = rng.standard_normal(g.L)
    assert np.max(np.abs(A.T @ y - g.backproject(y))) <= 1e-12


def test_sampled_rays_and_pixels(oracle_lib):
    g = oracle_lib.Geometry(24, 30, 37)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(g.J)
    y = rng.standard_normal(g.L)
    rays = rng.choice(g.L, 50, replace=False)
    pix = rng.choice(g.J, 50, replace=False)
    assert np.array_equal(g.project_rays(x, rays), g.project(x)[rays])
    assert np.array_equal(g.backproject_pixels(y, pix), g.backproject(y)[pix])


def test_narrow_detector(oracle_lib):
    """A detector narrower than the image: rays miss nothing they should see,
    and the adjoint still holds."""
    g = oracle_lib.Geometry(20, 12, 9)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(g.J)
    y = rng.standard_normal(g.L)
    assert abs(float(g.project(x) @ y) - float(x @ g.backproject(y))) <= 1e-12 * g.J
