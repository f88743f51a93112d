"""ctypes binding of the FP64 C oracle operators (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_ops.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle_ops.c with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = C.CDLL(_LIB)
    i, d, ll = C.c_int, C.c_double, C.c_longlong
    lib.or_trig.argtypes = [i, _dp, _dp]
    lib.or_max_threads.restype = i
    lib.or_project.argtypes = [i, i, i, _dp, _dp, _dp, _dp, i]
    lib.or_project_rays.argtypes = [i, i, i, _dp, _dp, _dp, _lp, ll, _dp, i]
    lib.or_dense_matrix.argtypes = [i, i, i, _dp, _dp, _dp]
    lib.or_backproject.argtypes = [i, i, i, _dp, _dp, _dp, _dp, i]
    lib.or_backproject_pixels.argtypes = [i, i, i, _dp, _dp, _dp, _lp, ll, _dp, i]
    lib.or_tv.argtypes = [i, _dp, d]
    lib.or_tv.restype = d
    lib.or_tv_subgrad.argtypes = [i, _dp, d, _dp]
    lib.or_filter_kernel.argtypes = [i, i, d, _dp]
    lib.or_filter.argtypes = [i, i, _dp, _dp, _dp, i]
    for name in ("or_trig", "or_project", "or_project_rays", "or_dense_matrix",
                 "or_backproject", "or_backproject_pixels", "or_filter"):
        getattr(lib, name).restype = i
    lib.or_tv_subgrad.restype = None
    lib.or_filter_kernel.restype = None
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().or_max_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Geometry:
    """Parallel-beam geometry: N x N unit pixels, n_angles angles uniform over
    [0, pi), n_bins unit bins centred on the rotation axis."""

    def __init__(self, n: int, n_angles: int, n_bins: int, threads: int = 0):
        if n <= 0 or n_angles <= 0 or n_bins <= 0:
            raise ValueError("sizes must be positive")
        self.n, self.n_angles, self.n_bins = int(n), int(n_angles), int(n_bins)
        self.threads = int(threads)
        self.cos = np.empty(n_angles)
        self.sin = np.empty(n_angles)
        if _load().or_trig(n_angles, self.cos, self.sin) != 0:
            raise RuntimeError("or_trig failed")

    @property
    def J(self) -> int:
        return self.n * self.n

    @property
    def L(self) -> int:
        return self.n_angles * self.n_bins

    def project(self, x) -> np.ndarray:
        """y = A x (flat length L)."""
        x = _f64(x).reshape(-1)
        assert x.size == self.J
        y = np.empty(self.L)
        rc = _load().or_project(self.n, self.n_angles, self.n_bins, self.cos, self.sin, x, y,
                                self.threads)
        if rc:
            raise RuntimeError("or_project failed")
        return y

    def project_rays(self, x, rays) -> np.ndarray:
        x = _f64(x).reshape(-1)
        rays = np.ascontiguousarray(rays, dtype=np.int64)
        out = np.empty(rays.size)
        rc = _load().or_project_rays(self.n, self.n_angles, self.n_bins, self.cos, self.sin, x,
                                     rays, rays.size, out, self.threads)
        if rc:
            raise RuntimeError("or_project_rays failed")
        return out

    def backproject(self, y) -> np.ndarray:
        """x = A^T y (flat length J)."""
        y = _f64(y).reshape(-1)
        assert y.size == self.L
        x = np.empty(self.J)
        _load().or_backproject(self.n, self.n_angles, self.n_bins, self.cos, self.sin, y, x,
                               self.threads)
        return x

    def backproject_pixels(self, y, pixels) -> np.ndarray:
        y = _f64(y).reshape(-1)
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        out = np.empty(pixels.size)
        _load().or_backproject_pixels(self.n, self.n_angles, self.n_bins, self.cos, self.sin, y,
                                      pixels, pixels.size, out, self.threads)
        return out

    def dense(self) -> np.ndarray:
        """Dense L x J system matrix (tiny problems only)."""
        if self.L * self.J > 60_000_000:
            raise ValueError("problem too large for a dense matrix")
        A = np.empty((self.L, self.J))
        if _load().or_dense_matrix(self.n, self.n_angles, self.n_bins, self.cos, self.sin, A):
            raise RuntimeError("or_dense_matrix failed")
        return A

    # -- total variation -------------------------------------------------
    def tv(self, x, kappa: float = 0.0) -> float:
        x = _f64(x).reshape(-1)
        return float(_load().or_tv(self.n, x, float(kappa)))

    def tv_subgrad(self, x, kappa: float = 0.0) -> np.ndarray:
        x = _f64(x).reshape(-1)
        s = np.empty(self.J)
        _load().or_tv_subgrad(self.n, x, float(kappa), s)
        return s

    # -- preconditioning filter ------------------------------------------
    def filter_pad(self) -> int:
        """P = 2^ceil(log2(2 n_bins)): zero padding that avoids wrap-around."""
        return 1 << int(np.ceil(np.log2(2 * self.n_bins)))

    def default_mu(self) -> float:
        return 2.0 * np.pi / self.filter_pad()

    def filter_kernel(self, mu: float | None = None) -> np.ndarray:
        mu = self.default_mu() if mu is None else float(mu)
        k = np.empty(self.n_bins)
        _load().or_filter_kernel(self.n_bins, self.filter_pad(), mu, k)
        return k

    def filter(self, r, mu: float | None = None, kernel=None) -> np.ndarray:
        """F^T C F r for each projection (row of the angle-major sinogram)."""
        r = _f64(r).reshape(-1)
        k = self.filter_kernel(mu) if kernel is None else _f64(kernel)
        out = np.empty(self.L)
        _load().or_filter(self.n_angles, self.n_bins, k, r, out, self.threads)
        return out
