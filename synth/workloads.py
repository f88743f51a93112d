"""Seeded workloads shaped like the paper's experiment (parallel beam, angles
uniform over [0, 180 degrees), unit bins, noisy synthetic sinograms; see its
Experimental Results section) at five sizes.

Seeds are 1000*config + instance. Everything here is data: phantoms, exact
analytic line integrals and noise. The stopping value eps of a solve is either
the paper's own discrepancy rule (eps = L*sigma^2, the data size times the
noise variance, generalised to a per-ray variance as the sum of variances) or
a multiple of the least-squares residual, which needs a solver and is
therefore computed by the caller.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .phantom import (add_gaussian_noise, add_poisson_like_noise, analytic_sinogram,
                      default_bins, random_ellipses, rasterize, texture_disks)


@dataclass
class Workload:
    name: str
    seed: int
    n: int
    n_angles: int
    n_bins: int
    y: np.ndarray            # (n_angles, n_bins) float64 noisy sinogram
    y_clean: np.ndarray      # (n_angles, n_bins) float64 exact line integrals
    x_true: np.ndarray       # (n, n) float64 pixel-averaged phantom
    noise_var_sum: float     # sum over rays of the noise variance
    eps_discrepancy: float   # the paper's eps = L*sigma^2 (sum of variances)
    meta: dict = field(default_factory=dict)

    @property
    def J(self) -> int:
        return self.n * self.n

    @property
    def L(self) -> int:
        return self.n_angles * self.n_bins


CONFIGS = {
    # 64x64, 90 angles, 95 bins, 10 ellipses, sigma = 1 % of max (FP64 solve).
    1: dict(n=64, n_angles=90, n_bins=95, ellipses=10, noise=("gauss", 0.01)),
    # 256x256, 360 angles, 367 bins, 20 ellipses, sigma = 2 % of max.
    2: dict(n=256, n_angles=360, n_bins=367, ellipses=20, noise=("gauss", 0.02)),
    # 512x512, 720 angles, 729 bins, 30 ellipses + texture 0.02, transmission noise.
    3: dict(n=512, n_angles=720, n_bins=729, ellipses=30, texture=0.02,
            noise=("poisson", 1e5)),
}

BATCH_SIZES = (128, 256, 384, 512)
BATCH_ANGLES = (180, 360, 540, 720)
SERVE_SHAPES = ((128, 180), (256, 360), (512, 720), (1024, 1440))
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


def _finish(name, seed, n, n_angles, n_bins, ells, rng, noise, supersample=4):
    y_clean = analytic_sinogram(ells, n, n_angles, n_bins)
    kind, level = noise
    if kind == "gauss":
        y, sigma = add_gaussian_noise(rng, y_clean, level)
        var_sum = sigma * sigma * y.size
        meta = {"sigma": sigma}
    else:
        y, var = add_poisson_like_noise(rng, y_clean, i0=level)
        var_sum = float(np.sum(var))
        meta = {"i0": level}
    x_true = rasterize(ells, n, supersample=supersample)
    return Workload(name=name, seed=seed, n=n, n_angles=n_angles, n_bins=n_bins,
                    y=y, y_clean=y_clean, x_true=x_true, noise_var_sum=var_sum,
                    eps_discrepancy=var_sum, meta=meta)


def make_workload(cfg: int, instance: int = 0, *, n: int | None = None,
                  n_angles: int | None = None, n_bins: int | None = None,
                  supersample: int = 4) -> Workload:
    """Build workload `instance` of config `cfg` (1, 2 or 3). Size overrides
    keep the config's phantom and noise recipe at another geometry."""
    c = CONFIGS[cfg]
    seed = 1000 * cfg + instance
    rng = np.random.default_rng(seed)
    n = n or c["n"]
    n_angles = n_angles or c["n_angles"]
    n_bins = n_bins or c["n_bins"]
    ells = random_ellipses(rng, c["ellipses"])
    if c.get("texture"):
        ells = ells + texture_disks(rng, n, c["texture"])
    return _finish(f"cfg{cfg}", seed, n, n_angles, n_bins, ells, rng, c["noise"],
                   supersample=supersample)


def make_batch_item(instance: int, supersample: int = 2) -> Workload:
    """One solve of the batched mix: N and the angle count drawn independently
    from their sets, bins = ceil(sqrt(2) N) + 1, sigma uniform in [0.5 %, 3 %]."""
    seed = 4000 + instance
    rng = np.random.default_rng(seed)
    n = int(rng.choice(BATCH_SIZES))
    n_angles = int(rng.choice(BATCH_ANGLES))
    n_bins = default_bins(n, 1)
    ells = random_ellipses(rng, 10)
    frac = rng.uniform(0.005, 0.03)
    return _finish(f"batch{instance}", seed, n, n_angles, n_bins, ells, rng,
                   ("gauss", frac), supersample=supersample)


def make_serve_item(instance: int, supersample: int = 2, shapes=SERVE_SHAPES,
                    weights=SERVE_WEIGHTS) -> Workload:
    """One request of the served stream: (N, angles) paired index-wise from
    the size and angle sets with weights 0.4/0.3/0.2/0.1, bins =
    ceil(sqrt(2) N) + 1, sigma uniform in [0.5 %, 3 %]."""
    seed = 5000 + instance
    rng = np.random.default_rng(seed)
    k = int(rng.choice(len(shapes), p=np.asarray(weights) / np.sum(weights)))
    n, n_angles = shapes[k]
    n_bins = default_bins(n, 1)
    ells = random_ellipses(rng, 10)
    frac = rng.uniform(0.005, 0.03)
    return _finish(f"serve{instance}", seed, n, n_angles, n_bins, ells, rng,
                   ("gauss", frac), supersample=supersample)


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given mean rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def uniform_image(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(n, n))


def uniform_sinogram(rng: np.random.Generator, n_angles: int, n_bins: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(n_angles, n_bins))


def diag_len(n: int) -> float:
    return math.sqrt(2.0) * n
