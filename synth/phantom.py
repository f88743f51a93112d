"""Random-ellipse phantoms and their exact parallel-beam line integrals.

Coordinate conventions (shared by the FP64 oracle and the HIP library, each of
which implements them on its own):

* The image has N x N unit pixels centred at the origin. Pixel (i, j), row i
  counted from the top and column j from the left, has centre
  x_j = j - (N-1)/2, y_i = (N-1)/2 - i and flat index i*N + j.
* Angle a of n_a is theta_a = a*pi/n_a (uniform over [0, 180 degrees), the
  paper's experimental set-up in its Experimental Results section).
* Bin b of n_b has centre t_b = b - (n_b-1)/2 (unit width).
* Ray (a, b) is the line {x cos theta_a + y sin theta_a = t_b}; the sinogram is
  angle-major, flat index a*n_b + b.

Ellipses are drawn in normalised coordinates in which the unit disk is the
inscribed disk of radius N/2 pixels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Ellipse:
    """One ellipse in normalised coordinates (unit disk = inscribed disk)."""

    x0: float
    y0: float
    a: float      # semi-axis along the rotated x direction
    b: float      # semi-axis along the rotated y direction
    phi: float    # rotation, radians
    rho: float    # additive density


def default_bins(n: int, extra: int) -> int:
    """Detector bins that cover the image diagonal: ceil(sqrt(2) N) + extra."""
    return int(math.ceil(math.sqrt(2.0) * n)) + extra


def geometry_angles(n_angles: int) -> np.ndarray:
    """theta_a = a*pi/n_a, a = 0..n_a-1 (radians, float64)."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


def bin_centres(n_bins: int) -> np.ndarray:
    """t_b = b - (n_b-1)/2 in pixel units (float64)."""
    return np.arange(n_bins, dtype=np.float64) - 0.5 * (n_bins - 1)


def random_ellipses(rng: np.random.Generator, count: int,
                    semi=(0.05, 0.6), intensity=(0.1, 1.0)) -> list[Ellipse]:
    """Draw `count` ellipses: centre uniform in the unit disk, semi-axes
    uniform in `semi`, rotation uniform in [0, pi), density +-U[intensity]
    with an equiprobable sign. A draw is rejected unless the ellipse lies
    inside the unit disk (|centre| + max semi-axis <= 1), which keeps all mass
    inside the image and inside the detector's field of view."""
    out: list[Ellipse] = []
    while len(out) < count:
        r = math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2.0 * math.pi)
        x0, y0 = r * math.cos(ang), r * math.sin(ang)
        a = rng.uniform(*semi)
        b = rng.uniform(*semi)
        phi = rng.uniform(0.0, math.pi)
        mag = rng.uniform(*intensity)
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        if r + max(a, b) > 1.0:
            continue
        out.append(Ellipse(x0, y0, a, b, phi, sign * mag))
    return out


def texture_disks(rng: np.random.Generator, n: int, amplitude: float,
                  spacing_px: float = 4.0, radius_px: float = 1.5) -> list[Ellipse]:
    """A fine random texture made of small disks: one disk per cell of a
    jittered grid with `spacing_px` pixel pitch inside the inscribed disk,
    radius `radius_px` pixels, density uniform in [-amplitude, amplitude].
    Being disks, their line integrals stay exact and analytic."""
    half = 0.5 * n
    rad = radius_px / half
    cells = int(n // spacing_px)
    out: list[Ellipse] = []
    for ci in range(cells):
        for cj in range(cells):
            px = -half + (cj + rng.uniform(0.25, 0.75)) * spacing_px
            py = -half + (ci + rng.uniform(0.25, 0.75)) * spacing_px
            x0, y0 = px / half, py / half
            if math.hypot(x0, y0) + rad > 1.0:
                continue
            out.append(Ellipse(x0, y0, rad, rad, 0.0,
                               rng.uniform(-amplitude, amplitude)))
    return out


def _params(ellipses, n):
    half = 0.5 * n
    e = np.array([[el.x0 * half, el.y0 * half, el.a * half, el.b * half,
                   el.phi, el.rho] for el in ellipses], dtype=np.float64)
    return e.reshape(-1, 6)


def analytic_sinogram(ellipses, n: int, n_angles: int, n_bins: int) -> np.ndarray:
    """Exact line integrals of the ellipse phantom along every ray.

    For an ellipse with centre c, semi-axes (A, B), rotation phi and density
    rho, the integral along {x cos t + y sin t = s} is
    2 rho A B sqrt(w^2 - d^2) / w^2 where d = s - c.(cos t, sin t) and
    w^2 = A^2 cos^2(t - phi) + B^2 sin^2(t - phi), and 0 when d^2 > w^2.
    Returns an (n_angles, n_bins) float64 array in pixel units."""
    e = _params(ellipses, n)
    th = geometry_angles(n_angles)
    t = bin_centres(n_bins)
    ct, st = np.cos(th), np.sin(th)
    y = np.zeros((n_angles, n_bins), dtype=np.float64)
    small = e[np.maximum(e[:, 2], e[:, 3]) < 4.0]
    large = e[np.maximum(e[:, 2], e[:, 3]) >= 4.0]
    for x0, y0, A, B, phi, rho in large:
        d = t[None, :] - (x0 * ct + y0 * st)[:, None]
        w2 = (A * np.cos(th - phi)) ** 2 + (B * np.sin(th - phi)) ** 2
        arg = w2[:, None] - d * d
        val = np.where(arg > 0.0, 2.0 * rho * A * B * np.sqrt(np.maximum(arg, 0.0)) / w2[:, None], 0.0)
        y += val
    if len(small):
        # Small ellipses touch only a few bins per angle: scatter those.
        x0, y0, A, B, phi, rho = (small[:, k] for k in range(6))
        hb = 0.5 * (n_bins - 1)
        reach = int(math.ceil(max(np.max(A), np.max(B)))) + 1
        for ia in range(n_angles):
            w2 = (A * np.cos(th[ia] - phi)) ** 2 + (B * np.sin(th[ia] - phi)) ** 2
            proj = x0 * ct[ia] + y0 * st[ia]
            b0 = np.floor(proj + hb).astype(np.int64)
            for off in range(-reach, reach + 2):
                bb = b0 + off
                ok = (bb >= 0) & (bb < n_bins)
                d = (bb - hb) - proj
                arg = w2 - d * d
                val = np.where(ok & (arg > 0.0),
                               2.0 * rho * A * B * np.sqrt(np.maximum(arg, 0.0)) / w2, 0.0)
                np.add.at(y[ia], np.clip(bb, 0, n_bins - 1), val)
    return y


def rasterize(ellipses, n: int, supersample: int = 8) -> np.ndarray:
    """Pixel image of the phantom: each pixel holds the phantom's average over
    its unit square, estimated on a supersample x supersample grid of points.
    Returns an (n, n) float64 array, row 0 at the top."""
    e = _params(ellipses, n)
    img = np.zeros((n, n), dtype=np.float64)
    ss = supersample
    sub = (np.arange(ss) + 0.5) / ss - 0.5
    h = 0.5 * (n - 1)
    for x0, y0, A, B, phi, rho in e:
        r = max(A, B) + 1.0
        j_lo = max(0, int(math.floor(x0 - r + h)))
        j_hi = min(n - 1, int(math.ceil(x0 + r + h)))
        i_lo = max(0, int(math.floor(h - (y0 + r))))
        i_hi = min(n - 1, int(math.ceil(h - (y0 - r))))
        if j_lo > j_hi or i_lo > i_hi:
            continue
        jj = np.arange(j_lo, j_hi + 1)
        ii = np.arange(i_lo, i_hi + 1)
        xs = (jj[:, None] - h + sub[None, :]).reshape(-1)          # columns x subsamples
        ys = (h - ii[:, None] + sub[None, :]).reshape(-1)
        X, Y = np.meshgrid(xs, ys)
        dx, dy = X - x0, Y - y0
        cp, sp = math.cos(phi), math.sin(phi)
        u = (dx * cp + dy * sp) / A
        v = (-dx * sp + dy * cp) / B
        inside = (u * u + v * v) <= 1.0
        frac = inside.reshape(len(ii), ss, len(jj), ss).mean(axis=(1, 3))
        img[i_lo:i_hi + 1, j_lo:j_hi + 1] += rho * frac
    return img


def add_gaussian_noise(rng: np.random.Generator, y: np.ndarray, frac_of_max: float):
    """Zero-mean Gaussian noise with sigma = frac_of_max * max|y|.
    Returns (noisy y, sigma)."""
    sigma = float(frac_of_max * np.max(np.abs(y)))
    return y + sigma * rng.standard_normal(y.shape), sigma


def add_poisson_like_noise(rng: np.random.Generator, y: np.ndarray,
                           i0: float = 1e5, peak_attenuation: float = 4.0):
    """Transmission-style noise: scale s so that max(s*y) = peak_attenuation,
    expected counts lam = i0*exp(-s*y), measured counts lam + sqrt(lam)*N(0,1)
    (Gaussian with variance equal to the counts) clamped to >= 1, and the
    noisy integral -ln(counts/i0)/s. Returns (noisy y, per-ray variance
    estimate 1/(s^2 lam))."""
    s = peak_attenuation / float(np.max(y))
    lam = i0 * np.exp(-s * y)
    counts = np.maximum(lam + np.sqrt(lam) * rng.standard_normal(y.shape), 1.0)
    noisy = -np.log(counts / i0) / s
    var = 1.0 / (s * s * lam)
    return noisy, var
