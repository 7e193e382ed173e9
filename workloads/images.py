"""Seeded synthetic polar images (float32 [n_images][n_azimuth][n_bins]) for
the epilogue: the value distribution of a radar scan's image without tracing
one.  Each column holds a few clusters of returns (a surface seen over a few
neighbouring bins) with energies log-uniform over 1e-12..1 of the emitted
energy, a sparse scatter of weak multipath returns, exact zeros elsewhere,
and rare values at or above 1 (a column whose returns pile up in one bin)."""
import numpy as np


def polar_images(seed: int, n_images: int, n_azimuth: int, n_bins: int, clusters: int = 6,
                 scatter: float = 0.02) -> np.ndarray:
    rng = np.random.default_rng(seed)
    img = np.zeros((n_images, n_azimuth, n_bins), np.float32)
    if n_bins == 0 or n_azimuth == 0:
        return img
    for i in range(n_images):
        for k in range(n_azimuth):
            row = img[i, k]
            for _ in range(rng.integers(0, clusters + 1)):
                c = int(rng.integers(0, n_bins))
                width = int(rng.integers(1, 6))
                lo, hi = max(0, c - width), min(n_bins, c + width + 1)
                peak = 10.0 ** rng.uniform(-8, 0)
                fall = np.exp(-0.5 * ((np.arange(lo, hi) - c) / max(width / 2, 0.5)) ** 2)
                row[lo:hi] += (peak * fall).astype(np.float32)
            m = rng.random(n_bins) < scatter
            row[m] += (10.0 ** rng.uniform(-12, -4, int(m.sum()))).astype(np.float32)
    hot = rng.random(img.shape) < 1e-4
    img[hot] = rng.uniform(1.0, 2.0, int(hot.sum())).astype(np.float32)
    return img
