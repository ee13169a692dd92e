"""Plain FP64 definitions of the map post-processing (test infrastructure only).

Only the tests import this module.  Maps follow the tracer's layout
[n_maps][nv][nu] with pixel centres -half + (j + 1/2) 2 half / n.

- disc_mean: the mean T_b over the pixels whose centre lies within a radius of
  the image centre (the disc-centre spectrum of Sec. 3.4.1).
- beam_convolve: convolution with a Gaussian beam of given FWHM sampled at
  pixel offsets (the convolved synthetic maps of Sec. 3.3), zero beyond the
  image, normalised by the sum of the untruncated sampled Gaussian.
"""
from __future__ import annotations

import math

import numpy as np


def pixel_centres(n, half):
    return -half + (np.arange(n) + 0.5) * (2.0 * half / n)


def disc_mean(maps, half_u, half_v, radius):
    maps = np.asarray(maps, dtype=np.float64)
    nv, nu = maps.shape[-2:]
    u = pixel_centres(nu, half_u)
    v = pixel_centres(nv, half_v)
    inside = (u[None, :] ** 2 + v[:, None] ** 2) < radius * radius
    if not inside.any():
        return np.zeros(maps.shape[0])
    return np.array([m[inside].mean() for m in maps])


def gaussian_taps(sigma, n):
    """Sampled Gaussian weights for offsets -(n-1) .. n-1, normalised by the sum
    over all integer offsets (taken to 40 sigma, beyond which the terms are
    below 1e-300)."""
    k = np.arange(-(n - 1), n, dtype=np.float64)
    if sigma == 0.0:
        return (k == 0).astype(np.float64)
    kk = np.arange(-int(math.ceil(40 * sigma)) - 1, int(math.ceil(40 * sigma)) + 2, dtype=np.float64)
    norm = np.exp(-kk * kk / (2.0 * sigma * sigma)).sum()
    return np.exp(-k * k / (2.0 * sigma * sigma)) / norm


def _axis_matrix(n, sigma):
    """out = G @ x for one axis: G[p, q] = w(q - p) (zero beyond the image)."""
    taps = gaussian_taps(sigma, n)
    idx = np.arange(n)
    return taps[(idx[None, :] - idx[:, None]) + (n - 1)]


def beam_convolve(maps, half_u, half_v, fwhm):
    maps = np.asarray(maps, dtype=np.float64)
    nv, nu = maps.shape[-2:]
    out = np.empty_like(maps)
    to_sigma = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    for m in range(maps.shape[0]):
        su = fwhm[m] * to_sigma / (2.0 * half_u / nu)
        sv = fwhm[m] * to_sigma / (2.0 * half_v / nv)
        out[m] = _axis_matrix(nv, sv) @ maps[m] @ _axis_matrix(nu, su).T
    return out
