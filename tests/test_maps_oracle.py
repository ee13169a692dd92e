"""Pins of the map post-processing oracle (CPU): a delta becomes the sampled
Gaussian with unit mass and variance sigma^2 along each axis (the
Poisson-summation error of a sampled Gaussian is below 1e-6 for sigma >= 1.6
pixels), a constant map stays
constant away from the edges, the beam is separable and symmetric, and the
disc mean is the mean of the pixel centres inside the circle (indicator and
odd-function checks)."""
import math

import numpy as np

from oracle import maps_oracle as MO

TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def test_delta_becomes_a_unit_gaussian_with_variance_sigma2():
    n, hu, hv = 101, 2.0, 1.5          # pixels of 0.0396 x 0.0297 R_sun
    fwhm = 0.15
    su, sv = fwhm * TO_SIGMA / (2 * hu / n), fwhm * TO_SIGMA / (2 * hv / n)   # 1.61, 2.15 pixels
    m = np.zeros((1, n, n))
    m[0, 50, 50] = 1.0
    out = MO.beam_convolve(m, hu, hv, [fwhm])[0]
    assert abs(out.sum() - 1.0) < 1e-12
    k = np.arange(n) - 50
    var_u = (out.sum(axis=0) * k * k).sum()    # along u (columns)
    var_v = (out.sum(axis=1) * k * k).sum()    # along v (rows)
    assert abs(var_u - su ** 2) < 1e-6 * su ** 2 and abs(var_v - sv ** 2) < 1e-6 * sv ** 2
    assert np.allclose(out, out[::-1, ::-1], rtol=0, atol=1e-15)
    # separable: the outer product of its marginals
    assert np.allclose(out, np.outer(out.sum(axis=1), out.sum(axis=0)), rtol=0, atol=1e-15)


def test_constant_stays_constant_away_from_the_edges_and_fwhm0_is_identity():
    n, half = 64, 1.0
    m = np.full((2, n, n), 3.0)
    fwhm = [0.05, 0.0]
    out = MO.beam_convolve(m, half, half, fwhm)
    sig = 0.05 * TO_SIGMA / (2 * half / n)
    r = int(math.ceil(12 * sig))
    assert np.allclose(out[0, r:-r, r:-r], 3.0, rtol=1e-13, atol=0)
    assert out[0, 0, 0] < 3.0                     # the dark sky beyond the edge
    assert np.array_equal(out[1], m[1])


def test_disc_mean_definition_checks():
    nv, nu, hu, hv = 40, 60, 3.0, 2.0
    u = MO.pixel_centres(nu, hu)
    v = MO.pixel_centres(nv, hv)
    inside = (u[None, :] ** 2 + v[:, None] ** 2) < 0.5 ** 2
    ind = inside.astype(np.float64)[None] * 7.0
    odd = np.broadcast_to(u[None, :], (nv, nu))[None]
    mixed = np.where(inside, 2.0, 100.0)[None]
    res = MO.disc_mean(np.concatenate([ind, odd, mixed]), hu, hv, 0.5)
    assert res[0] == 7.0 and abs(res[1]) < 1e-15 and res[2] == 2.0
    assert inside.sum() > 0
