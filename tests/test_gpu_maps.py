"""Map post-processing on the GPU (beam convolution, disc-centre mean) against
the plain FP64 definitions in oracle/maps_oracle.py, through the C ABI.

Bar: beam convolution max |gpu - oracle| <= 5e-6 max |map| (FP32 sums of up
to ~200 taps, and the beam cut at 5 sigma, whose tail mass is 6e-7); disc mean
relative 1e-12 (FP64 sums of FP32 values, only the order differs)."""
import numpy as np
import pytest

from oracle import maps_oracle as MO
from paper_2606_02413_amd import corona
from tests import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun
    return rtsun


def _maps(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 2.0e6, size=shape).astype(np.float32)


def test_beam_matches_the_definition_on_ragged_maps(R):
    import torch
    nv, nu, hu, hv = 29, 37, 3.0, 2.2
    m = _maps((4, nv, nu), 11)
    m[3] = 0.0
    m[3, 0, 0] = 1.0e6          # a delta at a corner: the cut at the image edge
    m[3, 14, 36] = 2.0e6        # and at an edge
    fwhm = [0.3, 0.0, 1.5, 0.45]
    im = R.image_desc(nu, hu, nv=nv, half_v=hv)
    print("case beam ragged", flush=True)
    got = R.beam_convolve(torch.from_numpy(m).cuda(), im, fwhm).cpu().numpy().astype(np.float64)
    ref = MO.beam_convolve(m, hu, hv, fwhm)
    err = np.abs(got - ref).max(axis=(1, 2)) / np.abs(m).max(axis=(1, 2))
    print("beam max err / max map", err, flush=True)
    assert np.all(err <= 5e-6)
    assert np.array_equal(got[1], m[1].astype(np.float64))


def test_beam_and_spectrum_of_traced_maps(R):
    """Maps of the structured model at three frequencies, convolved with the beam
    of a 15 km baseline, and their disc-centre means."""
    import torch
    cor = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=11, n_ar=4, n_feat=256)
    m = R.Model.from_corona(cor)
    freqs = np.array([40e6, 80e6, 150e6])
    im = R.image_desc(96, 3.0)
    print("case beam / spectrum of traced maps", flush=True)
    tb = R.trace_maps([m], freqs, im, R.params(ds_max=0.01, n_floor=0.1), info=False, stats=False)["tb"][0]
    fw = R.beam_fwhm(freqs, 15e3)
    got = R.beam_convolve(tb, im, fw).cpu().numpy().astype(np.float64)
    host = tb.cpu().numpy()
    ref = MO.beam_convolve(host, 3.0, 3.0, fw)
    assert np.abs(got - ref).max() <= 5e-6 * np.abs(host).max()
    for radius in (0.5, 1.2):
        spec = R.disc_mean(tb, im, radius).cpu().numpy()
        ref_s = MO.disc_mean(host, 3.0, 3.0, radius)
        print(f"spectrum r<{radius}", spec, flush=True)
        np.testing.assert_allclose(spec, ref_s, rtol=1e-12, atol=0)
    m.close()


def test_disc_mean_ragged_and_empty(R):
    import torch
    nv, nu = 31, 20
    m = _maps((3, nv, nu), 12)
    im = R.image_desc(nu, 1.0, nv=nv, half_v=1.6)
    print("case disc mean", flush=True)
    got = R.disc_mean(torch.from_numpy(m).cuda(), im, 0.7).cpu().numpy()
    np.testing.assert_allclose(got, MO.disc_mean(m, 1.0, 1.6, 0.7), rtol=1e-12, atol=0)
    # a radius smaller than the distance of every pixel centre: 0
    got0 = R.disc_mean(torch.from_numpy(m).cuda(), im, 1e-3).cpu().numpy()
    assert np.all(got0 == 0.0) and np.all(MO.disc_mean(m, 1.0, 1.6, 1e-3) == 0.0)
