"""The seeded input generator: conventions, reproducibility, statistics."""
import math

import numpy as np

from paper_2606_02413_amd import corona


def test_ba_profile_values():
    # Baumbach-Allen at the photosphere: 1e8 * (2.99 + 1.55 + 0.036)
    assert abs(corona.ba_density(1.0) - 4.576e8) < 1.0
    assert corona.ba_density(2.0) < corona.ba_density(1.5)


def test_vertex_conventions():
    r, th, ph = corona.vertex_coords(5, 4, 8, 1.0, 3.0)
    assert r[0] == 1.0 and abs(r[-1] - 3.0) < 1e-15
    assert np.allclose(np.diff(np.log(r)), math.log(3.0) / 4)
    assert np.allclose(th, (np.arange(4) + 0.5) * math.pi / 4)
    assert np.allclose(ph, 2 * math.pi * np.arange(8) / 8)
    xyz = corona.vertex_xyz(5, 4, 8, 1.0, 3.0)
    assert np.allclose(np.linalg.norm(xyz, axis=-1), r[:, None, None])


def test_frequencies_and_seeds():
    f = corona.log_freqs(8)
    assert f[0] == 40e6 and abs(f[-1] - 800e6) < 1e-3
    assert abs(f[3] / 1e6 - 144.426) < 1e-3
    a = corona.seeded_pixels(512, 4096, 3000)
    assert len(np.unique(a)) == 4096 and a.max() < 512 * 512
    assert np.array_equal(a, corona.seeded_pixels(512, 4096, 3000))


def test_structured_reproducible_and_statistics():
    a = corona.structured(nr=32, nt=16, nph=32, r_in=1.0, r_max=3.0, seed=7, n_ar=2, n_feat=256)
    b = corona.structured(nr=32, nt=16, nph=32, r_in=1.0, r_max=3.0, seed=7, n_ar=2, n_feat=256)
    assert np.array_equal(a.ne, b.ne) and np.array_equal(a.te, b.te)
    c = corona.structured(nr=32, nt=16, nph=32, r_in=1.0, r_max=3.0, seed=8, n_ar=2, n_feat=256)
    assert not np.array_equal(a.ne, c.ne)
    assert a.ne.dtype == np.float32 and a.ne.shape == (32, 16, 32)
    assert (a.ne > 0).all() and (a.te >= 1.2e6 * (1 - 1e-7)).all() and a.te.max() <= 3e6
    # log of the density ratio to the profile is 0.3 g (+ active regions)
    r, _, _ = corona.vertex_coords(32, 16, 32, 1.0, 3.0)
    g = np.log(a.ne / corona.ba_density(r)[:, None, None]) / 0.3
    outer = g[20:]  # away from the active regions (r > 1.9)
    assert abs(outer.mean()) < 0.3 and 0.5 < outer.std() < 1.5
