"""GPU parity with the oracle across the call's parameters away from their
defaults: a non-orthogonal `up` vector (the image axes are orthonormalised),
other perturbation ratios eta (Eq. 8), a Cartesian grid with its inner sphere
enabled, and the shortest step limit."""
import numpy as np
import pytest

from paper_2606_02413_amd import corona
from tests import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun
    return rtsun


@pytest.fixture(scope="module")
def model(R):
    cor = corona.structured(nr=48, nt=24, nph=48, r_in=1.0, r_max=10.0, seed=21, n_ar=4, n_feat=256)
    m = R.Model.from_corona(cor)
    yield cor, m
    m.close()


def test_non_orthogonal_up_vector(R, orc, model):
    cor, m = model
    obs, up = (0.8, -0.3, 0.2), (0.3, 0.2, 1.0)
    kw = PU.step_kwargs(0.01, 0.1)
    print("case non-orthogonal up", flush=True)
    g = PU.gpu_trace([m], [70e6, 250e6], 20, 2.2, kw, image=R.image_desc(20, 2.2, obs_dir=obs, up=up))
    pix = np.arange(400, dtype=np.int32)
    for k, f in enumerate((70e6, 250e6)):
        o = PU.oracle_trace(orc, cor, f, 20, 2.2, pix, kw, image=orc.make_image(20, 2.2, obs_dir=obs, up=up))
        PU.compare(g["tb"][0, k].reshape(-1), g["info"][0, k].reshape(-1), o, label=f"up-{f/1e6:.0f}")


@pytest.mark.parametrize("eta", [1e-3, 1e-1])
def test_perturbation_ratio(R, orc, model, eta):
    """M is independent of eta to first order; the GPU keeps parity with the
    oracle at either end of the useful range."""
    cor, m = model
    kw = PU.step_kwargs(0.01, 0.1, eta=eta)
    print(f"case eta {eta}", flush=True)
    g = PU.gpu_trace([m], [90e6], 16, 2.0, kw)
    o = PU.oracle_trace(orc, cor, 90e6, 16, 2.0, np.arange(256, dtype=np.int32), kw)
    PU.compare(g["tb"].reshape(-1), g["info"].reshape(-1), o, label=f"eta-{eta:g}")


def test_cartesian_grid_with_inner_sphere(R, orc):
    """A Cartesian lattice around the origin with the inner sphere enabled
    (r_in = 0.8): chords that reach it end with HIT and take tb_inner."""
    n = 33
    x = np.linspace(-4.0, 4.0, n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    ne = (4e7 * np.exp(-(r - 0.8) / 0.6) + 2e6 * (1.0 + 0.2 * np.sin(1.3 * X + 0.7 * Z))).astype(np.float32)
    te = np.full((n, n, n), 1.5e6, np.float32)
    d = R.grid_desc(R.RT_GRID_CARTESIAN, (n, n, n), 0.8, 3.8, origin=(-4, -4, -4), spacing=(0.25, 0.25, 0.25))
    m = R.Model(d, ne, te)
    kw = PU.step_kwargs(0.01, 0.1)
    print("case cartesian inner sphere", flush=True)
    try:
        g = PU.gpu_trace([m], [60e6, 400e6], 16, 2.0, kw)
    finally:
        m.close()
    med = orc.OracleMedium(orc.GRID_CARTESIAN, shape=(n, n, n), r_in=0.8, r_max=3.8, ne=ne, te=te,
                           origin=(-4, -4, -4), spacing=(0.25, 0.25, 0.25))
    pix = np.arange(256, dtype=np.int32)
    for k, f in enumerate((60e6, 400e6)):
        o = orc.trace_pixels(med, orc.make_params(twin_check=True, **kw), orc.make_image(16, 2.0), f, pix)
        PU.compare(g["tb"][0, k].reshape(-1), g["info"][0, k].reshape(-1), o, label=f"cart-inner-{f/1e6:.0f}")
    assert (g["info"]["code"] == 2).any()


def test_single_step_limit(R, orc, model):
    """max_steps = 1: every traced ray stops after its first step (an exit
    needs two), with that step's transfer."""
    cor, m = model
    kw = PU.step_kwargs(0.01, 0.1, max_steps=1)
    print("case max_steps 1", flush=True)
    g = PU.gpu_trace([m], [150e6], 16, 2.0, kw)
    info = g["info"].reshape(-1)
    traced = info["code"] != 3
    assert np.all(info["code"][traced] == 4) and np.all(info["n_steps"][traced] == 1)
    o = PU.oracle_trace(orc, cor, 150e6, 16, 2.0, np.arange(256, dtype=np.int32), kw)
    PU.compare(g["tb"].reshape(-1), info, o, label="max-steps-1")
