"""The binding's checks of caller-provided tensors: the library writes through
raw pointers, so an output tensor of the wrong shape, dtype or device, or a
closed model, is refused before any call into it."""
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


def test_output_tensors_are_checked(R):
    import torch
    m = R.Model.from_corona(corona.spherically_symmetric(nr=16, nt=8, nph=16))
    im = R.image_desc(16, 2.5)
    prm = R.params()
    print("case binding output checks", flush=True)
    try:
        good = R.trace_maps([m], [150e6], im, prm, info=True, stats=True)
        torch.cuda.synchronize()
        for bad in ({"tb": torch.empty((1, 1, 16, 15), device="cuda")},
                    {"tb": torch.empty((1, 1, 16, 16), dtype=torch.float64, device="cuda")},
                    {"tb": torch.empty((1, 1, 16, 16))},
                    {"tb": torch.empty((1, 1, 16, 32), device="cuda")[..., ::2]},
                    {"stats": torch.empty(39, dtype=torch.uint8, device="cuda")}):
            with pytest.raises(ValueError):
                R.trace_maps([m], [150e6], im, prm, info=False, stats=True, out=bad)
            with pytest.raises(ValueError):
                R.trace_maps_static([m], [150e6], im, prm, info=False, stats=True, out=dict(bad))
        again = R.trace_maps([m], [150e6], im, prm, info=True, stats=True, out=dict(good))
        torch.cuda.synchronize()
        assert torch.equal(again["tb"], good["tb"])
        w = torch.ones((1, 16, 16), dtype=torch.float32, device="cuda")
        with pytest.raises(ValueError):
            R.trace_adjoint(m, [150e6], im, prm, w, out={"grad_ln_ne": torch.empty((16, 8, 15), device="cuda")})
        with pytest.raises(ValueError):
            R.beam_convolve(good["tb"], R.image_desc(8, 2.5), [0.1])
        with pytest.raises(ValueError):
            R.beam_convolve(good["tb"], im, [0.1], out=torch.empty((1, 1, 16, 16), dtype=torch.float64,
                                                                    device="cuda"))
    finally:
        m.close()
    with pytest.raises(ValueError, match="closed"):
        R.trace_maps([m], [150e6], im, prm)
    with pytest.raises(ValueError, match="closed"):
        R.trace_adjoint(m, [150e6], im, prm, torch.ones((1, 16, 16), dtype=torch.float32, device="cuda"))
