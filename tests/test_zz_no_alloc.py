"""The allocation-free trace entry point against the allocating one.

rt_trace_maps_static keeps its per-call tables in a fixed device array instead
of library allocations; it launches the same kernels, so its maps, per-ray
records and statistics equal rt_trace_maps's bit for bit.  Two calls in a row,
the second with a smaller image and fewer frequencies and models, check that
the array's leftover contents do not leak into the next call; a call beyond the
array's size is refused.
"""
import ctypes as C

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


def _both(R, models, freqs, im, prm):
    import torch
    a = R.trace_maps(models, freqs, im, prm, info=True, stats=True)
    b = R.trace_maps_static(models, freqs, im, prm, info=True, stats=True)
    torch.cuda.synchronize()
    return a, b


def _same(a, b, label):
    import torch
    for k in ("tb", "info", "stats"):
        assert torch.equal(a[k], b[k]), (label, k)


def test_static_entry_point_equals_allocating_one(R):
    cor_a = corona.structured(nr=48, nt=24, nph=48, r_in=1.0, r_max=30.0, seed=21, n_ar=4, n_feat=128)
    cor_b = corona.structured(nr=48, nt=24, nph=48, r_in=1.0, r_max=30.0, seed=22, n_ar=4, n_feat=128)
    ma, mb = R.Model.from_corona(cor_a), R.Model.from_corona(cor_b)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    print("case static entry point: two models, 3 freq, 53x45", flush=True)
    a, b = _both(R, [ma, mb], corona.log_freqs(3), R.image_desc(53, 3.0, nv=45, half_v=2.5), prm)
    _same(a, b, "first call")
    assert R.decode_stats(b["stats"])["ray_steps"] > 0
    print("case static entry point: one model, 1 freq, 17x11 (after a larger call)", flush=True)
    a, b = _both(R, [mb], [150e6], R.image_desc(17, 2.0, nv=11, half_v=1.5), prm)
    _same(a, b, "second, smaller call")
    print("case static entry point: plain launches", flush=True)
    a, b = _both(R, [ma], [60e6, 300e6], R.image_desc(24, 2.0), R.params(ds_max=0.01, n_floor=0.1, plain=True))
    _same(a, b, "plain")
    ma.close()
    mb.close()


def test_static_entry_point_refuses_oversized_calls(R):
    import torch
    cor = corona.spherically_symmetric(nr=16, nt=8, nph=16)
    m = R.Model.from_corona(cor)
    im = R.image_desc(1200, 2.5)  # 1200^2 x (48 + 4) bytes > 64 MiB
    tb = torch.empty((1, 1, 1200, 1200), dtype=torch.float32, device="cuda")
    with pytest.raises(R.RtError) as e:
        R.trace_maps_static([m], [150e6], im, R.params(), info=False, stats=False, out={"tb": tb})
    assert e.value.status == 6
    m.close()
