"""The streaming-read probe that the tracer's gathers are compared with."""
import pytest

from tests import parity_util as PU

pytestmark = pytest.mark.gpu


def test_read_bandwidths_are_ordered_and_below_the_hbm_peak():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun as R
    print("case read probe", flush=True)
    bw = R.read_bandwidths(0)
    print("read bandwidths GB/s", bw, flush=True)
    # HBM3E peak 8 TB/s; the die-local L2 and the Infinity Cache serve more
    assert 1000.0 < bw["hbm_GBps"] < 8000.0
    assert bw["l2_GBps"] > bw["hbm_GBps"]
    assert bw["infinity_cache_GBps"] > bw["hbm_GBps"]


def test_path_keys_and_gather_replay():
    """Cell keys of recorded paths equal the spherical cell of each recorded
    point computed here in FP64; the replay of the walks runs and counts them."""
    if not PU.gpu_available():
        pytest.skip("no GPU")
    import numpy as np
    import ctypes as C
    import torch
    from paper_2606_02413_amd import corona, rtsun as R
    cor = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=11, n_ar=4, n_feat=256)
    m = R.Model.from_corona(cor)
    im = R.image_desc(16, 2.0)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    print("case path keys", flush=True)
    n_rays, cap = 2 * 16 * 16, 4000
    rec = R.trace_maps([m], [60e6, 300e6], im, prm, info=False, stats=False,
                       path_rays=np.arange(n_rays, dtype=np.int32), path_capacity=cap)
    keys = torch.empty((cap, n_rays), dtype=torch.int32, device="cuda")
    R._check(R.lib().rt_probe_path_keys(m.handle, C.c_void_p(rec["path"].data_ptr()),
                                        C.c_void_p(rec["path_len"].data_ptr()), n_rays, cap,
                                        C.c_void_p(keys.data_ptr()), None))
    torch.cuda.synchronize()
    path = rec["path"].cpu().numpy().astype(np.float64)
    plen = rec["path_len"].cpu().numpy()
    k = keys.cpu().numpy()
    n0, n1, n2 = cor.shape
    dl = np.log(cor.r_max / cor.r_in) / (n0 - 1)
    live = np.arange(cap)[None, :] < plen[:, None]                     # [walk][record]
    x, y, z = path[..., 0], path[..., 1], path[..., 2]
    rho = np.hypot(x, y)
    b0 = (0.5 * np.log(x * x + y * y + z * z) - np.log(cor.r_in)) / dl
    b1 = np.arctan2(rho, z) * n1 / np.pi - 0.5
    b2 = np.mod(np.arctan2(y, x), 2 * np.pi) * n2 / (2 * np.pi)
    a = np.clip(np.floor(b0), 0, n0 - 2).astype(np.int64)
    b = np.clip(np.floor(b1), 0, n1 - 2).astype(np.int64)
    c = np.floor(b2).astype(np.int64)
    c[(c < 0) | (c >= n2)] = 0
    want = np.where(live, (a * n1 + b) * (n2 + 1) + c, -1)
    got = k.T
    assert np.array_equal(got[~live], want[~live])
    agree = np.mean(got[live] == want[live])
    print("key agreement", agree, "records", int(live.sum()), flush=True)
    assert agree > 0.9999
    print("case gather replay", flush=True)
    ms = C.c_double(0.0)
    R._check(R.lib().rt_probe_gather_replay(m.handle, C.c_void_p(keys.data_ptr()), n_rays, cap, C.byref(ms), None))
    assert ms.value > 0.0
    res = R.gather_replay(m, [60e6, 300e6], im, prm)
    info = R.decode_info(R.trace_maps([m], [60e6, 300e6], im, prm, info=True, stats=False)["info"])
    n_steps = info["n_steps"].reshape(-1).astype(np.int64)
    assert res["capacity"] == int(n_steps.max())
    assert res["ray_steps"] == int(n_steps.sum()) and res["ray_steps_per_s"] > 0
    m.close()
