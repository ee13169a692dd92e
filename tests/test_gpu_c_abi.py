"""A trace through the C ABI from a C++ host program (tests/c/trace_check.cpp,
built by __graft_entry__.build(); no Python between the caller and the
library): the same model, image and frequencies give bitwise the maps and step
counts the Python binding gets, and both match the oracle."""
import os
import subprocess

import numpy as np
import pytest

from paper_2606_02413_amd import corona
from tests import parity_util as PU

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "trace_check")


@pytest.fixture(scope="module")
def R():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun
    return rtsun


def test_c_program_matches_binding_and_oracle(R, orc, tmp_path):
    import torch
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    cor = corona.structured(nr=32, nt=16, nph=32, r_in=1.0, r_max=5.0, seed=3, n_feat=128)
    freqs = [60e6, 200e6]
    npix, half = 12, 2.0
    ne_f, te_f = tmp_path / "ne.f32", tmp_path / "te.f32"
    np.ascontiguousarray(cor.ne, np.float32).tofile(ne_f)
    np.ascontiguousarray(cor.te, np.float32).tofile(te_f)
    tb_f, st_f = tmp_path / "tb.f32", tmp_path / "steps.i32"
    print("case C program trace", flush=True)
    r = subprocess.run([EXE, str(cor.ne.shape[0]), str(cor.ne.shape[1]), str(cor.ne.shape[2]), "1.0", "5.0",
                        str(ne_f), str(te_f), str(npix), str(half), str(tb_f), str(st_f)] +
                       [repr(f) for f in freqs], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    tb_c = np.fromfile(tb_f, np.float32).reshape(len(freqs), npix, npix)
    st_c = np.fromfile(st_f, np.int32).reshape(len(freqs), npix, npix)
    m = R.Model.from_corona(cor)
    try:
        out = R.trace_maps([m], freqs, R.image_desc(npix, half), R.params(), info=True, stats=False)
        torch.cuda.synchronize()
        tb_p = out["tb"][0].cpu().numpy()
        info = R.decode_info(out["info"])[0]
    finally:
        m.close()
    assert np.array_equal(tb_c, tb_p)
    assert np.array_equal(st_c, info["n_steps"])
    # the library's defaults (rt_params_default) are the oracle's stepping here
    kw = PU.step_kwargs(0.005, 1.0)
    pix = np.arange(npix * npix, dtype=np.int32)
    for k, f in enumerate(freqs):
        o = PU.oracle_trace(orc, cor, f, npix, half, pix, kw)
        PU.compare(tb_c[k].reshape(-1), info[k].reshape(-1), o, label=f"c-abi-{f/1e6:.0f}MHz")
