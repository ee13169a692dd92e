"""Host-side checks of the C ABI library: it loads, exports every declared entry
point, and rejects bad arguments and values before any device work (so these
run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsun.h")


@pytest.fixture(scope="module")
def R():
    from paper_2606_02413_amd import rtsun
    if not os.path.exists(rtsun.LIB_PATH):
        from paper_2606_02413_amd import build
        build.build()
    return rtsun


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(R):
    L = R.lib()
    names = declared_functions()
    assert "rt_trace_maps" in names and "rt_model_load" in names and "rt_trace_adjoint" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in rtsun.h but not exported"


def test_abi_version_and_defaults(R):
    L = R.lib()
    assert L.rt_abi_version() == R.ABI_VERSION
    p = R.Params()
    L.rt_params_default(C.byref(p))
    assert p.abi_version == 1 and p.flags == (R.RT_USE_MAGNIFICATION | R.RT_USE_REFRACTION)
    assert p.ds_max == 0.005 and p.n_floor == 1.0 and p.checkpoint_every == 64 and p.perturb_ratio == 1e-2
    assert L.rt_status_string(3) == b"RT_E_OUT_OF_MEMORY"


def _load(R, desc, ne, te):
    h = C.c_void_p()
    st = R.lib().rt_model_load(C.byref(desc), ne.ctypes.data_as(C.c_void_p) if ne is not None else None,
                               te.ctypes.data_as(C.c_void_p) if te is not None else None, 0, None, C.byref(h))
    return st, R.lib().rt_last_error_message().decode()


def test_model_load_validation(R):
    good = R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (4, 3, 5), 1.0, 3.0)
    ne = np.full(60, 1e7, np.float32)
    te = np.full(60, 1e6, np.float32)
    bad_ver = R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (4, 3, 5), 1.0, 3.0)
    bad_ver.abi_version = 99
    assert _load(R, bad_ver, ne, te)[0] == 1
    assert _load(R, R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (1, 3, 5), 1.0, 3.0), ne, te)[0] == 1
    assert _load(R, R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (4, 3, 5), 3.0, 1.0), ne, te)[0] == 1
    assert _load(R, R.grid_desc(7, (4, 3, 5), 1.0, 3.0), ne, te)[0] == 1
    assert _load(R, R.grid_desc(R.RT_GRID_CARTESIAN, (4, 3, 5), 1.0, 3.0, spacing=(1, 0, 1)), ne, te)[0] == 1
    assert _load(R, good, None, te)[0] == 1
    nan = ne.copy()
    nan[17] = np.nan
    st, msg = _load(R, good, nan, te)
    assert st == 2 and "17" in msg
    neg = ne.copy()
    neg[3] = -1.0
    assert _load(R, good, neg, te)[0] == 2
    zt = te.copy()
    zt[59] = 0.0
    assert _load(R, good, ne, zt)[0] == 2



def test_grid_capacity_limits(R):
    """Cell keys are formed with 24-bit multiplies and kept in 32-bit ints: grids
    with n0*n1 >= 2^24, a packed row of 2^24 or more, or more than 2^31-1 packed
    vertices are refused before any value is read (the small arrays passed here
    are never touched)."""
    ne = np.full(8, 1e7, np.float32)
    te = np.full(8, 1e6, np.float32)
    for kind, shape in ((R.RT_GRID_SPHERICAL_LOGR, (4096, 4096, 3)),      # n0*n1 = 2^24
                        (R.RT_GRID_CARTESIAN, (2, 2, 1 << 24)),            # row of 2^24
                        (R.RT_GRID_SPHERICAL_LOGR, (2, 2, (1 << 24) - 1)),  # packed row n2 + 1 = 2^24
                        (R.RT_GRID_SPHERICAL_LOGR, (2048, 2048, 512)),      # 2048*2048*513 > 2^31-1
                        (R.RT_GRID_CARTESIAN, (2048, 2048, 512))):          # 2^31 > 2^31-1
        st, msg = _load(R, R.grid_desc(kind, shape, 1.0, 3.0), ne, te)
        assert st == 6, (shape, st, msg)

def test_device_byte_cap(R, monkeypatch):
    monkeypatch.setenv("RT_MAX_DEVICE_BYTES", "100")
    good = R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (4, 3, 5), 1.0, 3.0)
    st, msg = _load(R, good, np.full(60, 1e7, np.float32), np.full(60, 1e6, np.float32))
    assert st == 3 and "RT_MAX_DEVICE_BYTES" in msg


def test_trace_argument_validation(R):
    L = R.lib()
    im = R.image_desc(8, 2.0)
    p = R.params()
    f = (C.c_double * 1)(150e6)
    st = L.rt_trace_maps(None, 0, f, 1, C.byref(im), C.byref(p), None, None, None, None, 0, 0, None, None, None)
    assert st == 1
    st = L.rt_trace_adjoint(None, f, 1, C.byref(im), C.byref(p), None, None, None, None, None, None)
    assert st in (1, 5)


def test_tuning_defaults_and_validation(R):
    """Launch tuning: defaults, and values out of range rejected before any
    device work; the autotuner rejects bad arguments the same way."""
    L = R.lib()
    t = R.Tuning()
    L.rt_tuning_default(C.byref(t))
    assert t.as_dict() == {"refill_min_idle": 64, "blocks_per_cu": 0, "xcd_bands": 8} and t.abi_version == 1
    for kw in (dict(refill_min_idle=0), dict(refill_min_idle=65), dict(blocks_per_cu=-1), dict(blocks_per_cu=9),
               dict(xcd_bands=2), dict(xcd_bands=0)):
        bad = R.tuning(**kw)
        assert L.rt_set_tuning(0, C.byref(bad)) == 1, kw
    bad = R.tuning()
    bad.abi_version = 7
    assert L.rt_set_tuning(0, C.byref(bad)) == 1
    assert L.rt_set_tuning(0, None) == 1 and L.rt_get_tuning(0, None) == 1
    im = R.image_desc(8, 2.0)
    f = (C.c_double * 1)(150e6)
    p = R.params()
    assert L.rt_autotune(None, 1, f, 1, C.byref(im), C.byref(p), 4, None, None, None, None) == 1
    assert L.rt_autotune(None, 1, f, 1, C.byref(im), C.byref(p), 0, None, None, None, None) == 1
    plain = R.params(plain=True)
    h = (C.c_void_p * 1)(1)
    assert L.rt_autotune(h, 1, f, 1, C.byref(im), C.byref(plain), 4, None, None, None, None) == 1


def test_map_postprocessing_validation(R):
    L = R.lib()
    fw = (C.c_double * 2)(0.1, 0.1)
    buf = C.c_void_p(16)
    other = C.c_void_p(32)
    assert L.rt_beam_convolve(None, other, 2, 8, 8, 1.0, 1.0, fw, None) == 1
    assert L.rt_beam_convolve(buf, buf, 2, 8, 8, 1.0, 1.0, fw, None) == 1        # in place
    assert L.rt_beam_convolve(buf, other, 0, 8, 8, 1.0, 1.0, fw, None) == 1
    assert L.rt_beam_convolve(buf, other, 129, 8, 8, 1.0, 1.0, fw, None) == 1
    assert L.rt_beam_convolve(buf, other, 2, 8, 8, 0.0, 1.0, fw, None) == 1
    bad = (C.c_double * 2)(0.1, -1.0)
    assert L.rt_beam_convolve(buf, other, 2, 8, 8, 1.0, 1.0, bad, None) == 1
    assert L.rt_disc_mean(None, 1, 8, 8, 1.0, 1.0, 0.5, other, None) == 1
    assert L.rt_disc_mean(buf, 1, 8, 8, 1.0, 1.0, 0.0, other, None) == 1
    assert L.rt_disc_mean(buf, 1, 0, 8, 1.0, 1.0, 0.5, other, None) == 1
    assert abs(R.beam_fwhm([40e6], 15e3)[0] - 0.1074) < 1e-3   # 7.49 m / 15 km = 5.0e-4 rad
    # lambda / B in units of the 1 au angle of 1 R_sun, at two frequencies
    fw = R.beam_fwhm([100e6, 300e6], 5e3)
    assert abs(fw[0] / (299792458.0 / 100e6 / 5e3 / (6.957e8 / 1.495978707e11)) - 1) < 1e-15
    assert abs(fw[0] / fw[1] - 3.0) < 1e-14
    L = R.lib()
    out = (C.c_double * 1)()
    f = (C.c_double * 1)(100e6)
    assert L.rt_beam_fwhm(f, 1, 0.0, out) == 1
    assert L.rt_beam_fwhm(f, 0, 5e3, out) == 1
    assert L.rt_beam_fwhm((C.c_double * 1)(-1.0), 1, 5e3, out) == 1


def test_read_probe_validation(R):
    """The streaming-read probe rejects bad sizes before touching a device."""
    L = R.lib()
    out = C.c_double(0.0)
    assert L.rt_probe_read_bandwidth(0, 1 << 20, 1 << 20, 64, 1, None, None) == 1
    assert L.rt_probe_read_bandwidth(0, 0, 16, 64, 1, C.byref(out), None) == 1
    assert L.rt_probe_read_bandwidth(0, 1000, 16, 64, 1, C.byref(out), None) == 1          # not a multiple of 16
    assert L.rt_probe_read_bandwidth(0, 1 << 20, 2 << 20, 64, 1, C.byref(out), None) == 1  # span > bytes
    assert L.rt_probe_read_bandwidth(0, 1 << 20, 1 << 20, 0, 1, C.byref(out), None) == 1
    assert L.rt_probe_read_bandwidth(0, 1 << 20, 1 << 20, 64, 0, C.byref(out), None) == 1
    buf = C.c_void_p(16)
    assert L.rt_probe_path_keys(None, buf, buf, 4, 4, buf, None) == 1
    assert L.rt_probe_gather_replay(None, buf, 4, 4, C.byref(out), None) == 1


def test_binding_fails_loudly_without_library(R, monkeypatch):
    monkeypatch.setattr(R, "_lib", None)
    monkeypatch.setattr(R, "LIB_PATH", "/nonexistent/librtsun.so")
    with pytest.raises(RuntimeError, match="not built"):
        R.lib()


def test_oracle_and_gpu_library_share_no_code():
    """The oracle and the HIP library neither include nor import each other."""
    osrc = [os.path.join(ROOT, "oracle", f) for f in os.listdir(os.path.join(ROOT, "oracle"))
            if f.endswith((".cpp", ".h", ".py"))]
    for p in osrc:
        t = open(p).read()
        assert "paper_2606_02413_amd" not in t and "rtsun" not in t, p
    csrc = os.path.join(ROOT, "paper_2606_02413_amd", "csrc")
    for f in os.listdir(csrc):
        if f.endswith((".cpp", ".hpp", ".hip", ".h")):
            t = open(os.path.join(csrc, f)).read()
            assert "oracle" not in t.lower(), f
    for f in ("rtsun.py", "build.py", "corona.py"):
        t = open(os.path.join(ROOT, "paper_2606_02413_amd", f)).read()
        assert "import oracle" not in t and "from oracle" not in t, f
