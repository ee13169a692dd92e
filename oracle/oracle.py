"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  It loads ``librt_oracle.so`` built from ``rt_oracle.cpp`` in this
directory and never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_oracle.so")
SRC_PATH = os.path.join(_HERE, "rt_oracle.cpp")

# Per-ray termination codes and flags (same numbering as the GPU library's ABI).
EXIT_OUTER, HIT_INNER, MISS, MAX_STEPS, NONFINITE = 1, 2, 3, 4, 5
GRAZING, MARGINAL, POLAR = 1, 2, 4

GRID_SPHERICAL_LOGR, GRID_CARTESIAN = 0, 1
ANALYTIC_BA, ANALYTIC_UNIFORM, ANALYTIC_SLAB, ANALYTIC_LENS = 10, 11, 12, 13

PATH_FIELDS = ("x", "y", "z", "s", "ln_m", "dlns_ds", "tau", "ne", "te", "dtau", "gamma", "dt")


NATIVE_LIB_PATH = os.path.join(_HERE, "librt_oracle_native.so")


def build(force=True, native=False):
    """Compile the oracle with g++, no fast-math.  The default build uses portable
    x86-64 flags (the library may run on another host than the one that built
    it); native=True builds a copy tuned for the building host (-march=native),
    which the benchmark's CPU baseline compiles and times on its own host."""
    path = NATIVE_LIB_PATH if native else LIB_PATH
    if not force and os.path.exists(path):
        return path
    arch = "-march=native" if native else "-march=x86-64-v2"
    cmd = ["g++", "-O3", "-std=c++17", arch, "-fno-fast-math", "-shared", "-fPIC", SRC_PATH, "-o", path + ".tmp",
           "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


def build_flags(native=False):
    return "g++ -O3 -std=c++17 " + ("-march=native" if native else "-march=x86-64-v2") + " -fno-fast-math"


class Medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n0", C.c_int32), ("n1", C.c_int32), ("n2", C.c_int32),
                ("r_in", C.c_double), ("r_max", C.c_double),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("ne", C.POINTER(C.c_float)), ("te", C.POINTER(C.c_float)),
                ("a0", C.c_double), ("a1", C.c_double), ("a2", C.c_double), ("t_const", C.c_double)]


class Params(C.Structure):
    _fields_ = [("stepper", C.c_int32), ("use_refraction", C.c_int32), ("use_magnification", C.c_int32),
                ("no_absorption", C.c_int32), ("ds_max", C.c_double), ("n_floor", C.c_double),
                ("max_steps", C.c_int32), ("twin_check", C.c_int32), ("eta", C.c_double),
                ("tb_inner", C.c_double), ("tb_sky", C.c_double),
                ("dp_rtol", C.c_double), ("dp_atol", C.c_double), ("carried_tube", C.c_int32),
                ("_pad", C.c_int32), ("twin_exit_tol", C.c_double)]


class Image(C.Structure):
    _fields_ = [("obs_dir", C.c_double * 3), ("up", C.c_double * 3), ("nu", C.c_int32), ("nv", C.c_int32),
                ("half_u", C.c_double), ("half_v", C.c_double)]


class Result(C.Structure):
    _fields_ = [("tb", C.c_double), ("tau", C.c_double), ("ln_s_end", C.c_double), ("r_min", C.c_double),
                ("exit_pos", C.c_double * 3), ("lam_last", C.c_double),
                ("bouguer_drift", C.c_double), ("ham_drift", C.c_double), ("ln_s_min", C.c_double),
                ("twin_dexit", C.c_double), ("n_steps", C.c_int32), ("code", C.c_int32), ("flags", C.c_int32), ("_pad", C.c_int32),
                ("event_hash", C.c_uint64)]


RESULT_DTYPE = np.dtype([("tb", "f8"), ("tau", "f8"), ("ln_s_end", "f8"), ("r_min", "f8"),
                         ("exit_pos", "f8", (3,)), ("lam_last", "f8"), ("bouguer_drift", "f8"),
                         ("ham_drift", "f8"), ("ln_s_min", "f8"), ("twin_dexit", "f8"), ("n_steps", "i4"), ("code", "i4"), ("flags", "i4"),
                         ("_pad", "i4"), ("event_hash", "u8")])
assert RESULT_DTYPE.itemsize == C.sizeof(Result)

_lib = None
_lib_path = LIB_PATH


def use_library(path):
    """Load the oracle from another build of rt_oracle.cpp (e.g. NATIVE_LIB_PATH)
    for every later call."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build(native=_lib_path == NATIVE_LIB_PATH)
        L = C.CDLL(_lib_path)
        dp = C.POINTER(C.c_double)
        L.orc_trace_launch.argtypes = [C.POINTER(Medium), C.POINTER(Params), C.c_double, C.c_int, dp, dp,
                                       C.c_void_p, dp, C.c_int, C.POINTER(C.c_int), C.c_int]
        L.orc_trace_pixels.argtypes = [C.POINTER(Medium), C.POINTER(Params), C.POINTER(Image), C.c_double,
                                       C.c_int, C.POINTER(C.c_int32), C.c_void_p, C.c_int]
        L.orc_trace_pixel_path.argtypes = [C.POINTER(Medium), C.POINTER(Params), C.POINTER(Image), C.c_double,
                                           C.c_int, C.c_void_p, dp, C.c_int, C.POINTER(C.c_int)]
        L.orc_eval_medium.argtypes = [C.POINTER(Medium), C.c_int, dp, dp]
        L.orc_kappa_n.argtypes = [C.c_int, dp, dp, C.c_double, dp]
        L.orc_dual_loss.argtypes = [C.POINTER(Medium), C.POINTER(Params), C.POINTER(Image), C.c_int, dp,
                                    C.POINTER(C.c_float), dp, dp, dp, dp, C.c_int]
        L.orc_grad_loss.argtypes = [C.POINTER(Medium), C.POINTER(Params), C.POINTER(Image), C.c_int, dp,
                                    C.POINTER(C.c_float), dp, dp, dp, C.c_int]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_threads():
    return max(1, min(os.cpu_count() or 1, 16))


class OracleMedium:
    """Keeps the arrays a Medium struct points at alive."""

    def __init__(self, kind, *, shape=(2, 2, 2), r_in=1.0, r_max=3.0, ne=None, te=None,
                 origin=(0, 0, 0), spacing=(1, 1, 1), a0=0.0, a1=0.0, a2=1.0, t_const=1e6):
        self._ne = None if ne is None else np.ascontiguousarray(ne, dtype=np.float32)
        self._te = None if te is None else np.ascontiguousarray(te, dtype=np.float32)
        m = Medium()
        m.kind = kind
        m.n0, m.n1, m.n2 = shape
        m.r_in, m.r_max = r_in, r_max
        m.origin = (C.c_double * 3)(*origin)
        m.spacing = (C.c_double * 3)(*spacing)
        fp = C.POINTER(C.c_float)
        m.ne = self._ne.ctypes.data_as(fp) if self._ne is not None else fp()
        m.te = self._te.ctypes.data_as(fp) if self._te is not None else fp()
        m.a0, m.a1, m.a2, m.t_const = a0, a1, a2, t_const
        self.struct = m
        self.r_max = r_max
        self.r_in = r_in

    @classmethod
    def from_corona(cls, cor):
        return cls(GRID_SPHERICAL_LOGR, shape=cor.shape, r_in=cor.r_in, r_max=cor.r_max, ne=cor.ne, te=cor.te)

    def eval(self, pos):
        pos = np.ascontiguousarray(np.atleast_2d(pos), dtype=np.float64)
        out = np.zeros((pos.shape[0], 5))
        lib().orc_eval_medium(C.byref(self.struct), pos.shape[0], _dptr(pos), _dptr(out))
        return out


# Twin check (ill-conditioned rays): a twin launched TWIN_OFFSET away in u whose
# exit moves by more than TWIN_EXIT_TOL marks the ray GRAZING.  The threshold is
# an exit amplification of 50: an FP32 evaluation of the model acts on a ray like
# a launch perturbation of about 2e-7 R_sun, and 50 x 2e-7 = 1e-5 R_sun is the
# exit-position bar of the GPU parity checks, so a ray below the threshold can be
# held to that bar.
TWIN_OFFSET = 1e-6
TWIN_EXIT_TOL = 50.0 * TWIN_OFFSET


def make_params(*, stepper=0, refraction=True, magnification=True, no_absorption=False, ds_max=0.005,
                n_floor=1.0, max_steps=200000, twin_check=False, eta=1e-2, tb_inner=1.0e4, tb_sky=0.0,
                rtol=1e-12, atol=1e-12, carried_tube=False, twin_exit_tol=TWIN_EXIT_TOL):
    p = Params()
    p.stepper = stepper
    p.use_refraction = int(refraction)
    p.use_magnification = int(magnification)
    p.no_absorption = int(no_absorption)
    p.ds_max, p.n_floor, p.max_steps = ds_max, n_floor, max_steps
    p.twin_check = int(twin_check)
    p.eta, p.tb_inner, p.tb_sky = eta, tb_inner, tb_sky
    p.dp_rtol, p.dp_atol = rtol, atol
    p.carried_tube = int(carried_tube)
    p.twin_exit_tol = float(twin_exit_tol)
    return p


def make_image(n, half_width, obs_dir=(1.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), nv=None, half_v=None):
    im = Image()
    im.obs_dir = (C.c_double * 3)(*obs_dir)
    im.up = (C.c_double * 3)(*up)
    im.nu = n
    im.nv = n if nv is None else nv
    im.half_u = half_width
    im.half_v = half_width if half_v is None else half_v
    return im


def trace_pixels(med, params, image, freq, pixels, n_threads=None):
    pix = np.ascontiguousarray(pixels, dtype=np.int32)
    out = np.zeros(pix.shape[0], dtype=RESULT_DTYPE)
    rc = lib().orc_trace_pixels(C.byref(med.struct), C.byref(params), C.byref(image), float(freq), pix.shape[0],
                                pix.ctypes.data_as(C.POINTER(C.c_int32)), out.ctypes.data,
                                n_threads or default_threads())
    assert rc == 0
    return out


def trace_image(med, params, image, freq, n_threads=None):
    return trace_pixels(med, params, image, freq, np.arange(image.nu * image.nv, dtype=np.int32), n_threads)


def trace_launch(med, params, freq, r0, direction, n_threads=None):
    r0 = np.ascontiguousarray(np.atleast_2d(r0), dtype=np.float64)
    d = np.ascontiguousarray(np.atleast_2d(direction), dtype=np.float64)
    out = np.zeros(r0.shape[0], dtype=RESULT_DTYPE)
    rc = lib().orc_trace_launch(C.byref(med.struct), C.byref(params), float(freq), r0.shape[0], _dptr(r0),
                                _dptr(d), out.ctypes.data, None, 0, None, n_threads or default_threads())
    assert rc == 0
    return out


def trace_launch_path(med, params, freq, r0, direction, cap=400000):
    r0 = np.ascontiguousarray(np.asarray(r0, dtype=np.float64).reshape(1, 3))
    d = np.ascontiguousarray(np.asarray(direction, dtype=np.float64).reshape(1, 3))
    out = np.zeros(1, dtype=RESULT_DTYPE)
    path = np.zeros((cap, len(PATH_FIELDS)))
    n = C.c_int(0)
    rc = lib().orc_trace_launch(C.byref(med.struct), C.byref(params), float(freq), 1, _dptr(r0), _dptr(d),
                                out.ctypes.data, _dptr(path), cap, C.byref(n), 1)
    assert rc == 0
    return out[0], path[:n.value]


def trace_pixel_path(med, params, image, freq, pixel, cap=400000):
    out = np.zeros(1, dtype=RESULT_DTYPE)
    path = np.zeros((cap, len(PATH_FIELDS)))
    n = C.c_int(0)
    rc = lib().orc_trace_pixel_path(C.byref(med.struct), C.byref(params), C.byref(image), float(freq), int(pixel),
                                    out.ctypes.data, _dptr(path), cap, C.byref(n))
    assert rc == 0
    return out[0], path[:n.value]


def kappa_n(ne, te, freq):
    ne = np.ascontiguousarray(np.atleast_1d(ne), dtype=np.float64)
    te = np.ascontiguousarray(np.atleast_1d(te), dtype=np.float64)
    out = np.zeros_like(ne)
    lib().orc_kappa_n(ne.shape[0], _dptr(ne), _dptr(te), float(freq), _dptr(out))
    return out


def dual_loss(med, params, image, freqs, weights, vn=None, vt=None, n_threads=None):
    """(loss, directional derivative) of sum w*T_b along (vn, vt) in (ln n_e, ln T)."""
    freqs = np.ascontiguousarray(freqs, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    loss = C.c_double(0)
    dl = C.c_double(0)
    vn_a = None if vn is None else np.ascontiguousarray(vn, dtype=np.float64)
    vt_a = None if vt is None else np.ascontiguousarray(vt, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    rc = lib().orc_dual_loss(C.byref(med.struct), C.byref(params), C.byref(image), freqs.shape[0], _dptr(freqs),
                             w.ctypes.data_as(C.POINTER(C.c_float)),
                             _dptr(vn_a) if vn_a is not None else dp(),
                             _dptr(vt_a) if vt_a is not None else dp(),
                             C.byref(loss), C.byref(dl), n_threads or default_threads())
    assert rc == 0
    return loss.value, dl.value


def grad_loss(med, params, image, freqs, weights, n_threads=None):
    """(loss, d loss / d ln n_e, d loss / d ln T) of loss = sum w*T_b by reverse-mode
    sweeps of per-ray tapes; weights are [n_freq][nv][nu] (zero weights skip the ray)
    and the gradients have the grid's shape."""
    freqs = np.ascontiguousarray(freqs, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    shape = (med.struct.n0, med.struct.n1, med.struct.n2)
    gne = np.zeros(shape, dtype=np.float64)
    gte = np.zeros(shape, dtype=np.float64)
    loss = C.c_double(0)
    rc = lib().orc_grad_loss(C.byref(med.struct), C.byref(params), C.byref(image), freqs.shape[0], _dptr(freqs),
                             w.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss), _dptr(gne), _dptr(gte),
                             n_threads or default_threads())
    assert rc == 0
    return loss.value, gne, gte
