"""Python binding of the HIP library's C ABI (argument marshalling only).

Every step of the ray tracing runs in the HIP kernels of ``librtsun.so``; this
module only fills the ABI structs, passes torch device pointers and the current
HIP stream, and raises on a non-OK status.  There is no CPU fallback: if the
library is missing the import of ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtsun.so")
ABI_VERSION = 1

RT_GRID_SPHERICAL_LOGR, RT_GRID_CARTESIAN = 0, 1
RT_USE_MAGNIFICATION = 1 << 0
RT_USE_REFRACTION = 1 << 1
RT_PREC_ALL_FP32 = 1 << 2
RT_SCHED_PLAIN = 1 << 3
RT_DETERMINISTIC_GRAD = 1 << 4
RT_CARRIED_TUBE = 1 << 5
RT_PREC_FP32_STEP = 1 << 6
RT_TEST_NO_ABSORPTION = 1 << 30

EXIT_OUTER, HIT_INNER, MISS, MAX_STEPS, NONFINITE = 1, 2, 3, 4, 5
FLAG_MARGINAL = 2
PATH_FIELDS = ("x", "y", "z", "s", "ln_m", "dlns_ds", "tau", "ne", "te")

STATUS = {0: "RT_OK", 1: "RT_E_INVALID_ARG", 2: "RT_E_NONFINITE_INPUT", 3: "RT_E_OUT_OF_MEMORY",
          4: "RT_E_DEVICE", 5: "RT_E_UNSUPPORTED", 6: "RT_E_CAPACITY", 7: "RT_E_INTERNAL"}


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("kind", C.c_uint32), ("n0", C.c_int32), ("n1", C.c_int32),
                ("n2", C.c_int32), ("_reserved", C.c_int32), ("r_in", C.c_double), ("r_max", C.c_double),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class ImageDesc(C.Structure):
    _fields_ = [("obs_dir", C.c_double * 3), ("up", C.c_double * 3), ("nu", C.c_int32), ("nv", C.c_int32),
                ("half_u", C.c_double), ("half_v", C.c_double)]


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("flags", C.c_uint32), ("ds_max", C.c_double),
                ("n_floor", C.c_double), ("max_steps", C.c_int32), ("checkpoint_every", C.c_int32),
                ("perturb_ratio", C.c_double), ("tb_inner_K", C.c_double), ("tb_sky_K", C.c_double)]


INFO_DTYPE = np.dtype([("n_steps", "<i4"), ("code", "i1"), ("flags", "i1"), ("_pad", "i1", (2,)),
                       ("exit_pos", "<f4", (3,)), ("tau", "<f4"), ("ln_s_end", "<f4"), ("r_min", "<f4")])
class Tuning(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("refill_min_idle", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("xcd_bands", C.c_int32)]

    def as_dict(self):
        return {"refill_min_idle": int(self.refill_min_idle), "blocks_per_cu": int(self.blocks_per_cu),
                "xcd_bands": int(self.xcd_bands)}


STATS_DTYPE = np.dtype([("ray_steps", "<u8"), ("max_steps", "<u4"), ("code_count", "<u4", (6,)), ("_pad", "<u4")])
assert INFO_DTYPE.itemsize == 32 and STATS_DTYPE.itemsize == 40

_lib = None


def lib():
    """Load librtsun.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.rt_model_load.argtypes = [C.POINTER(GridDesc), vp, vp, C.c_int32, vp, C.POINTER(vp)]
        L.rt_model_load.restype = C.c_int
        L.rt_model_update.argtypes = [vp, vp, vp, C.c_int32, vp]
        L.rt_model_update.restype = C.c_int
        L.rt_model_free.argtypes = [vp]
        L.rt_model_free.restype = None
        L.rt_trace_maps.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(ImageDesc), C.POINTER(Params), vp, vp, vp, C.POINTER(C.c_int32),
                                    C.c_int32, C.c_int32, vp, vp, vp]
        L.rt_trace_maps.restype = C.c_int
        L.rt_trace_maps_static.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                           C.POINTER(ImageDesc), C.POINTER(Params), vp, vp, vp, vp]
        L.rt_trace_maps_static.restype = C.c_int
        L.rt_trace_adjoint.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(ImageDesc),
                                       C.POINTER(Params), vp, vp, vp, vp, vp, vp]
        L.rt_trace_adjoint.restype = C.c_int
        L.rt_status_string.argtypes = [C.c_int]
        L.rt_status_string.restype = C.c_char_p
        L.rt_last_error_message.argtypes = []
        L.rt_last_error_message.restype = C.c_char_p
        L.rt_abi_version.argtypes = []
        L.rt_abi_version.restype = C.c_uint32
        L.rt_params_default.argtypes = [C.POINTER(Params)]
        L.rt_params_default.restype = None
        L.rt_tuning_default.argtypes = [C.POINTER(Tuning)]
        L.rt_tuning_default.restype = None
        L.rt_set_tuning.argtypes = [C.c_int, C.POINTER(Tuning)]
        L.rt_set_tuning.restype = C.c_int
        L.rt_get_tuning.argtypes = [C.c_int, C.POINTER(Tuning)]
        L.rt_get_tuning.restype = C.c_int
        L.rt_autotune.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(ImageDesc),
                                  C.POINTER(Params), C.c_int32, C.POINTER(Tuning), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), vp]
        L.rt_autotune.restype = C.c_int
        L.rt_beam_fwhm.argtypes = [C.POINTER(C.c_double), C.c_int32, C.c_double, C.POINTER(C.c_double)]
        L.rt_beam_fwhm.restype = C.c_int
        L.rt_beam_convolve.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                       C.POINTER(C.c_double), vp]
        L.rt_beam_convolve.restype = C.c_int
        L.rt_disc_mean.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, vp, vp]
        L.rt_disc_mean.restype = C.c_int
        L.rt_probe_read_bandwidth.argtypes = [C.c_int32, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                              C.POINTER(C.c_double), vp]
        L.rt_probe_read_bandwidth.restype = C.c_int
        L.rt_probe_path_keys.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp, vp]
        L.rt_probe_path_keys.restype = C.c_int
        L.rt_probe_gather_replay.argtypes = [vp, vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
        L.rt_probe_gather_replay.restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise RtError(status, lib().rt_last_error_message().decode())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def grid_desc(kind, shape, r_in, r_max, origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0)):
    d = GridDesc()
    d.abi_version = ABI_VERSION
    d.kind = kind
    d.n0, d.n1, d.n2 = (int(x) for x in shape)
    d._reserved = 0
    d.r_in, d.r_max = float(r_in), float(r_max)
    d.origin = (C.c_double * 3)(*origin)
    d.spacing = (C.c_double * 3)(*spacing)
    return d


def image_desc(n, half_width, obs_dir=(1.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), nv=None, half_v=None):
    im = ImageDesc()
    im.obs_dir = (C.c_double * 3)(*obs_dir)
    im.up = (C.c_double * 3)(*up)
    im.nu = int(n)
    im.nv = int(n if nv is None else nv)
    im.half_u = float(half_width)
    im.half_v = float(half_width if half_v is None else half_v)
    return im


def params(*, ds_max=0.005, n_floor=1.0, max_steps=200000, eta=1e-2, tb_inner=1.0e4, tb_sky=0.0,
           refraction=True, magnification=True, all_fp32=False, plain=False, no_absorption=False,
           checkpoint_every=64, carried_tube=False, fp32_step=False):
    p = Params()
    lib().rt_params_default(C.byref(p))
    f = 0
    f |= RT_USE_REFRACTION if refraction else 0
    f |= RT_USE_MAGNIFICATION if magnification else 0
    f |= RT_PREC_ALL_FP32 if all_fp32 else 0
    f |= RT_PREC_FP32_STEP if fp32_step else 0
    f |= RT_SCHED_PLAIN if plain else 0
    f |= RT_TEST_NO_ABSORPTION if no_absorption else 0
    f |= RT_CARRIED_TUBE if carried_tube else 0
    p.flags = f
    p.ds_max, p.n_floor, p.max_steps = float(ds_max), float(n_floor), int(max_steps)
    p.perturb_ratio, p.tb_inner_K, p.tb_sky_K = float(eta), float(tb_inner), float(tb_sky)
    p.checkpoint_every = int(checkpoint_every)
    return p


class Model:
    """A model loaded on a device (owns the library's rt_model)."""

    def __init__(self, desc, ne, te, device=0, stream=None):
        ne = np.ascontiguousarray(ne, dtype=np.float32)
        te = np.ascontiguousarray(te, dtype=np.float32)
        self.desc = desc
        self.shape = (desc.n0, desc.n1, desc.n2)
        if ne.size != desc.n0 * desc.n1 * desc.n2 or te.size != ne.size:
            raise ValueError("array sizes do not match the descriptor")
        h = C.c_void_p()
        s = _stream_ptr(stream) if stream is not False else C.c_void_p(0)
        _check(lib().rt_model_load(C.byref(desc), ne.ctypes.data_as(C.c_void_p), te.ctypes.data_as(C.c_void_p),
                                   int(device), s, C.byref(h)))
        self.handle = h
        self.device = device

    @classmethod
    def from_corona(cls, cor, device=0):
        d = grid_desc(RT_GRID_SPHERICAL_LOGR, cor.shape, cor.r_in, cor.r_max)
        return cls(d, cor.ne, cor.te, device)

    def update_device(self, ne_t, te_t, stream=None):
        """Replace values from torch device tensors (float32, C-order, same shape)."""
        assert ne_t.is_contiguous() and te_t.is_contiguous()
        _check(lib().rt_model_update(self.handle, C.c_void_p(ne_t.data_ptr()), C.c_void_p(te_t.data_ptr()), 1,
                                     _stream_ptr(stream)))

    def update_device_log(self, ln_ne_t, ln_te_t, stream=None):
        """Replace values from the natural logarithms (float32 device tensors,
        C-order, same shape); the library exponentiates them."""
        assert ln_ne_t.is_contiguous() and ln_te_t.is_contiguous()
        _check(lib().rt_model_update(self.handle, C.c_void_p(ln_ne_t.data_ptr()), C.c_void_p(ln_te_t.data_ptr()),
                                     2, _stream_ptr(stream)))

    def update_host(self, ne, te, stream=None):
        ne = np.ascontiguousarray(ne, dtype=np.float32)
        te = np.ascontiguousarray(te, dtype=np.float32)
        _check(lib().rt_model_update(self.handle, ne.ctypes.data_as(C.c_void_p), te.ctypes.data_as(C.c_void_p), 0,
                                     _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().rt_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _out(res, key, shape, dtype, dev):
    """res[key]: allocated when absent, else checked to be a contiguous tensor of
    exactly this shape, dtype and device (the library writes through its raw
    pointer)."""
    import torch
    t = res.get(key)
    if t is None:
        t = torch.empty(shape, dtype=dtype, device=dev)
        res[key] = t
    elif tuple(t.shape) != tuple(shape) or t.dtype != dtype or t.device != dev or not t.is_contiguous():
        raise ValueError(f"out[{key!r}] must be a contiguous {dtype} tensor of shape {tuple(shape)} on {dev}")
    return t


def _handles(models):
    if any(m.handle is None for m in models):
        raise ValueError("a model was closed")
    return (C.c_void_p * len(models))(*[m.handle.value for m in models])


def trace_maps(models, freqs, image, prm, *, info=True, stats=True, path_rays=None, path_capacity=0,
               stream=None, out=None):
    """Trace all (model, frequency) maps.  Returns a dict of torch tensors on the device:
    tb [M][F][nv][nu] float32, info [...][32] uint8 (decode with decode_info), stats [40] uint8,
    path [P][cap][9] float32 and path_len [P] int32 when path_rays is given."""
    import torch
    if isinstance(models, Model):
        models = [models]
    freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    M, F = len(models), freqs.shape[0]
    dev = torch.device("cuda", models[0].device)
    shape = (M, F, image.nv, image.nu)
    res = {} if out is None else out
    _out(res, "tb", shape, torch.float32, dev)
    if info:
        _out(res, "info", shape + (32,), torch.uint8, dev)
    if stats:
        _out(res, "stats", (40,), torch.uint8, dev)
    handles = _handles(models)
    n_path = 0
    pr = None
    if path_rays is not None and len(path_rays) > 0:
        pr = np.ascontiguousarray(np.sort(np.asarray(path_rays, dtype=np.int32)))
        n_path = pr.shape[0]
        res["path"] = torch.zeros((n_path, path_capacity, 9), dtype=torch.float32, device=dev)
        res["path_len"] = torch.zeros(n_path, dtype=torch.int32, device=dev)
    ptr = lambda k: C.c_void_p(res[k].data_ptr()) if k in res and res[k] is not None else C.c_void_p(0)
    _check(lib().rt_trace_maps(handles, M, freqs.ctypes.data_as(C.POINTER(C.c_double)), F, C.byref(image),
                               C.byref(prm), ptr("tb"), ptr("info") if info else C.c_void_p(0),
                               ptr("stats") if stats else C.c_void_p(0),
                               pr.ctypes.data_as(C.POINTER(C.c_int32)) if n_path else None, n_path,
                               int(path_capacity), ptr("path") if n_path else C.c_void_p(0),
                               ptr("path_len") if n_path else C.c_void_p(0), _stream_ptr(stream)))
    return res


def tuning(refill_min_idle=64, blocks_per_cu=0, xcd_bands=8):
    t = Tuning()
    lib().rt_tuning_default(C.byref(t))
    t.refill_min_idle, t.blocks_per_cu, t.xcd_bands = int(refill_min_idle), int(blocks_per_cu), int(xcd_bands)
    return t


def set_tuning(t, device=0):
    """Install a launch tuning of the persistent trace on `device` (a Tuning or a dict)."""
    if isinstance(t, dict):
        t = tuning(**t)
    _check(lib().rt_set_tuning(int(device), C.byref(t)))


def get_tuning(device=0):
    t = Tuning()
    _check(lib().rt_get_tuning(int(device), C.byref(t)))
    return t


def tuning_key(models, freqs, image, prm, max_freqs):
    """Cache key of a tuning: the device, grid, image, batch shape and stepping
    controls it was measured on (the frequencies by count and range)."""
    import torch
    if isinstance(models, Model):
        models = [models]
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    d = models[0].desc
    parts = [torch.cuda.get_device_name(models[0].device), f"kind{d.kind}", f"{d.n0}x{d.n1}x{d.n2}",
             f"r{d.r_in:g}-{d.r_max:g}", f"img{image.nu}x{image.nv}", f"hw{image.half_u:g}x{image.half_v:g}",
             f"models{len(models)}", f"freqs{freqs.size}:{freqs.min():.6g}-{freqs.max():.6g}",
             f"flags{prm.flags}", f"ds{prm.ds_max:g}", f"nf{prm.n_floor:g}", f"sample{int(max_freqs)}"]
    return "|".join(parts)


def autotune(models, freqs, image, prm, *, max_freqs=8, cache=None, stream=None):
    """Pick the launch tuning of the persistent trace for this workload and install it.

    Runs rt_autotune (every candidate on a sample of at most max_freqs
    frequencies, maps checked bitwise against the defaults) unless `cache` (a
    JSON file path) already holds a tuning for the same key; stores new results
    there.  Returns a dict: tuning, key, best_ms, default_ms, cached."""
    import json
    if isinstance(models, Model):
        models = [models]
    key = tuning_key(models, freqs, image, prm, max_freqs)
    table = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table:
        set_tuning(table[key]["tuning"], models[0].device)
        return dict(table[key], key=key, cached=True)
    freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    handles = (C.c_void_p * len(models))(*[m.handle.value for m in models])
    best = Tuning()
    best_ms, default_ms = C.c_double(0.0), C.c_double(0.0)
    _check(lib().rt_autotune(handles, len(models), freqs.ctypes.data_as(C.POINTER(C.c_double)), freqs.shape[0],
                             C.byref(image), C.byref(prm), int(max_freqs), C.byref(best), C.byref(best_ms),
                             C.byref(default_ms), _stream_ptr(stream)))
    rec = {"tuning": best.as_dict(), "best_ms": best_ms.value, "default_ms": default_ms.value}
    if cache is not None:
        table[key] = rec
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(rec, key=key, cached=False)


def beam_fwhm(freqs, baseline_m):
    """Beam FWHM in R_sun of an interferometer with maximum baseline `baseline_m`
    (metres): lambda / B radians, over the angle 1 R_sun subtends at 1 au."""
    f = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    out = np.empty_like(f)
    _check(lib().rt_beam_fwhm(f.ctypes.data_as(C.POINTER(C.c_double)), f.shape[0], float(baseline_m),
                              out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def _check_maps(maps, image):
    import torch
    if maps.dtype != torch.float32 or not maps.is_cuda or maps.dim() < 2 or \
            tuple(maps.shape[-2:]) != (image.nv, image.nu):
        raise ValueError(f"maps must be a float32 device tensor [..., {image.nv}, {image.nu}]")


def beam_convolve(maps, image, fwhm, *, stream=None, out=None):
    """Maps [..., nv, nu] (float32 device tensor) convolved with Gaussian beams of
    the given FWHM (R_sun, one per map in the flattened leading dimensions)."""
    import torch
    _check_maps(maps, image)
    x = maps.contiguous()
    n_maps = x.numel() // (image.nu * image.nv)
    fw = np.ascontiguousarray(np.broadcast_to(np.asarray(fwhm, dtype=np.float64), (n_maps,)))
    y = torch.empty_like(x) if out is None else out
    if y.shape != x.shape or y.dtype != x.dtype or y.device != x.device or not y.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the maps' shape, dtype and device")
    _check(lib().rt_beam_convolve(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), n_maps, image.nu, image.nv,
                                  image.half_u, image.half_v, fw.ctypes.data_as(C.POINTER(C.c_double)),
                                  _stream_ptr(stream)))
    return y


def disc_mean(maps, image, radius=0.5, *, stream=None):
    """Mean T_b within `radius` R_sun of the image centre of each map [..., nv, nu]
    (float64 device tensor of the leading shape)."""
    import torch
    _check_maps(maps, image)
    x = maps.contiguous()
    lead = x.shape[:-2]
    n_maps = x.numel() // (image.nu * image.nv)
    y = torch.empty(n_maps, dtype=torch.float64, device=x.device)
    _check(lib().rt_disc_mean(C.c_void_p(x.data_ptr()), n_maps, image.nu, image.nv, image.half_u, image.half_v,
                              float(radius), C.c_void_p(y.data_ptr()), _stream_ptr(stream)))
    return y.reshape(lead)


def probe_read_bandwidth(device, nbytes, span_bytes, blocks, reps, *, stream=None):
    """GB/s of the library's streaming-read probe (rt_probe_read_bandwidth)."""
    out = C.c_double(0.0)
    _check(lib().rt_probe_read_bandwidth(int(device), int(nbytes), int(span_bytes), int(blocks), int(reps),
                                         C.byref(out), _stream_ptr(stream)))
    return out.value


def read_bandwidths(device=0, *, stream=None):
    """Measured streaming-read bandwidths (GB/s) of one die's L2 (2 MiB read
    whole by every block), the Infinity Cache (128 MiB partitioned) and HBM
    (4 GiB partitioned), 2048 blocks of 256 threads."""
    blocks = 2048
    l2 = probe_read_bandwidth(device, 2 << 20, 2 << 20, blocks, 16, stream=stream)
    mall = probe_read_bandwidth(device, 128 << 20, (128 << 20) // blocks, blocks, 64, stream=stream)
    hbm = probe_read_bandwidth(device, 4 << 30, (4 << 30) // blocks, blocks, 4, stream=stream)
    return {"l2_GBps": l2, "infinity_cache_GBps": mall, "hbm_GBps": hbm}


def gather_replay(model, freqs, image, prm, *, max_bytes=40 << 30, stream=None):
    """Gather-only replay of one trace_maps call's walks (rt_probe_path_keys,
    rt_probe_gather_replay): every ray of the call is recorded (capacity = the
    longest ray, capped so the records fit in max_bytes), its points turned into
    cell keys, and the replay of all walks timed.  Returns a dict with the
    replayed ray-steps, the replay time and their ratio."""
    import torch
    first = trace_maps([model], freqs, image, prm, info=True, stats=False, stream=stream)
    n_rays = first["tb"].numel()
    n_steps = decode_info(first["info"])["n_steps"].reshape(-1)
    cap = int(max(1, min(int(n_steps.max()), max_bytes // (n_rays * 9 * 4))))
    rec = trace_maps([model], freqs, image, prm, info=False, stats=False, stream=stream,
                     path_rays=np.arange(n_rays, dtype=np.int32), path_capacity=cap)
    keys = torch.empty((cap, n_rays), dtype=torch.int32, device=rec["tb"].device)
    _check(lib().rt_probe_path_keys(model.handle, C.c_void_p(rec["path"].data_ptr()),
                                    C.c_void_p(rec["path_len"].data_ptr()), n_rays, cap,
                                    C.c_void_p(keys.data_ptr()), _stream_ptr(stream)))
    steps = int(rec["path_len"].sum().item())
    del rec
    ms = C.c_double(0.0)
    _check(lib().rt_probe_gather_replay(model.handle, C.c_void_p(keys.data_ptr()), n_rays, cap, C.byref(ms),
                                        _stream_ptr(stream)))
    return {"walks": n_rays, "capacity": cap, "ray_steps": steps, "ms": ms.value,
            "ray_steps_per_s": steps / (ms.value * 1e-3)}


def trace_maps_static(models, freqs, image, prm, *, info=True, stats=True, stream=None, out=None):
    """rt_trace_maps_static: trace_maps without any device allocation by the
    library (per-call tables in its fixed device array; no path outputs).  The
    output tensors are allocated here unless passed in `out`."""
    import torch
    if isinstance(models, Model):
        models = [models]
    freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    M, F = len(models), freqs.shape[0]
    dev = torch.device("cuda", models[0].device)
    shape = (M, F, image.nv, image.nu)
    res = {} if out is None else out
    _out(res, "tb", shape, torch.float32, dev)
    if info:
        _out(res, "info", shape + (32,), torch.uint8, dev)
    if stats:
        _out(res, "stats", (40,), torch.uint8, dev)
    handles = _handles(models)
    ptr = lambda k: C.c_void_p(res[k].data_ptr()) if k in res and res[k] is not None else C.c_void_p(0)
    _check(lib().rt_trace_maps_static(handles, M, freqs.ctypes.data_as(C.POINTER(C.c_double)), F, C.byref(image),
                                      C.byref(prm), ptr("tb"), ptr("info") if info else C.c_void_p(0),
                                      ptr("stats") if stats else C.c_void_p(0), _stream_ptr(stream)))
    return res


class CapturedTrace:
    """A captured rt_trace_maps call: `replay()` re-runs the whole call (counter
    and statistics fills, the launch table and the trace kernels) into the
    tensors of `out`.  The graph was captured on `stream`, a stream of its own,
    whose library tables it uses; the object keeps that stream and the models
    alive.  The graph reads the models' device arrays: replaying after a model
    was closed raises, and rt_model_update between replays changes what the
    next replay traces."""

    def __init__(self, graph, out, stream, models):
        self.graph = graph
        self.out = out
        self.stream = stream
        self.models = list(models)

    def replay(self):
        if any(m.handle is None for m in self.models):
            raise RuntimeError("a model of this captured trace was closed")
        self.graph.replay()


def capture_trace_maps(models, freqs, image, prm, *, info=False, stats=True):
    """Capture one rt_trace_maps call (no path output) in a HIP graph.

    Returns (captured, out) with `captured.replay()` and the output tensors.  A
    warm-up call on the capture stream first sizes that stream's library tables,
    so the captured call allocates nothing and only launches kernels (every
    clear is a fill kernel, no memset node)."""
    import torch
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        out = trace_maps(models, freqs, image, prm, info=info, stats=stats)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        trace_maps(models, freqs, image, prm, info=info, stats=stats, out=out)
    torch.cuda.current_stream().wait_stream(stream)
    return CapturedTrace(graph, out, stream, models), out


def trace_adjoint(model, freqs, image, prm, weights, *, tb=True, stream=None, out=None):
    """Reverse mode of the forward maps of one model: loss = sum w T_b and its
    gradient w.r.t. ln n_e and ln T of every vertex.  `weights` is a float32
    device tensor [F][nv][nu].  Returns a dict of device tensors: loss (float64
    [1]), grad_ln_ne and grad_ln_te (float32, grid shape), tb [F][nv][nu] when
    `tb` is true."""
    import torch
    freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    F = freqs.shape[0]
    dev = torch.device("cuda", model.device)
    if tuple(weights.shape) != (F, image.nv, image.nu) or weights.dtype != torch.float32:
        raise ValueError("weights must be float32 [n_freq][nv][nu]")
    if not weights.is_contiguous() or weights.device != dev:
        raise ValueError(f"weights must be contiguous and on {dev}")
    if model.handle is None:
        raise ValueError("the model was closed")
    res = {} if out is None else out
    _out(res, "loss", (1,), torch.float64, dev)
    _out(res, "grad_ln_ne", tuple(model.shape), torch.float32, dev)
    _out(res, "grad_ln_te", tuple(model.shape), torch.float32, dev)
    if tb:
        _out(res, "tb", (F, image.nv, image.nu), torch.float32, dev)
    ptr = lambda k: C.c_void_p(res[k].data_ptr())
    _check(lib().rt_trace_adjoint(model.handle, freqs.ctypes.data_as(C.POINTER(C.c_double)), F, C.byref(image),
                                  C.byref(prm), C.c_void_p(weights.data_ptr()), ptr("loss"), ptr("grad_ln_ne"),
                                  ptr("grad_ln_te"), ptr("tb") if tb else C.c_void_p(0), _stream_ptr(stream)))
    return res


def _make_function():
    import torch

    class RTSunFunction(torch.autograd.Function):
        """T_b maps of one model as a differentiable function of (ln n_e, ln T).

        forward: the model's values are replaced from (ln n_e, ln T)
        (rt_model_update, which exponentiates on the device), then rt_trace_maps;
        backward: rt_trace_adjoint with the incoming gradient of the maps as the
        loss weights."""

        @staticmethod
        def forward(ctx, ln_ne, ln_te, model, freqs, image, prm):
            ln_ne_c = ln_ne.detach().to(torch.float32).contiguous()
            ln_te_c = ln_te.detach().to(torch.float32).contiguous()
            model.update_device_log(ln_ne_c, ln_te_c)
            out = trace_maps([model], freqs, image, prm, info=False, stats=False)
            ctx.save_for_backward(ln_ne_c, ln_te_c)
            ctx.model, ctx.freqs, ctx.image, ctx.prm = model, freqs, image, prm
            return out["tb"][0]

        @staticmethod
        def backward(ctx, grad_tb):
            ln_ne_c, ln_te_c = ctx.saved_tensors
            ctx.model.update_device_log(ln_ne_c, ln_te_c)  # the model may have been changed since the forward
            w = grad_tb.detach().to(torch.float32).contiguous()
            res = trace_adjoint(ctx.model, ctx.freqs, ctx.image, ctx.prm, w, tb=False)
            return res["grad_ln_ne"], res["grad_ln_te"], None, None, None, None

    return RTSunFunction


_function = None


def rtsun_function():
    """The torch.autograd.Function over the library (created on first use)."""
    global _function
    if _function is None:
        _function = _make_function()
    return _function


def decode_info(info_t):
    """Device uint8 [..., 32] tensor -> numpy structured array of INFO_DTYPE."""
    a = info_t.detach().cpu().numpy()
    return a.reshape(-1, 32).copy().view(INFO_DTYPE).reshape(a.shape[:-1])


def decode_stats(stats_t):
    return stats_t.detach().cpu().numpy().copy().view(STATS_DTYPE)[0]
