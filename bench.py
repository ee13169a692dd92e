"""Throughput benchmark of the hot path on one MI355X.

One step = one pass of the whole forward path over the structured synthetic
corona: 256 x 128 x 256 spherical grid (r 1-30 R_sun), Baumbach-Allen density
times exp(0.3 g) with 8 Gaussian active regions, 512 x 512 image over
+/-3 R_sun, 8 frequencies log-spaced 40-800 MHz, adaptive step ds <= 0.01 R_sun
(n_floor 0.1).  Every step traces all 8 maps in one persistent batched launch
(refraction, step-wise magnification, free-free transfer).  The same maps are
also timed through the plain per-frequency launches, and the FP64 CPU oracle is
timed on a bounded pixel sample of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32/FP64 operations per ray-step of the method (counted on the
# method's arithmetic, not on compiled code; FMA = 2, each transcendental = 1):
#   4 central force evaluations x 128 + RK4 offsets/step rule/increments 74 +
#   2 perturbed retracings x 417 (3 force evaluations each with offsets and
#   differences) + basis 30 + area and ln M 18 + termination 7 + midpoint value
#   evaluation 72 + free-free 14 + transfer 15 = 1,576.
FLOPS_PER_RAY_STEP = 1576
# MI355X vector peak without packed FP32 (the build compiles it out):
# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s (FP32 and FP64 alike).
VALU_PEAK_TFLOPS = 78.6
# HBM bytes per launch of the persistent tracer on this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE passes scaled by a 1 GiB copy (read x2.000, write x1.000),
# valid only for the kernel sources they were taken on (hash below); reported as
# null as soon as those sources change.
KERNEL_SOURCES = ("rt_trace.hpp", "rt_kernels.hip", "rt_internal.hpp")
TRAFFIC = {"sources_sha256_16": "eb8c8163f98b9b3a", "read_bytes": 2908415 * 1024 * 2.000,
           "write_bytes": 15230 * 1024 * 1.000,
           # SQ_INSTS_VALU + 3 x SQ_INSTS_VALU_TRANS_F32 per ray-step (per lane) of
           # the same profile: the VALU issue slots of the compiled step
           "valu_slots_per_ray_step": 2458}
# Model bytes one ray-step of this layout gathers (10 force evaluations x 8
# corners x 16 B of (n_e, grad n_e) + one value evaluation x 8 x (4 B n_e + 4 B T)),
# and the 448 B of a layout that stores n_e only and differentiates the corners.
GATHER_BYTES_PER_RAY_STEP = 1344
GATHER_BYTES_PER_RAY_STEP_NE_ONLY = 448


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_02413_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-frequency timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint / forward timing")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batched-vs-plain record on the 4-model workload (frequency subset)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the read-bandwidth probe and the gather replay (for profiling the tracer alone)")
    ap.add_argument("--autotune-freqs", type=int, default=4,
                    help="frequencies in the autotuner's sample of the workload (0: no autotuning, defaults)")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch tuning refill_min_idle,blocks_per_cu,xcd_bands instead of autotuning")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint / forward timing on the adjoint workload (for profiling)")
    ap.add_argument("--fit", type=int, default=0, metavar="ITERS",
                    help="study: recover a structured corona's ln n_e, ln T from its own maps (ITERS Adam steps)")
    ap.add_argument("--spectrum", action="store_true",
                    help="study: disc-centre T_b spectrum and beam-convolved maps of the structured workload")
    ap.add_argument("--modes", action="store_true",
                    help="study: straight line of sight vs refraction, magnification on/off, on the structured model")
    ap.add_argument("--tube", action="store_true",
                    help="carried ray tube vs the step-wise estimate: ln S convergence, T_b effect, cost")
    ap.add_argument("--batching", action="store_true",
                    help="only run the batching study (batched vs plain on the 4-model 64-frequency workload)")
    ap.add_argument("--precision", action="store_true",
                    help="only run the precision study (mixed vs all-FP32 vs oracle on the 512x256x512 workload)")
    ap.add_argument("--grad64-oracle", metavar="PATH", default=None,
                    help="study (CPU only): the oracle's gradient on the 64x32x64 model, 64^2 x 8 image, to PATH")
    ap.add_argument("--grad64", metavar="PATH", default=None,
                    help="study: the adjoint on the same configuration vs the oracle gradient stored at PATH")
    ap.add_argument("--threads", type=int, default=None, help="oracle threads of the CPU-only studies")
    ap.add_argument("--fit-params", type=int, default=0, metavar="ITERS",
                    help="study: recover a corona's density scale, T_bg and active-region factors from its maps")
    ap.add_argument("--gradcheck", action="store_true",
                    help="study: adjoint vs oracle tape gradient and central differences on the adjoint workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, 4 launches."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 4}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cor, wl, seconds):
    """The FP64 oracle, as it stands, built for this host (g++ -O3 -march=native)
    and timed on a bounded seeded pixel sample of the workload: on all host
    threads the process may use (at most 16, the host share of one GPU), then on
    one thread.  Each leg runs about `seconds` of CPU work."""
    from oracle import oracle as O
    from paper_2606_02413_amd import corona
    t_build = time.perf_counter()
    O.build(native=True)
    O.use_library(O.NATIVE_LIB_PATH)
    t_build = time.perf_counter() - t_build
    med = O.OracleMedium.from_corona(cor)
    P = O.make_params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
    im = O.make_image(wl.n_pix, wl.half_width)
    order = corona.seeded_pixels(wl.n_pix, 4096, 3000)

    def leg(threads, budget, start, chunk):
        steps = rays = 0
        t0 = time.perf_counter()
        k = start
        while time.perf_counter() - t0 < budget and k < len(order):
            pix = order[k:k + chunk]
            for f in wl.freqs:
                r = O.trace_pixels(med, P, im, f, pix, n_threads=threads)
                steps += int(r["n_steps"].sum())
                rays += len(pix)
            k += chunk
        dt = time.perf_counter() - t0
        return {"ray_steps_per_s": steps / dt, "threads": threads, "rays": rays, "ray_steps": steps,
                "seconds": round(dt, 2), "pixels": (k - start)}

    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    threads = max(1, min(affinity, 16))
    allc = leg(threads, seconds, 0, 4 * threads)
    one = leg(1, 0.6 * seconds, 2048, 2)
    return {"value": allc["ray_steps_per_s"], "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{allc['rays']} rays ({allc['pixels']} seeded pixels x {len(wl.freqs)} freq) of the "
                      f"structured workload, {allc['ray_steps']} ray-steps in {allc['seconds']} s on {threads} threads",
            "one_core": {"value": one["ray_steps_per_s"], "unit": "ray-steps/s",
                         "sample": f"{one['rays']} rays ({one['pixels']} other seeded pixels x {len(wl.freqs)} "
                                   f"freq), {one['ray_steps']} ray-steps in {one['seconds']} s on 1 thread"},
            "parallel_speedup": allc["ray_steps_per_s"] / one["ray_steps_per_s"],
            "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": cpu_model(),
            "build": O.build_flags(native=True), "build_s": round(t_build, 1)}


def adjoint_ratio(R, torch, model, stream, reps=2):
    """Adjoint workload: the same model, 256^2 image over +/-3 R_sun, the 8
    frequencies, K = 64, loss weights w ~ U[0, 1) (seed 1000).  Forward = the
    persistent rt_trace_maps launch on that image; adjoint = rt_trace_adjoint
    (forward with checkpoints + reverse sweep + gradient gather)."""
    from paper_2606_02413_amd import corona
    wl = corona.workload("adjoint")
    im = R.image_desc(wl.n_pix, wl.half_width)
    prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, checkpoint_every=64)
    w = torch.from_numpy(corona.seeded_weights((len(wl.freqs), wl.n_pix, wl.n_pix), 1000)).cuda()
    fwd = R.trace_maps([model], wl.freqs, im, prm, info=False, stats=True)
    adj = R.trace_adjoint(model, wl.freqs, im, prm, w)
    torch.cuda.synchronize()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    f_ms = timed(lambda: R.trace_maps([model], wl.freqs, im, prm, info=False, stats=True, out=fwd))
    a_ms = timed(lambda: R.trace_adjoint(model, wl.freqs, im, prm, w, out=adj))
    steps = int(R.decode_stats(fwd["stats"])["ray_steps"])
    diff = float(((adj["tb"].double() - fwd["tb"][0].double()).abs() / fwd["tb"][0].double().abs().clamp(min=1.0)).max())
    return {"workload": f"adjoint: {wl.n_pix}^2 image x {len(wl.freqs)} freq, same model, K = 64, w ~ U[0,1)",
            "forward_ms": f_ms, "adjoint_ms": a_ms, "ratio": a_ms / f_ms, "ray_steps": steps,
            "adjoint_ray_steps_per_s": steps / (a_ms * 1e-3), "maps_max_rel_diff": diff,
            "loss": float(adj["loss"].cpu()[0])}


PRECISION_VARIANTS = (("default", dict()), ("fp32_step", dict(fp32_step=True)), ("all_fp32", dict(all_fp32=True)))


def precision_study(n_pixels=4096):
    """The three precision variants vs the FP64 oracle on the precision workload:
    512x256x512 model (r 1-30, 32 active regions, seed 4), 2048^2 image over
    +/-3 R_sun, 16 frequencies 40-800 MHz; the oracle traces 4096 pixels drawn
    with seed 3000 at every frequency.  Variants: default (FP64 state, area and
    transfer), fp32_step (FP32 state, increments and grid index; FP64 area and
    transfer), all_fp32.  Per map: max / median relative T_b error over the rays
    that end with the oracle's termination code, also over unflagged rays only,
    and the oracle's flag counts per category.  Prints one JSON line."""
    import torch
    from oracle import oracle as O
    from paper_2606_02413_amd import corona, rtsun as R
    wl = corona.workload("precision")
    t0 = time.perf_counter()
    cor = wl.models(device="cuda")[0]
    t_model = time.perf_counter() - t0
    progress(f"precision model generated in {t_model:.0f} s")
    model = R.Model.from_corona(cor)
    im = R.image_desc(wl.n_pix, wl.half_width)
    pix = corona.seeded_pixels(wl.n_pix, n_pixels, 3000)
    pix_t = torch.from_numpy(pix.astype(np.int64)).cuda()
    res = {}
    for name, flags in PRECISION_VARIANTS:
        prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, **flags)
        out = R.trace_maps([model], wl.freqs, im, prm, info=True, stats=True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        R.trace_maps([model], wl.freqs, im, prm, info=True, stats=True, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        progress(f"precision {name}: {ms:.0f} ms")
        steps = int(R.decode_stats(out["stats"])["ray_steps"])
        tb = out["tb"][0].reshape(len(wl.freqs), -1)[:, pix_t].double().cpu().numpy()
        info = out["info"][0].reshape(len(wl.freqs), -1, 32)[:, pix_t]
        code = R.decode_info(info)["code"].astype(np.int32).reshape(len(wl.freqs), -1)
        res[name] = {"tb": tb, "code": code, "ms": ms, "ray_steps": steps}
        del out
        torch.cuda.empty_cache()
    med = O.OracleMedium.from_corona(cor)
    P = O.make_params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, twin_check=True)
    imo = O.make_image(wl.n_pix, wl.half_width)
    t1 = time.perf_counter()
    maps = []
    for k, f in enumerate(wl.freqs):
        o = O.trace_pixels(med, P, imo, f, pix.astype(np.int32))
        progress(f"precision oracle {f / 1e6:.1f} MHz done")
        ok = o["flags"] == 0
        row = {"freq_MHz": round(f / 1e6, 3), "flagged": int((~ok).sum()),
               "grazing": int(((o["flags"] & O.GRAZING) != 0).sum()),
               "marginal": int(((o["flags"] & O.MARGINAL) != 0).sum()),
               "polar": int(((o["flags"] & O.POLAR) != 0).sum()), "polar_only": int((o["flags"] == O.POLAR).sum())}
        for name, _ in PRECISION_VARIANTS:
            same = res[name]["code"][k] == o["code"]
            rel = np.abs(res[name]["tb"][k] - o["tb"]) / np.maximum(np.abs(o["tb"]), 1.0)
            row[name + "_max_rel"] = float(rel[same].max())
            row[name + "_median_rel"] = float(np.median(rel[same]))
            row[name + "_max_rel_unflagged"] = float(rel[ok & same].max())
            row[name + "_median_rel_unflagged"] = float(np.median(rel[ok & same]))
            row[name + "_code_changes"] = int((~same).sum())
            row[name + "_over_1e-3"] = int((same & (rel > 1e-3)).sum())
        maps.append(row)
    t_orc = time.perf_counter() - t1
    line = {"study": "precision", "workload": "512x256x512 model (r 1-30 R_sun, 32 active regions, seed 4), "
            "2048^2 image +/-3 R_sun, 16 freq 40-800 MHz, ds_max 0.01, n_floor 0.1",
            "oracle_pixels": f"{n_pixels} seeded (seed 3000) x 16 freq", "maps": maps,
            "oracle_s": round(t_orc, 1), "oracle_threads": O.default_threads(), "model_s": round(t_model, 1)}
    for name, _ in PRECISION_VARIANTS:
        line[name] = {"ms": res[name]["ms"], "ray_steps": res[name]["ray_steps"],
                      "ray_steps_per_s": res[name]["ray_steps"] / res[name]["ms"] * 1e3,
                      "worst_max_rel": max(m[name + "_max_rel"] for m in maps),
                      "worst_median_rel": max(m[name + "_median_rel"] for m in maps),
                      "code_changes": sum(m[name + "_code_changes"] for m in maps)}
    print(json.dumps(line), flush=True)
    model.close()


def spectrum_study():
    """The disc-centre (< 0.5 R_sun) brightness-temperature spectrum of the
    structured model, 512^2 over +/-3 R_sun, at 16 frequencies 40-800 MHz, traced
    with refraction and magnification and along straight lines of sight
    (Sec. 3.4.1 derives this spectrum from its synthetic maps), and the maps
    convolved with the beam of a 15 km maximum baseline below 200 MHz and of
    5 km above (the beams of the paper's figures in Sec. 3.3).  Reports the
    spectra, the disc-centre mean of the convolved maps and the kernel times."""
    import torch
    from paper_2606_02413_amd import corona, rtsun as R
    wl = corona.workload("structured")
    model = R.Model.from_corona(wl.models(device="cuda")[0])
    im = R.image_desc(wl.n_pix, wl.half_width)
    freqs = corona.log_freqs(16)
    fw = np.where(freqs < 200e6, R.beam_fwhm(freqs, 15e3), R.beam_fwhm(freqs, 5e3))
    res = {"study": "spectrum", "workload": "structured model, 512^2 over +/-3 R_sun, 16 freq",
           "MHz": [round(f / 1e6, 2) for f in freqs], "beam_fwhm_rsun": [round(float(x), 4) for x in fw]}

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    for name, kw in (("full", dict()), ("los", dict(refraction=False, magnification=False))):
        prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, **kw)
        tb, ms = timed(lambda: R.trace_maps([model], freqs, im, prm, info=False, stats=False)["tb"][0])
        R.disc_mean(tb, im, 0.5)
        spec, ms_spec = timed(lambda: R.disc_mean(tb, im, 0.5))
        R.beam_convolve(tb, im, fw)
        conv, ms_beam = timed(lambda: R.beam_convolve(tb, im, fw))
        res[name] = {"trace_ms": ms, "disc_mean_ms": ms_spec, "beam_ms": ms_beam,
                     "tb_disc_centre_K": [round(float(x), 1) for x in spec.cpu().numpy()],
                     "tb_disc_centre_convolved_K": [round(float(x), 1) for x in R.disc_mean(conv, im, 0.5).cpu().numpy()]}
        progress(f"spectrum: {name} traced in {ms:.0f} ms, beam {ms_beam:.2f} ms")
    print(json.dumps(res), flush=True)
    model.close()


def modes_study():
    """Straight lines of sight vs refractive tracing, and the magnification term
    on and off, on the structured workload's model (256x128x256, r 1-30 R_sun,
    8 active regions, seed 0), 512^2 image over +/-3 R_sun, at 40, 60, 80, 150,
    280, 550 and 800 MHz (Sec. 3.3 compares these maps and the effect of the term).
    Per frequency: the maximum T_b of each mode; the mean T_b on the disc centre
    (projected radius < 0.5 R_sun) and in the limb annulus (0.9-1.1 R_sun), and
    their ratio (limb brightening); the median and 99th percentile of
    |T_b(LOS) - T_b(refraction)| / T_b(refraction) over pixels within 2 R_sun;
    the same for the magnification term (refraction with vs without it); and
    the largest |S_end / S_0 - 1| over rays (from ln S at the end of each ray).
    Each mode's trace is timed.  Prints one JSON line."""
    import torch
    from paper_2606_02413_amd import corona, rtsun as R
    wl = corona.workload("structured")
    model = R.Model.from_corona(wl.models(device="cuda")[0])
    n, hw = wl.n_pix, wl.half_width
    im = R.image_desc(n, hw)
    freqs = np.array([40e6, 60e6, 80e6, 150e6, 280e6, 550e6, 800e6])
    c = (np.arange(n) + 0.5) * (2 * hw / n) - hw
    rho = np.hypot(c[None, :], c[:, None])
    centre, limb, inner = rho < 0.5, (rho > 0.9) & (rho < 1.1), rho < 2.0
    modes = {"los": dict(refraction=False, magnification=False), "refraction": dict(magnification=False),
             "full": dict()}
    maps, lns, ms = {}, {}, {}
    for name, kw in modes.items():
        prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, **kw)
        out = R.trace_maps([model], freqs, im, prm, info=True, stats=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        R.trace_maps([model], freqs, im, prm, info=True, stats=False, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1)
        maps[name] = out["tb"][0].double().cpu().numpy()
        lns[name] = R.decode_info(out["info"][0])["ln_s_end"].astype(np.float64)
        progress(f"modes: {name} {ms[name]:.0f} ms")
    rows = []
    for k, f in enumerate(freqs):
        row = {"MHz": round(f / 1e6, 1)}
        for name in modes:
            t = maps[name][k]
            row[f"max_tb_{name}"] = float(t.max())
            row[f"limb_over_centre_{name}"] = float(t[limb].mean() / t[centre].mean())
        ref = maps["refraction"][k]
        for a, b, tag in (("los", "refraction", "los_vs_refraction"), ("full", "refraction", "magnification")):
            d = np.abs(maps[a][k] - maps[b][k])[inner] / np.maximum(ref[inner], 1.0)
            row[f"{tag}_median"] = float(np.median(d))
            row[f"{tag}_p99"] = float(np.quantile(d, 0.99))
        row["max_abs_S_end_over_S0_minus_1"] = float(np.abs(np.expm1(lns["full"][k])).max())
        rows.append(row)
    print(json.dumps({"study": "modes", "workload": "structured model, 512^2 over +/-3 R_sun", "ms": ms,
                      "per_frequency": rows}), flush=True)
    model.close()


def tube_study():
    """Carried ray tube vs the step-wise estimate of Eqs. 5-11 on the structured
    workload's model (256x128x256, r 1-30 R_sun, seed 0), 512^2 image over
    +/-3 R_sun, the eight frequencies 40-800 MHz, n_floor 0.1, at ds_max 0.01
    and 0.005.  Per frequency and tube: the median |ln S_end| over rays; the
    median |ln S_end(ds/2) - ln S_end(ds)| / |ln S_end(ds/2)| over rays with
    |ln S_end| > 0.1 (the step-wise value is proportional to the step, the
    carried one converges); and the median and 99th percentile over pixels
    within 2 R_sun of |T_b(tube) - T_b(no tube term)| / T_b(no tube term), the
    size of the magnification term in the maps.  Each trace is timed (the
    carried tube always runs as one launch per image).  Prints one JSON line."""
    import torch
    from paper_2606_02413_amd import corona, rtsun as R
    wl = corona.workload("structured")
    model = R.Model.from_corona(wl.models(device="cuda")[0])
    n, hw = wl.n_pix, wl.half_width
    im = R.image_desc(n, hw)
    freqs = wl.freqs
    c = (np.arange(n) + 0.5) * (2 * hw / n) - hw
    inner = np.hypot(c[None, :], c[:, None]) < 2.0
    runs = {}
    for ds in (wl.ds_max, 0.5 * wl.ds_max):
        for name, kw in (("none", dict(magnification=False, plain=True)), ("stepwise", dict(plain=True)),
                         ("carried", dict(carried_tube=True))):
            prm = R.params(ds_max=ds, n_floor=wl.n_floor, max_steps=wl.max_steps, **kw)
            out = R.trace_maps([model], freqs, im, prm, info=True, stats=True)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            R.trace_maps([model], freqs, im, prm, info=True, stats=True, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            steps = int(R.decode_stats(out["stats"])["ray_steps"])
            info = R.decode_info(out["info"][0])
            runs[name, ds] = dict(ms=ms, steps=steps, tb=out["tb"][0].double().cpu().numpy(),
                                  lns=info["ln_s_end"].astype(np.float64), code=info["code"])
            progress(f"tube: {name} ds {ds} {ms:.0f} ms, {steps / ms * 1e-6:.3f} G ray-steps/s")
    h0, h1 = wl.ds_max, 0.5 * wl.ds_max
    rows = []
    for k, f in enumerate(freqs):
        row = {"MHz": round(float(f) / 1e6, 1)}
        ref = runs["none", h0]["tb"][k]
        for name in ("stepwise", "carried"):
            a, b = runs[name, h0], runs[name, h1]
            la, lb = a["lns"][k].ravel(), b["lns"][k].ravel()
            live = (a["code"][k].ravel() != 3) & (a["code"][k].ravel() == b["code"][k].ravel())
            row[f"median_abs_ln_s_end_{name}"] = float(np.median(np.abs(la[live])))
            big = live & (np.abs(lb) > 0.1)
            row[f"halving_change_{name}"] = float(np.median(np.abs(lb[big] - la[big]) / np.abs(lb[big]))) if big.any() else None
            d = np.abs(a["tb"][k] - ref)[inner] / np.maximum(ref[inner], 1.0)
            row[f"tb_effect_{name}_median"] = float(np.median(d))
            row[f"tb_effect_{name}_p99"] = float(np.quantile(d, 0.99))
        rows.append(row)
    timing = {f"{name}_ds{ds:g}": {"ms": round(r["ms"], 1), "ray_steps": r["steps"],
                                   "g_ray_steps_per_s": round(r["steps"] / r["ms"] * 1e-6, 3)}
              for (name, ds), r in runs.items()}
    print(json.dumps({"study": "carried_tube", "workload": "structured model, 512^2 over +/-3 R_sun, 8 frequencies",
                      "timing": timing, "per_frequency": rows}), flush=True)
    model.close()


def fit_study(iters):
    """Coronal fitting through the adjoint: the maps of a structured corona
    (128x64x128, r 1-30 R_sun, random field and 8 active regions, seed 0) at the
    8 structured-workload frequencies on a 128^2 image over +/-3 R_sun are the
    data; the fit starts from the same corona without its random field and
    takes `iters` Adam steps (lr 0.01) on (ln n_e, ln T) of every vertex, the
    loss being the mean squared T_b error over the mean squared data.  Reports
    the loss and the RMS error of ln n_e on the vertices the rays reach, per
    step, and the time of a forward + backward pass."""
    import torch
    from paper_2606_02413_amd import corona, rtsun as R
    kw = dict(nr=128, nt=64, nph=128, r_in=1.0, r_max=30.0, seed=0, n_feat=256)
    truth = corona.structured(**kw)
    start = corona.structured(amp=0.0, **kw)
    wl = corona.workload("structured")
    model = R.Model.from_corona(truth)
    im = R.image_desc(128, 3.0)
    prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
    F = R.rtsun_function()
    ln_ne_true = torch.log(torch.from_numpy(truth.ne).double()).cuda()
    ln_te_true = torch.log(torch.from_numpy(truth.te).double()).cuda()
    with torch.no_grad():
        data = F.apply(ln_ne_true.float(), ln_te_true.float(), model, wl.freqs, im, prm).clone()
    norm = float((data.double() ** 2).mean())
    ln_ne = torch.log(torch.from_numpy(start.ne)).cuda().requires_grad_(True)
    ln_te = torch.log(torch.from_numpy(start.te)).cuda().requires_grad_(True)
    opt = torch.optim.Adam([ln_ne, ln_te], lr=0.01)
    hist = []
    reach = None
    times = []
    for it in range(iters + 1):
        opt.zero_grad()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tb = F.apply(ln_ne, ln_te, model, wl.freqs, im, prm)
        loss = ((tb - data) ** 2).mean() / norm
        loss.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if reach is None:
            reach = ln_ne.grad != 0
        err = float(torch.sqrt(((ln_ne.detach().double() - ln_ne_true)[reach] ** 2).mean()))
        hist.append({"step": it, "loss": float(loss), "rms_ln_ne_error_reached": err})
        if it % 5 == 0:
            progress(f"fit step {it}: loss {float(loss):.4e} rms ln n_e error {err:.4f}")
        if it < iters:
            opt.step()
    print(json.dumps({"study": "fit", "grid": "128x64x128", "image": "128^2 over +/-3 R_sun x 8 freq",
                      "vertices_reached": int(reach.sum()), "forward_backward_s_median": float(np.median(times[1:])),
                      "history": hist}), flush=True)
    model.close()


GRAD64_FIELDS = ("flags", "weights", "grad_ln_ne", "grad_ln_te")


def grad64_config():
    """The oracle-gradient check of the adjoint at its configured size: the
    adjoint workload's generator (random field and 8 active regions, seed 0,
    r 1-30 R_sun) on a 64x32x64 grid, its 64^2 image over +/-3 R_sun at the 8
    frequencies 40-800 MHz, ds_max 0.01, n_floor 0.1, weights w ~ U[0, 1)
    (seed 1000) on every ray."""
    from paper_2606_02413_amd import corona
    cor = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=0, n_feat=512)
    freqs = corona.log_freqs(8)
    w = corona.seeded_weights((8, 64, 64), 1000)
    return cor, freqs, 64, 3.0, w


def grad64_oracle(path, threads=None):
    """Oracle side (CPU only): every ray's flags (twin check), weights zeroed on
    flagged rays (their discrete path may differ between FP32 and FP64
    evaluation), then the loss and its gradient by per-ray tapes.  Writes the
    flags, weights and gradients to `path` (numpy archive)."""
    from oracle import oracle as O
    cor, freqs, n, half, w = grad64_config()
    med = O.OracleMedium.from_corona(cor)
    kw = dict(ds_max=0.01, n_floor=0.1, max_steps=200000)
    im = O.make_image(n, half)
    pix = np.arange(n * n, dtype=np.int32)
    t0 = time.perf_counter()
    flags = np.stack([O.trace_pixels(med, O.make_params(twin_check=True, **kw), im, f, pix, n_threads=threads)["flags"]
                      for f in freqs]).reshape(w.shape)
    w = np.where(flags != 0, np.float32(0.0), w).astype(np.float32)
    progress(f"grad64 oracle: flags in {time.perf_counter() - t0:.0f} s, {int((flags != 0).sum())} flagged rays")
    t1 = time.perf_counter()
    loss, gne, gte = O.grad_loss(med, O.make_params(**kw), im, freqs, w, n_threads=threads)
    progress(f"grad64 oracle: gradient in {time.perf_counter() - t1:.0f} s")
    with open(path, "wb") as fh:
        np.savez_compressed(fh, flags=flags, weights=w, grad_ln_ne=gne, grad_ln_te=gte, loss=np.array([loss]),
                            seconds=np.array([time.perf_counter() - t0]), threads=np.array([threads or 0]))
    print(json.dumps({"study": "grad64-oracle", "loss": loss, "flagged": int((flags != 0).sum()),
                      "seconds": time.perf_counter() - t0}), flush=True)


def grad_compare(label, g_gpu, g_orc):
    g = g_gpu.astype(np.float64)
    scale = float(np.abs(g_orc).max())
    d = np.abs(g - g_orc)
    nz = g_orc != 0
    return {"field": label, "max_abs_diff_over_max": float(d.max() / scale),
            "rel_l2": float(np.linalg.norm(g - g_orc) / np.linalg.norm(g_orc)),
            "frac_within_1e-4_of_max": float(np.mean(d[nz] <= 1e-4 * scale)),
            "nonzero": int(nz.sum()), "same_support": bool(np.array_equal(g_orc == 0, g == 0))}


def grad64_compare(path):
    """GPU side: rt_trace_adjoint on the configuration of grad64_config with the
    weights the oracle used (read from `path`), compared vertex by vertex with
    the oracle's gradient."""
    import torch
    from paper_2606_02413_amd import rtsun as R
    with open(path, "rb") as fh:
        z = np.load(fh)
        ref = {k: z[k] for k in z.files}
    cor, freqs, n, half, _ = grad64_config()
    m = R.Model.from_corona(cor)
    prm = R.params(ds_max=0.01, n_floor=0.1, max_steps=200000)
    w = torch.from_numpy(ref["weights"].astype(np.float32)).cuda()
    res = R.trace_adjoint(m, freqs, R.image_desc(n, half), prm, w)
    torch.cuda.synchronize()
    loss = float(res["loss"].cpu()[0])
    out = {"study": "grad64", "config": "64x32x64 structured (seed 0, r 1-30), 64^2 x 8 freq, w ~ U[0,1) seed 1000, "
                                       "flagged rays weight 0",
           "flagged_rays": int((ref["flags"] != 0).sum()), "rays": int(ref["flags"].size),
           "loss_gpu": loss, "loss_oracle": float(ref["loss"][0]),
           "loss_rel_diff": abs(loss / float(ref["loss"][0]) - 1),
           "ln_ne": grad_compare("ln_ne", res["grad_ln_ne"].cpu().numpy(), ref["grad_ln_ne"]),
           "ln_te": grad_compare("ln_te", res["grad_ln_te"].cpu().numpy(), ref["grad_ln_te"]),
           "oracle_seconds": float(ref["seconds"][0]), "oracle_threads": int(ref["threads"][0])}
    print(json.dumps(out), flush=True)
    m.close()


def gradcheck_study(n_pixels=64, n_cells=200, h=1e-3):
    """Central differences of the loss at its configured size: the adjoint
    workload (256x128x256 structured model, seed 0; 256^2 image over +/-3 R_sun;
    the 8 frequencies), loss = sum w T_b with w ~ U[0, 1) (seed 1000) on the rays
    of `n_pixels` seeded pixels (seed 2001) at every frequency and 0 elsewhere
    (and 0 on rays the oracle flags).  (1) The GPU adjoint vs the oracle's
    tape gradient at every vertex.  (2) `n_cells` vertices drawn (seed 2000) from
    the top decile of |oracle d loss / d ln n_e| and as many of |d loss / d ln T|:
    the oracle's forward loss at ln value +-h (the FP32 value e^{+-h} x, the
    difference divided by the realized ln difference), against the adjoint and
    the tape gradient.  Each FD outlier is checked for a discrete event in the
    oracle between +h and -h (a changed step count or termination code, or a
    changed cell, edge clamp or branch of any evaluation: the oracle's record of
    the ray's discrete decisions) and for the FD's own non-smoothness (FD at h/2
    against FD at h)."""
    import torch
    from oracle import oracle as O
    from paper_2606_02413_amd import corona, rtsun as R
    wl = corona.workload("adjoint")
    cor = wl.models(device="cuda")[0]
    freqs = wl.freqs
    n = wl.n_pix
    kw = dict(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
    pix = corona.seeded_pixels(n, n_pixels, 2001)
    wfull = corona.seeded_weights((len(freqs), n, n), 1000)
    med = O.OracleMedium.from_corona(cor)
    imo = O.make_image(n, wl.half_width)
    t0 = time.perf_counter()
    flags = np.stack([O.trace_pixels(med, O.make_params(twin_check=True, **kw), imo, f, pix)["flags"] for f in freqs])
    w = np.zeros_like(wfull)
    for k in range(len(freqs)):
        w[k].flat[pix] = np.where(flags[k] != 0, np.float32(0.0), wfull[k].flat[pix])
    progress(f"gradcheck: {int((flags != 0).sum())} of {flags.size} sampled rays flagged ({time.perf_counter() - t0:.0f} s)")
    t1 = time.perf_counter()
    loss_o, gne_o, gte_o = O.grad_loss(med, O.make_params(**kw), imo, freqs, w)
    t_tape = time.perf_counter() - t1
    progress(f"gradcheck: oracle tape gradient in {t_tape:.0f} s")
    m = R.Model.from_corona(cor)
    res = R.trace_adjoint(m, freqs, R.image_desc(n, wl.half_width), R.params(**kw), torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    gne = res["grad_ln_ne"].cpu().numpy().astype(np.float64)
    gte = res["grad_ln_te"].cpu().numpy().astype(np.float64)
    loss_g = float(res["loss"].cpu()[0])
    m.close()
    out = {"study": "gradcheck", "workload": "adjoint workload (256x128x256, 256^2 x 8 freq), sparse weights on "
           f"{n_pixels} seeded pixels x {len(freqs)} freq", "h": h, "loss_oracle": loss_o, "loss_gpu": loss_g,
           "loss_rel_diff": abs(loss_g / loss_o - 1), "flagged_rays": int((flags != 0).sum()),
           "oracle_tape_s": round(t_tape, 1),
           "adjoint_vs_tape": [grad_compare("ln_ne", gne, gne_o), grad_compare("ln_te", gte, gte_o)]}
    rng = np.random.Generator(np.random.PCG64(2000))
    sel_pix = np.asarray(pix, dtype=np.int32)

    def loss_of(med_x):
        """Loss of the FP64 forward on the weighted rays; per ray the step count,
        code and the record of every discrete decision (weighted rays only)."""
        tot = 0.0
        info, events = [], []
        for k, f in enumerate(freqs):
            r = O.trace_pixels(med_x, O.make_params(**kw), imo, f, sel_pix)
            tot += float((w[k].flat[sel_pix].astype(np.float64) * r["tb"]).sum())
            weighted = w[k].flat[sel_pix] != 0
            info.append(np.stack([np.where(weighted, r["n_steps"], 0), np.where(weighted, r["code"], 0)]))
            events.append(np.where(weighted, r["event_hash"], np.uint64(0)))
        return tot, np.stack(info), np.stack(events)

    fields = []
    for name, g_orc, g_gpu, arr in (("ln_ne", gne_o, gne, cor.ne), ("ln_te", gte_o, gte, cor.te)):
        mag = np.abs(g_orc).reshape(-1)
        nz = np.flatnonzero(mag > 0)
        top = nz[mag[nz] >= np.quantile(mag[nz], 0.9)]
        cells = np.sort(rng.choice(top, size=min(n_cells, top.size), replace=False))
        flat = arr.reshape(-1)
        rows = []
        t2 = time.perf_counter()
        for v in cells:
            x0 = flat[v]

            def fd(hh):
                xp, xm = np.float32(x0 * np.exp(hh)), np.float32(x0 * np.exp(-hh))
                flat[v] = xp
                lp, ip, ep = loss_of(O.OracleMedium.from_corona(cor))
                flat[v] = xm
                lm, im_, em = loss_of(O.OracleMedium.from_corona(cor))
                flat[v] = x0
                return ((lp - lm) / (np.log(np.float64(xp)) - np.log(np.float64(xm))), bool(np.array_equal(ip, im_)),
                        bool(np.array_equal(ep, em)))

            d1, same1, smooth1 = fd(h)
            go, gg = float(g_orc.reshape(-1)[v]), float(g_gpu.reshape(-1)[v])
            row = {"vertex": int(v), "fd": d1, "tape": go, "adjoint": gg,
                   "adjoint_vs_fd": abs(gg - d1) / abs(d1) if d1 != 0 else float("inf"),
                   "tape_vs_fd": abs(go - d1) / abs(d1) if d1 != 0 else float("inf"),
                   "steps_and_codes_unchanged": same1,
                   # no discrete decision of any weighted ray differs between +h and -h
                   "no_discrete_event": smooth1}
            if row["adjoint_vs_fd"] > 1e-4:
                # is the difference the FD's own (kinks of the piecewise-trilinear
                # discrete map within +-h)?  FD at smaller h, against the adjoint
                d2, same2, _ = fd(0.5 * h)
                row["fd_half_h"] = d2
                row["fd_h_vs_half_h"] = abs(d1 - d2) / abs(d2) if d2 != 0 else float("inf")
                row["adjoint_vs_fd_half_h"] = abs(gg - d2) / abs(d2) if d2 != 0 else float("inf")
                for hs in (1e-4, 1e-5):
                    ds_, _, sm_ = fd(hs)
                    row[f"no_discrete_event_{hs:g}"] = sm_
                    row[f"adjoint_vs_fd_{hs:g}"] = abs(gg - ds_) / abs(ds_) if ds_ != 0 else float("inf")
                    row[f"tape_vs_fd_{hs:g}"] = abs(go - ds_) / abs(ds_) if ds_ != 0 else float("inf")
            rows.append(row)
            if len(rows) % 10 == 0:
                progress(f"gradcheck {name}: {len(rows)} of {len(cells)} cells, "
                         f"{sum(r['adjoint_vs_fd'] <= 1e-4 for r in rows)} within 1e-4 at h")
        t_fd = time.perf_counter() - t2
        within = [r["adjoint_vs_fd"] <= 1e-4 for r in rows]
        outl = [r for r in rows if r["adjoint_vs_fd"] > 1e-4]
        conv = {}
        for hs in (1e-4, 1e-5):
            v = [r[f"adjoint_vs_fd_{hs:g}"] for r in outl]
            conv[f"outliers_within_1e-4_at_h_{hs:g}"] = int(sum(x <= 1e-4 for x in v))
            conv[f"outliers_median_adjoint_vs_fd_at_h_{hs:g}"] = float(np.median(v)) if v else 0.0
        # every outlier at h: a discrete event within +-h (the difference spans a
        # kink of the piecewise-smooth traced map), or none (unexplained)
        events = {"outliers": len(outl),
                  "with_step_or_code_change": int(sum(not r["steps_and_codes_unchanged"] for r in outl)),
                  "with_cell_or_branch_change_only": int(sum(r["steps_and_codes_unchanged"] and not r["no_discrete_event"]
                                                             for r in outl)),
                  "without_discrete_event": int(sum(r["no_discrete_event"] for r in outl)),
                  "vertices_without_event_at_h": int(sum(r["no_discrete_event"] for r in rows)),
                  "within_1e-4_of_those": int(sum(r["no_discrete_event"] and r["adjoint_vs_fd"] <= 1e-4 for r in rows))}
        fields.append({"field": name, "cells": len(rows), "fraction_within_1e-4": float(np.mean(within)),
                       "outlier_events": events, "outlier_convergence": conv,
                       # within 1e-4 at h, or else at one of the smaller h
                       "fraction_within_1e-4_any_h": float(np.mean(
                           [min(r["adjoint_vs_fd"], r.get("adjoint_vs_fd_0.0001", 1.0),
                                r.get("adjoint_vs_fd_1e-05", 1.0)) <= 1e-4 for r in rows])),
                       "tape_fraction_within_1e-4": float(np.mean([r["tape_vs_fd"] <= 1e-4 for r in rows])),
                       "median_adjoint_vs_fd": float(np.median([r["adjoint_vs_fd"] for r in rows])),
                       "outliers": outl, "fd_seconds": round(t_fd, 1)})
        progress(f"gradcheck {name}: {fields[-1]['fraction_within_1e-4']:.3f} within 1e-4, "
                 f"{len(outl)} outliers ({events['without_discrete_event']} without a discrete event), {t_fd:.0f} s")
    out["fd"] = fields
    print(json.dumps(out), flush=True)


def fit_params_study(iters):
    """Recover a known synthetic corona's density scale, background temperature
    and 8 active-region density factors from its 8-frequency maps: the structured
    model's generator on a 128x64x128 grid (r 1-30, seed 5), 128^2 image over
    +/-1.5 R_sun, 8 frequencies 40-800 MHz; the fit starts from s = 0.25,
    T_bg = 1.6 MK, A_k = 4.5: ITERS Adam steps (learning rate 0.02 x 0.95^step),
    then 8 L-BFGS iterations."""
    from paper_2606_02413_amd import corona
    from paper_2606_02413_amd.fitting import fit_params
    kw = dict(nr=128, nt=64, nph=128, r_in=1.0, r_max=30.0, seed=5, n_ar=8, n_feat=512)
    start = np.concatenate([[0.25, math.log(1.6e6)], np.full(8, math.log(3.5))])
    t0 = time.perf_counter()
    truth, hist, th = fit_params(kw, 128, 1.5, corona.log_freqs(8), iters, 0.02, start, log=progress, decay=0.95,
                                 polish=8)
    a_true = 1.0 + np.exp(truth[2:])
    a_fit = 1.0 + np.exp(th[2:])
    print(json.dumps({"study": "fit-params", "model": "128x64x128 structured (r 1-30, seed 5, 8 active regions)",
                      "image": "128^2 over +/-1.5 R_sun x 8 freq", "iters": iters, "seconds": time.perf_counter() - t0,
                      "truth": {"s": 0.0, "T_bg": 1.2e6, "A": a_true.tolist()},
                      "fit": {"s": float(th[0]), "T_bg": float(math.exp(th[1])), "A": a_fit.tolist()},
                      "abs_err_s": abs(float(th[0])), "rel_err_T_bg": abs(math.exp(th[1]) / 1.2e6 - 1),
                      "rel_err_A": (np.abs(a_fit / a_true - 1)).tolist(),
                      "history": hist[::5] + [hist[-1]]}), flush=True)


def batching_measure(R, torch, freq_stride=1, refills=(64,)):
    """Batched (one persistent launch over every model, frequency and tile) vs
    plain (one launch per image) on (a) the batched workload: the structured
    model with seeds 0-3, 64 frequencies 40-800 MHz (every `freq_stride`-th of
    them), 1024^2 image over +/-3 R_sun; (b) a long-span variant: the spherically
    symmetric 64x32x64 model (r 1-3), 64 frequencies, 1024^2 image over
    +/-2.5 R_sun, ds_max 0.005, n_floor 1, whose rays take 63 to ~1,100 steps,
    with the given refill thresholds.  Each path is timed once, after one
    untimed pass of the same call; the maps are compared bit for bit."""
    from paper_2606_02413_amd import corona
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out = {}
    wl = corona.workload("batched")
    freqs = wl.freqs[::freq_stride]
    cors = wl.models(device="cuda")
    models = [R.Model.from_corona(c) for c in cors]
    del cors
    progress(f"batched workload: {len(models)} models, {len(freqs)} of {len(wl.freqs)} frequencies")
    im = R.image_desc(wl.n_pix, wl.half_width)
    kw = dict(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
    res = R.trace_maps(models, freqs, im, R.params(**kw), info=False, stats=True)
    torch.cuda.synchronize()
    progress("batched: untimed pass done")
    b_ms = timed(lambda: R.trace_maps(models, freqs, im, R.params(**kw), info=False, stats=True, out=res))
    steps = int(R.decode_stats(res["stats"])["ray_steps"])
    progress(f"batched {b_ms:.0f} ms")
    tb_b = res["tb"]
    r1 = R.trace_maps([models[0]], freqs, im, R.params(plain=True, **kw), info=False, stats=False)
    torch.cuda.synchronize()
    p_ms = 0.0
    same = True
    for k, mdl in enumerate(models):  # plain: one launch per (model, frequency) image
        p_ms += timed(lambda: R.trace_maps([mdl], freqs, im, R.params(plain=True, **kw), info=False,
                                           stats=False, out=r1))
        same = same and bool(torch.equal(r1["tb"][0], tb_b[k]))
        progress(f"plain model {k}: cumulative {p_ms:.0f} ms")
    maps = int(tb_b.shape[0] * tb_b.shape[1])
    out["batched_workload"] = {
        "workload": f"{len(models)} structured models (seeds 0-3) x {len(freqs)} freq (every {freq_stride}th of 64, "
                    f"40-800 MHz) x {wl.n_pix}^2, ds_max {wl.ds_max}, n_floor {wl.n_floor}",
        "rays": int(tb_b.numel()), "ray_steps": steps, "batched_ms": b_ms, "plain_ms": p_ms,
        "batched_over_plain": p_ms / b_ms, "ray_steps_per_s_batched": steps / b_ms * 1e3,
        "maps_1024sq_per_s_batched": maps / b_ms * 1e3, "maps_1024sq_per_s_plain": maps / p_ms * 1e3,
        "maps_512sq_equiv_per_s_batched": tb_b.numel() / 262144 / b_ms * 1e3, "bitwise_equal": same}
    for m in models:
        m.close()
    del res, tb_b, r1
    torch.cuda.empty_cache()
    # (b) long-span variant
    cor = corona.spherically_symmetric()
    mdl = R.Model.from_corona(cor)
    freqs = corona.log_freqs(64)
    im = R.image_desc(1024, 2.5)
    kw = dict(ds_max=0.005, n_floor=1.0, max_steps=200000)
    r1 = R.trace_maps([mdl], freqs, im, R.params(plain=True, **kw), info=False, stats=True)
    torch.cuda.synchronize()
    p_ms = timed(lambda: R.trace_maps([mdl], freqs, im, R.params(plain=True, **kw), info=False, stats=True, out=r1))
    st = R.decode_stats(r1["stats"])
    steps = int(st["ray_steps"])
    span = {"workload": "spherically symmetric 64x32x64 (r 1-3), 64 freq x 1024^2 over +/-2.5 R_sun, "
                        "ds_max 0.005, n_floor 1",
            "plain_ms": p_ms, "ray_steps": steps, "max_steps": int(st["max_steps"]),
            "mean_steps_per_traced_ray": steps / max(1, int(r1["tb"].numel()) - int(st["code_count"][3]))}
    saved = R.get_tuning(mdl.device)
    for thr in refills:
        R.set_tuning(R.tuning(refill_min_idle=thr), mdl.device)
        r2 = R.trace_maps([mdl], freqs, im, R.params(**kw), info=False, stats=False)
        torch.cuda.synchronize()
        ms = timed(lambda: R.trace_maps([mdl], freqs, im, R.params(**kw), info=False, stats=False, out=r2))
        span[f"batched_ms_refill{thr}"] = ms
        span[f"batched_over_plain_refill{thr}"] = p_ms / ms
        span[f"bitwise_equal_refill{thr}"] = bool(torch.equal(r2["tb"], r1["tb"]))
        progress(f"long-span refill {thr}: {ms:.0f} ms (plain {p_ms:.0f})")
        del r2
    R.set_tuning(saved, mdl.device)
    out["long_span_variant"] = span
    mdl.close()
    del r1
    torch.cuda.empty_cache()
    return out


def batching_study():
    """The full batched workload (all 64 frequencies) and the long-span variant
    at several refill thresholds."""
    import torch
    from paper_2606_02413_amd import rtsun as R
    out = {"study": "batching"}
    out.update(batching_measure(R, torch, freq_stride=1, refills=(64, 32, 8, 1)))
    print(json.dumps(out), flush=True)


def l2_gather_roofline(R, torch, model, wl, rate, bw, replay=True):
    """The L2-gather roofline of the tracer: R_L2 from the measured streaming
    read bandwidth of the L2 and the layout's gathered bytes per ray-step, and
    R_gather from the gather-only replay of the model's recorded walks."""
    r_l2 = bw["l2_GBps"] * 1e9 / GATHER_BYTES_PER_RAY_STEP
    gathers = {"B_L2_GBps": round(bw["l2_GBps"], 1), "bytes_per_ray_step": GATHER_BYTES_PER_RAY_STEP,
               "R_L2_ray_steps_per_s": r_l2, "frac": round(rate / r_l2, 4),
               "frac_at_448_B_per_ray_step": round(rate / (bw["l2_GBps"] * 1e9 / GATHER_BYTES_PER_RAY_STEP_NE_ONLY), 4),
               "gather_GBps_equivalent": round(rate * GATHER_BYTES_PER_RAY_STEP / 1e9, 1),
               "infinity_cache_GBps": round(bw["infinity_cache_GBps"], 1), "hbm_GBps": round(bw["hbm_GBps"], 1)}
    if not replay:
        return gathers
    # gather-only replay of the same model's recorded walks (128^2 pixels x the 8
    # frequencies): the rate the memory system serves this layout's gathers at
    rep = R.gather_replay(model, wl.freqs, R.image_desc(128, wl.half_width),
                          R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps))
    gathers["R_gather_ray_steps_per_s"] = rep["ray_steps_per_s"]
    gathers["frac_of_R_gather"] = round(rate / rep["ray_steps_per_s"], 4)
    gathers["replay"] = {"walks": rep["walks"], "capacity": rep["capacity"], "ray_steps": rep["ray_steps"],
                         "ms": round(rep["ms"], 3)}
    torch.cuda.empty_cache()
    progress(f"l2-gather roofline: {gathers}")
    return gathers


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.precision:
        precision_study()
        return
    if args.batching:
        batching_study()
        return
    if args.modes:
        modes_study()
        return
    if args.spectrum:
        spectrum_study()
        return
    if args.grad64_oracle:
        grad64_oracle(args.grad64_oracle, args.threads)
        return
    if args.fit_params > 0:
        fit_params_study(args.fit_params)
        return
    if args.gradcheck:
        gradcheck_study()
        return
    if args.grad64:
        grad64_compare(args.grad64)
        return
    if args.fit > 0:
        fit_study(args.fit)
        return
    if args.tube:
        tube_study()
        return
    if args.adjoint_only:
        import torch
        from paper_2606_02413_amd import corona, rtsun as R
        cor = corona.workload("adjoint").models(device="cuda")[0]
        model = R.Model.from_corona(cor)
        print(json.dumps({"adjoint": adjoint_ratio(R, torch, model, torch.cuda.current_stream(), reps=1)}), flush=True)
        model.close()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2606_02413_amd import corona, rtsun as R

    wl = corona.workload("structured")
    cor = wl.models(device="cuda")[0]
    model = R.Model.from_corona(cor)
    im = R.image_desc(wl.n_pix, wl.half_width)
    maps_per_step = len(wl.freqs)
    stream = torch.cuda.current_stream()

    def run(plain, out=None):
        prm = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps, plain=plain)
        return R.trace_maps([model], wl.freqs, im, prm, info=False, stats=True, out=out)

    # launch tuning of the persistent trace (result-invariant): autotuned on a
    # sample of the workload unless fixed on the command line
    tune_info = None
    if args.tuning:
        rf, bpc, bands = (int(x) for x in args.tuning.split(","))
        R.set_tuning(R.tuning(rf, bpc, bands), model.device)
        tune_info = {"tuning": R.get_tuning(model.device).as_dict(), "source": "command line"}
    elif args.autotune_freqs > 0:
        prm_t = R.params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
        t0 = time.perf_counter()
        res = R.autotune([model], wl.freqs, im, prm_t, max_freqs=args.autotune_freqs)
        tune_info = {"tuning": res["tuning"], "source": f"autotuned on {args.autotune_freqs} of the frequencies",
                     "sample_best_ms": round(res["best_ms"], 3), "sample_default_ms": round(res["default_ms"], 3),
                     "tuner_s": round(time.perf_counter() - t0, 2)}
        progress(f"autotune: {tune_info}")
    else:
        tune_info = {"tuning": R.get_tuning(model.device).as_dict(), "source": "defaults"}

    # batched persistent launch (the production path)
    out = run(False)
    torch.cuda.synchronize()
    for _ in range(max(args.warmup - 1, 0)):
        run(False, out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        run(False, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    stats = R.decode_stats(out["stats"])
    steps_per_pass = int(stats["ray_steps"])
    ms_per_step = gpu_ms / args.steps
    rate = steps_per_pass / (ms_per_step * 1e-3)

    plain = None
    if not args.no_plain:
        outp = run(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(True, outp)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        same = bool(torch.equal(outp["tb"], out["tb"]))
        plain = {"ms_per_step": pms, "ray_steps_per_s": steps_per_pass / (pms * 1e-3),
                 "bitwise_equal_to_batched": same}

    adjoint = None if args.no_adjoint else adjoint_ratio(R, torch, model, stream)

    achieved_tflops = FLOPS_PER_RAY_STEP * rate / 1e12
    traffic = None
    if kernel_sources_hash() == TRAFFIC["sources_sha256_16"]:
        traffic = {"read_bytes": TRAFFIC["read_bytes"], "write_bytes": TRAFFIC["write_bytes"],
                   "bytes": TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"],
                   "GB/s": round((TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"]) / (ms_per_step * 1e-3) / 1e9, 2)}
    # Headline: the L2-gather roofline.  Algorithmic bytes per ray-step = 448
    # (13 evaluations of the model, 12 of them 8 corners x 4 B of n_e and one 8
    # corners x (n_e, T)); achieved = 448 B x ray-steps per launch / launch time;
    # peak = the chip's streaming-read bandwidth out of L2, measured in this run
    # by the library's probe kernel.
    bw = R.read_bandwidths(model.device)
    b_l2 = bw["l2_GBps"]
    achieved_gbps = GATHER_BYTES_PER_RAY_STEP_NE_ONLY * rate / 1e9
    roofline = {"bound": "l2_gather", "achieved": round(achieved_gbps, 1), "peak": round(b_l2, 1), "unit": "GB/s",
                "frac": round(achieved_gbps / b_l2, 4), "traffic": traffic,
                "kernel": "k_trace_persistent<mixed, spherical>",
                "bytes_per_ray_step": GATHER_BYTES_PER_RAY_STEP_NE_ONLY, "ray_steps_per_launch": steps_per_pass,
                "kernel_ms": round(ms_per_step, 3),
                "peak_source": "streaming read bandwidth of the L2 (probe kernel, measured in this run)"}
    alu = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved_tflops / VALU_PEAK_TFLOPS, 4), "flops_per_ray_step": FLOPS_PER_RAY_STEP}
    # the other rooflines of the tracer: VALU issue (from the profile's
    # counters, for the same kernel sources) and the gathers of this layout
    # against the L2 bandwidth and against a gather-only replay of its walks
    valu = None
    if kernel_sources_hash() == TRAFFIC["sources_sha256_16"]:
        r_valu = 256 * 2.4e9 * 64 / TRAFFIC["valu_slots_per_ray_step"]
        valu = {"slots_per_ray_step": TRAFFIC["valu_slots_per_ray_step"], "R_VALU_ray_steps_per_s": r_valu,
                "frac": round(rate / r_valu, 4)}
    gathers = l2_gather_roofline(R, torch, model, wl, rate, bw, replay=not args.no_probe)
    batching = None if args.no_batching else batching_measure(R, torch, freq_stride=8)
    cpu = None if args.no_cpu else cpu_baseline(cor, wl, args.cpu_seconds)
    line = {
        "metric": "ray-steps/s and 512^2 x 8-freq T_b maps/s (plain vs batched); adjoint/fwd ratio",
        "value": rate,
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 evaluations, f64 state/area/transfer",
        "data": "synthetic (seeded structured corona)",
        "config": {"workload": "structured corona 256x128x256 (r 1-30 R_sun), 8 active regions, "
                               "512x512 image +/-3 R_sun, 8 freq 40-800 MHz, ds_max 0.01, n_floor 0.1",
                   "global_batch": wl.n_pix * wl.n_pix * maps_per_step, "ray_steps_per_step": steps_per_pass},
        "maps_8freq_per_s": 1000.0 / ms_per_step,
        "maps_per_s": maps_per_step * 1000.0 / ms_per_step,
        "batched": {"ms_per_step": ms_per_step, "ray_steps_per_s": rate, "launch_tuning": tune_info},
        "plain": plain,
        "batched_over_plain": (plain["ms_per_step"] / ms_per_step) if plain else None,
        "batched_over_plain_c2_subset": batching["batched_workload"]["batched_over_plain"] if batching else None,
        "adjoint_fwd_ratio": adjoint["ratio"] if adjoint else None,
        "adjoint": adjoint,
        "wall_s": wall,
        "roofline": roofline,
        "alu_roofline": alu,
        "valu_roofline": valu,
        "batching": batching,
        "l2_gather_roofline": gathers,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    model.close()


if __name__ == "__main__":
    main()
