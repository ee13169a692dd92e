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
TRAFFIC = {"sources_sha256_16": "352d79bc859cc874", "read_bytes": 2667213 * 1024 * 2.0,
           "write_bytes": 15429 * 1024 * 1.0}


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
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, 4 launches."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 4}), flush=True)


def cpu_baseline(cor, wl, seconds):
    """The FP64 oracle, as it stands, on a bounded seeded pixel sample."""
    from oracle import oracle as O
    from paper_2606_02413_amd import corona
    med = O.OracleMedium.from_corona(cor)
    P = O.make_params(ds_max=wl.ds_max, n_floor=wl.n_floor, max_steps=wl.max_steps)
    im = O.make_image(wl.n_pix, wl.half_width)
    threads = O.default_threads()
    order = corona.seeded_pixels(wl.n_pix, 4096, 3000)
    steps = 0
    rays = 0
    t0 = time.perf_counter()
    k = 0
    chunk = 32
    while time.perf_counter() - t0 < seconds and k < len(order):
        pix = order[k:k + chunk]
        for f in wl.freqs:
            r = O.trace_pixels(med, P, im, f, pix, n_threads=threads)
            steps += int(r["n_steps"].sum())
            rays += len(pix)
        k += chunk
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{rays} rays ({rays // len(wl.freqs)} seeded pixels x {len(wl.freqs)} freq) of the "
                      f"structured workload, {steps} ray-steps in {dt:.1f} s"}


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


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
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
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_trace_persistent<mixed, spherical>", "flops_per_ray_step": FLOPS_PER_RAY_STEP,
                "kernel_ms": round(ms_per_step, 3)}
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
        "batched": {"ms_per_step": ms_per_step, "ray_steps_per_s": rate},
        "plain": plain,
        "batched_over_plain": (plain["ms_per_step"] / ms_per_step) if plain else None,
        "adjoint_fwd_ratio": adjoint["ratio"] if adjoint else None,
        "adjoint": adjoint,
        "wall_s": wall,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    model.close()


if __name__ == "__main__":
    main()
