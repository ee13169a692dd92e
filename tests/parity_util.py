"""Helpers shared by the GPU parity tests (not collected as tests).

The GPU side is called only through the library's C ABI binding; the oracle
side only through oracle/oracle.py.  Both take the same seeded float32 model
arrays and the same image / stepping parameters.
"""
from __future__ import annotations

import numpy as np

# Parity bar: identical step counts and termination codes, exit position within
# 1e-5 R_sun, brightness temperature within 1e-3 relative per pixel (floored at
# 1 K).  Rays the oracle flags (grazing, marginal, polar) keep the T_b bar and
# must end with the same termination code (GRAZING rays excepted: their flag
# says a 1e-6 R_sun change of the launch may change the outcome); their step
# count is excused, and their exit bar is conditioning-aware: within 1e-5 plus
# the exit movement of the oracle's twin ray launched 1e-6 R_sun away, i.e. the
# FP32 evaluation may move a ray at most as far as a 1e-6 R_sun change of its
# launch does (its effect is that of a ~2e-7 R_sun change).  POLAR rays are
# excused from the exit bar: within a theta row of the grid's polar axis the
# FP32 azimuth of a point is resolved only to ~ulp(x)/rho (1e-5 of a cell at
# rho ~ 0.01 R_sun against ~6e-8 elsewhere) and the force is singular, so that
# noise model does not hold there (measured: exits 1.6e-5 - 4.8e-5 from the
# oracle's where the u-twin moved them 5e-6 - 2.6e-5).
EXIT_TOL = 1e-5
TB_REL_TOL = 1e-3
TB_FLOOR = 1.0
FLAG_NAMES = (("grazing", 1), ("marginal", 2), ("polar", 4))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def step_kwargs(ds_max, n_floor, *, max_steps=200000, eta=1e-2, tb_inner=1e4, tb_sky=0.0, refraction=True,
                magnification=True, no_absorption=False):
    return dict(ds_max=ds_max, n_floor=n_floor, max_steps=max_steps, eta=eta, tb_inner=tb_inner, tb_sky=tb_sky,
                refraction=refraction, magnification=magnification, no_absorption=no_absorption)


def gpu_trace(models, freqs, n_pix, half, kw, *, plain=False, all_fp32=False, fp32_step=False, path_rays=None,
              path_capacity=0,
              image=None):
    import torch
    from paper_2606_02413_amd import rtsun as R
    im = image if image is not None else R.image_desc(n_pix, half)
    prm = R.params(plain=plain, all_fp32=all_fp32, fp32_step=fp32_step, **kw)
    out = R.trace_maps(models, freqs, im, prm, info=True, stats=True, path_rays=path_rays,
                       path_capacity=path_capacity)
    torch.cuda.synchronize()
    res = {"tb": out["tb"].cpu().numpy(), "info": R.decode_info(out["info"]), "stats": R.decode_stats(out["stats"])}
    if "path" in out:
        res["path"] = out["path"].cpu().numpy()
        res["path_len"] = out["path_len"].cpu().numpy()
    return res


def oracle_trace(orc, cor, freq, n_pix, half, pixels, kw, *, twin=True, image=None):
    med = orc.OracleMedium.from_corona(cor)
    P = orc.make_params(twin_check=twin, **kw)
    im = image if image is not None else orc.make_image(n_pix, half)
    return orc.trace_pixels(med, P, im, freq, pixels)


def compare(tb_gpu, info_gpu, orc_res, *, tb_tol=TB_REL_TOL, exit_tol=EXIT_TOL, label="", flagged_tb_tol=None):
    """Compare flat arrays of GPU results with the oracle's; returns a summary dict
    (with per-flag counts and the worst differences of each category) and raises
    AssertionError with the details on failure.  `flagged_tb_tol` (per ray, or
    None for tb_tol) replaces the T_b bar on flagged rays only."""
    flags = orc_res["flags"]
    flagged = flags != 0
    ok = ~flagged
    grazing = (flags & 1) != 0
    n = len(orc_res)
    code_g = info_gpu["code"].astype(np.int32)
    steps_g = info_gpu["n_steps"]
    same_code = code_g == orc_res["code"]
    same_steps = steps_g == orc_res["n_steps"]
    dexit = np.linalg.norm(info_gpu["exit_pos"].astype(np.float64) - orc_res["exit_pos"], axis=1)
    rel = np.abs(tb_gpu.astype(np.float64) - orc_res["tb"]) / np.maximum(np.abs(orc_res["tb"]), TB_FLOOR)
    twin = orc_res["twin_dexit"]
    # a flagged ray without a twin measurement (twin check off) has no exit bar
    cond_exit = np.where((twin >= 0) & ((flags & 4) == 0), exit_tol + twin, np.inf)
    tb_bar = np.full(n, tb_tol)
    if flagged_tb_tol is not None:
        tb_bar = np.where(flagged, np.maximum(tb_tol, flagged_tb_tol), tb_bar)
    bad_code = ~same_code & ~grazing
    bad_steps = ok & ~same_steps
    bad_exit = same_code & np.where(ok, dexit > exit_tol, dexit > cond_exit)
    bad_tb = same_code & (rel > tb_bar)

    def worst(a, m):
        return float(a[m].max()) if m.any() else 0.0

    summary = dict(label=label, n=n, flagged=int(flagged.sum()), bad_code=int(bad_code.sum()),
                   bad_steps=int(bad_steps.sum()), bad_exit=int(bad_exit.sum()), bad_tb=int(bad_tb.sum()),
                   max_rel_tb=worst(rel, ok), median_rel_tb=float(np.median(rel[ok])) if ok.any() else 0.0,
                   max_dexit=worst(dexit, ok), flagged_max_rel_tb=worst(rel, flagged & same_code),
                   flagged_code_changes=int((flagged & ~same_code).sum()),
                   flagged_max_dexit_over_bar=worst(dexit / cond_exit, flagged & same_code))
    for name, bit in FLAG_NAMES + (("polar_only", 4),):
        m = (flags == bit) if name == "polar_only" else ((flags & bit) != 0)
        summary[name] = dict(n=int(m.sum()), code_changes=int((m & ~same_code).sum()),
                             step_changes=int((m & ~same_steps).sum()), max_dexit=worst(dexit, m),
                             max_rel_tb=worst(rel, m & same_code))
    print("parity", summary, flush=True)
    if bad_code.any() or bad_steps.any() or bad_exit.any() or bad_tb.any():
        idx = np.flatnonzero(bad_code | bad_steps | bad_exit | bad_tb)[:10]
        rows = [(int(i), int(flags[i]), int(orc_res["code"][i]), int(code_g[i]), int(orc_res["n_steps"][i]),
                 int(steps_g[i]), float(dexit[i]), float(twin[i]), float(rel[i]), float(orc_res["tb"][i]),
                 float(tb_gpu[i])) for i in idx]
        raise AssertionError(f"{label}: parity failures {summary}; first (idx, flags, code_o, code_g, n_o, n_g, "
                             f"dexit, twin_dexit, rel_tb, tb_o, tb_g): {rows}")
    return summary
