"""Helpers shared by the GPU parity tests (not collected as tests).

The GPU side is called only through the library's C ABI binding; the oracle
side only through oracle/oracle.py.  Both take the same seeded float32 model
arrays and the same image / stepping parameters.
"""
from __future__ import annotations

import numpy as np

# Parity bar: identical step counts and termination codes, exit position within
# 1e-5 R_sun, brightness temperature within 1e-3 relative per pixel (floored at
# 1 K), excluding rays the oracle flags as grazing, marginal or polar (counted).
EXIT_TOL = 1e-5
TB_REL_TOL = 1e-3
TB_FLOOR = 1.0


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


def gpu_trace(models, freqs, n_pix, half, kw, *, plain=False, all_fp32=False, path_rays=None, path_capacity=0,
              image=None):
    import torch
    from paper_2606_02413_amd import rtsun as R
    im = image if image is not None else R.image_desc(n_pix, half)
    prm = R.params(plain=plain, all_fp32=all_fp32, **kw)
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


def compare(tb_gpu, info_gpu, orc_res, *, tb_tol=TB_REL_TOL, exit_tol=EXIT_TOL, label=""):
    """Compare flat arrays of GPU results with the oracle's; returns a summary dict
    and raises AssertionError with the details on failure."""
    flagged = orc_res["flags"] != 0
    ok = ~flagged
    n = len(orc_res)
    code_g = info_gpu["code"].astype(np.int32)
    steps_g = info_gpu["n_steps"]
    bad_code = ok & (code_g != orc_res["code"])
    bad_steps = ok & (steps_g != orc_res["n_steps"])
    dexit = np.linalg.norm(info_gpu["exit_pos"].astype(np.float64) - orc_res["exit_pos"], axis=1)
    rel = np.abs(tb_gpu.astype(np.float64) - orc_res["tb"]) / np.maximum(np.abs(orc_res["tb"]), TB_FLOOR)
    bad_exit = ok & (dexit > exit_tol)
    bad_tb = ok & (rel > tb_tol)
    summary = dict(label=label, n=n, flagged=int(flagged.sum()),
                   grazing=int((orc_res["flags"] & 1 != 0).sum()), marginal=int((orc_res["flags"] & 2 != 0).sum()),
                   polar=int((orc_res["flags"] & 4 != 0).sum()), bad_code=int(bad_code.sum()),
                   bad_steps=int(bad_steps.sum()), bad_exit=int(bad_exit.sum()), bad_tb=int(bad_tb.sum()),
                   max_rel_tb=float(rel[ok].max()) if ok.any() else 0.0,
                   median_rel_tb=float(np.median(rel[ok])) if ok.any() else 0.0,
                   max_dexit=float(dexit[ok].max()) if ok.any() else 0.0)
    print("parity", summary, flush=True)
    if bad_code.any() or bad_steps.any() or bad_exit.any() or bad_tb.any():
        idx = np.flatnonzero(bad_code | bad_steps | bad_exit | bad_tb)[:10]
        rows = [(int(i), int(orc_res["code"][i]), int(code_g[i]), int(orc_res["n_steps"][i]), int(steps_g[i]),
                 float(dexit[i]), float(rel[i]), float(orc_res["tb"][i]), float(tb_gpu[i])) for i in idx]
        raise AssertionError(f"{label}: parity failures {summary}; first (idx, code_o, code_g, n_o, n_g, dexit, "
                             f"rel_tb, tb_o, tb_g): {rows}")
    return summary
