"""Seeded synthetic coronae, image planes and frequency lists.

This module produces inputs only: electron density n_e [cm^-3] and electron
temperature T [K] sampled at the vertices of a spherical grid, plus the
frequency lists, image sizes and seeded pixel/weight draws of the workloads.
It holds none of the ray-tracing or transfer arithmetic, so both the FP64 CPU
oracle and the GPU library can take its arrays as inputs.

Grid vertex convention (the meaning of a spherical-grid descriptor; the
paper's coronal model is a spherical (r, theta, phi) grid, Sec. 3.1):

* r_a     = r_in * (r_max / r_in) ** (a / (N_r - 1)),   a = 0 .. N_r - 1
* theta_b = (b + 1/2) * pi / N_theta,                    b = 0 .. N_theta - 1
* phi_c   = 2 * pi * c / N_phi,                          c = 0 .. N_phi - 1

Arrays are float32, C-order [N_r][N_theta][N_phi].

The density follows the Baumbach-Allen form; the random-field and
active-region structure stand in for the global MHD cube used in the paper
(Sec. 3.1), which is not available here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

R_SUN_CM = 6.957e10


def ba_density(r):
    """Baumbach-Allen electron density [cm^-3] at heliocentric radius r [R_sun]."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0e8 * (2.99 * r ** -16 + 1.55 * r ** -6 + 0.036 * r ** -1.5)


def log_freqs(n, lo=40e6, hi=800e6):
    """n frequencies [Hz] log-spaced from lo to hi inclusive (40-800 MHz band, Sec. 1)."""
    if n == 1:
        return np.array([lo], dtype=np.float64)
    f = np.exp(np.linspace(math.log(lo), math.log(hi), n))
    f[0], f[-1] = lo, hi
    return f


def vertex_coords(nr, nt, nph, r_in, r_max):
    """Vertex coordinates (r, theta, phi) of a spherical grid (see module doc)."""
    a = np.arange(nr, dtype=np.float64)
    r = r_in * (r_max / r_in) ** (a / (nr - 1))
    th = (np.arange(nt, dtype=np.float64) + 0.5) * math.pi / nt
    ph = 2.0 * math.pi * np.arange(nph, dtype=np.float64) / nph
    return r, th, ph


def vertex_xyz(nr, nt, nph, r_in, r_max):
    """Cartesian positions [R_sun] of all vertices, shape (nr, nt, nph, 3), float64."""
    r, th, ph = vertex_coords(nr, nt, nph, r_in, r_max)
    st, ct = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    x = r[:, None, None] * st[None, :, None] * cp[None, None, :]
    y = r[:, None, None] * st[None, :, None] * sp[None, None, :]
    z = r[:, None, None] * ct[None, :, None] * np.ones_like(ph)[None, None, :]
    return np.stack([x, y, z], axis=-1)


@dataclasses.dataclass
class Corona:
    """A gridded corona: descriptor fields plus float32 n_e and T arrays."""
    nr: int
    nt: int
    nph: int
    r_in: float
    r_max: float
    ne: np.ndarray  # float32 [nr][nt][nph], cm^-3
    te: np.ndarray  # float32 [nr][nt][nph], K
    label: str = ""

    @property
    def shape(self):
        return (self.nr, self.nt, self.nph)


def spherically_symmetric(nr=64, nt=32, nph=64, r_in=1.0, r_max=3.0, t_iso=1.0e6):
    """Baumbach-Allen density, isothermal; the small plain-method workload."""
    r, _, _ = vertex_coords(nr, nt, nph, r_in, r_max)
    ne = np.broadcast_to(ba_density(r)[:, None, None], (nr, nt, nph)).astype(np.float32)
    te = np.full((nr, nt, nph), t_iso, dtype=np.float32)
    return Corona(nr, nt, nph, r_in, r_max, np.ascontiguousarray(ne), te, "ba-symmetric")


def _random_field(xyz_flat, rng, n_feat, ell, device):
    """Gaussian random field with unit variance and covariance exp(-d^2 / 2 ell^2).

    Random Fourier features: g(x) = sqrt(2/M) sum_m cos(k_m . x + phi_m) with
    k_m ~ N(0, ell^-2 I) and phi_m ~ U[0, 2 pi).  Evaluated in float64.
    """
    k = rng.standard_normal((n_feat, 3)) / ell
    ph = rng.uniform(0.0, 2.0 * math.pi, n_feat)
    scale = math.sqrt(2.0 / n_feat)
    try:
        import torch
    except ImportError:  # pragma: no cover - torch is present in this image
        torch = None
    n = xyz_flat.shape[0]
    out = np.empty(n, dtype=np.float64)
    chunk = 1 << 18
    if torch is not None:
        dev = torch.device(device)
        kt = torch.from_numpy(k).to(dev)
        pt = torch.from_numpy(ph).to(dev)
        for s in range(0, n, chunk):
            xt = torch.from_numpy(xyz_flat[s:s + chunk]).to(dev)
            g = torch.cos(xt @ kt.T + pt).sum(dim=1) * scale
            out[s:s + chunk] = g.cpu().numpy()
    else:
        for s in range(0, n, chunk):
            out[s:s + chunk] = np.cos(xyz_flat[s:s + chunk] @ k.T + ph).sum(axis=1) * scale
    return out


def structured_parts(nr=256, nt=128, nph=256, r_in=1.0, r_max=30.0, seed=0, n_ar=8, n_feat=512, ell=0.1,
                     device="cpu"):
    """The seeded pieces of a structured corona (see structured()), float64 over
    the vertices in C order: ln of the Baumbach-Allen density, the random field
    g, the unit Gaussian profile G_k of every active region, and the active
    regions' density factors A_k and peak temperatures T_k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = vertex_xyz(nr, nt, nph, r_in, r_max).reshape(-1, 3)
    r, _, _ = vertex_coords(nr, nt, nph, r_in, r_max)
    g = _random_field(xyz, rng, n_feat, ell, device)
    ba = np.broadcast_to(ba_density(r)[:, None, None], (nr, nt, nph)).reshape(-1)
    prof, dens, temp = [], [], []
    for _ in range(n_ar):
        rc = rng.uniform(1.05, 1.2)
        ctc = rng.uniform(-0.5, 0.5)
        phc = rng.uniform(-0.5 * math.pi, 0.5 * math.pi)
        w = rng.uniform(0.05, 0.15)
        dens.append(rng.uniform(3.0, 8.0))
        temp.append(rng.uniform(2.0e6, 3.0e6))
        stc = math.sqrt(1.0 - ctc * ctc)
        c = np.array([rc * stc * math.cos(phc), rc * stc * math.sin(phc), rc * ctc])
        d2 = ((xyz - c) ** 2).sum(axis=1)
        prof.append(np.exp(-d2 / (2.0 * w * w)))
    return {"ba": ba, "g": g, "G": np.array(prof).reshape(n_ar, -1), "A": np.array(dens), "T": np.array(temp)}


def structured(nr=256, nt=128, nph=256, r_in=1.0, r_max=30.0, seed=0, n_ar=8,
               t_bg=1.2e6, n_feat=512, ell=0.1, amp=0.3, device="cpu"):
    """Baumbach-Allen x exp(amp*g) with Gaussian active regions (seeded).

    Draw order from numpy PCG64(seed): field wave vectors, field phases, then per
    active region (r_c, cos theta_c, phi_c, width, density factor, temperature).
    Active regions: centre r_c ~ U[1.05, 1.2], cos theta_c ~ U[-0.5, 0.5],
    phi_c ~ U[-pi/2, pi/2] (facing +x), width ~ U[0.05, 0.15], density factor
    A ~ U[3, 8], peak temperature ~ U[2, 3] MK.  With G = exp(-|x - x_c|^2 / 2w^2):
    n_e <- n_e * prod(1 + (A - 1) G);  T = t_bg + max_k (T_k - t_bg) G_k.
    """
    p = structured_parts(nr, nt, nph, r_in, r_max, seed, n_ar, n_feat, ell, device)
    ne = p["ba"] * np.exp(amp * p["g"])
    te = np.full(ne.shape[0], t_bg, dtype=np.float64)
    dte = np.zeros(ne.shape[0], dtype=np.float64)
    for k in range(n_ar):
        gk = p["G"][k]
        ne *= 1.0 + (p["A"][k] - 1.0) * gk
        dte = np.maximum(dte, (p["T"][k] - t_bg) * gk)
    te = te + dte
    return Corona(nr, nt, nph, r_in, r_max,
                  ne.reshape(nr, nt, nph).astype(np.float32),
                  te.reshape(nr, nt, nph).astype(np.float32),
                  f"structured-seed{seed}-ar{n_ar}")


# ---------------------------------------------------------------------------
# Workloads.  Each names the model, image, frequencies and stepping controls.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    model_kwargs: list          # one dict per model (structured() or symmetric)
    symmetric: bool
    n_pix: int                  # image is n_pix x n_pix
    half_width: float           # image half-width [R_sun]
    freqs: np.ndarray           # Hz
    ds_max: float
    n_floor: float
    max_steps: int = 200000

    def models(self, device="cpu"):
        if self.symmetric:
            return [spherically_symmetric(**kw) for kw in self.model_kwargs]
        return [structured(device=device, **kw) for kw in self.model_kwargs]


def workload(name):
    """The five workloads: plain-small, structured, batched, adjoint, precision."""
    if name == "small":
        return Workload("small", [dict()], True, 64, 2.5, np.array([150e6]), 0.005, 1.0)
    if name == "structured":
        return Workload("structured", [dict(seed=0)], False, 512, 3.0, log_freqs(8), 0.01, 0.1)
    if name == "batched":
        return Workload("batched", [dict(seed=s) for s in range(4)], False, 1024, 3.0,
                        log_freqs(64), 0.01, 0.1)
    if name == "adjoint":
        return Workload("adjoint", [dict(seed=0)], False, 256, 3.0, log_freqs(8), 0.01, 0.1)
    if name == "precision":
        return Workload("precision", [dict(nr=512, nt=256, nph=512, seed=4, n_ar=32)], False,
                        2048, 3.0, log_freqs(16), 0.01, 0.1)
    raise KeyError(name)


def seeded_pixels(n_pix, count, seed):
    """`count` distinct flat pixel indices of an n_pix x n_pix image (row = v, col = u)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_pix * n_pix, size=count, replace=False)).astype(np.int32)


def seeded_weights(shape, seed):
    """Loss weights w ~ U[0, 1), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=shape).astype(np.float32)
