"""Precision variants of the tracer against the FP64 oracle, through the C ABI.

The precision form of the method: the model is evaluated in FP32 everywhere;
the ray-tube area from differences of perturbed neighbour rays (Sec. 2.1,
Eqs. 9-11, where the separations cancel) and the optical depth / brightness
accumulation (Eqs. 2-3, 12) may be FP64 or FP32, and so may the stepping (ray
state, increments, grid index).  Three variants are traced on a reduced model
of the precision workload's construction (random field and 32 active regions,
seed 4, r 1-30 R_sun; 128 x 64 x 128 instead of 512 x 256 x 512, a 192^2
image instead of 2048^2), 16 frequencies 40-800 MHz, and compared with the
oracle on seeded pixels:

  default        FP64 state, increments, grid index, area and transfer;
  FP32 stepping  FP32 state, increments and grid index; FP64 area and transfer;
  all-FP32       everything FP32.

The default variant is held to the common parity bars.  The two FP32-stepping
variants are measured: per map, the max and median relative T_b error over
every sampled ray that ends with the oracle's termination code, printed, and
bounded loosely (their stepping differs from the oracle's by FP32 rounding
accumulated over ~6,000 steps, which moves exits by up to ~1e-3 R_sun near
caustics; they are not parity variants).
"""
import numpy as np
import pytest

from paper_2606_02413_amd import corona
from tests import parity_util as PU

pytestmark = pytest.mark.gpu

N_PIX, HALF, N_SAMPLE = 192, 3.0, 64


@pytest.fixture(scope="module")
def R():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun
    return rtsun


@pytest.fixture(scope="module")
def case(R, orc):
    cor = corona.structured(nr=128, nt=64, nph=128, r_in=1.0, r_max=30.0, seed=4, n_ar=32, n_feat=512)
    m = R.Model.from_corona(cor)
    freqs = corona.log_freqs(16)
    kw = PU.step_kwargs(0.01, 0.1)
    pix = corona.seeded_pixels(N_PIX, N_SAMPLE, 3000)
    print("case precision: oracle on the sampled pixels", flush=True)
    orc_res = [PU.oracle_trace(orc, cor, f, N_PIX, HALF, pix, kw) for f in freqs]
    yield cor, m, freqs, kw, pix, orc_res
    m.close()


def _errors(g, orc_res, pix):
    rows = []
    for k, o in enumerate(orc_res):
        tb = g["tb"][0, k].reshape(-1)[pix].astype(np.float64)
        info = g["info"][0, k].reshape(-1)[pix]
        same = info["code"].astype(np.int32) == o["code"]
        rel = np.abs(tb - o["tb"]) / np.maximum(np.abs(o["tb"]), PU.TB_FLOOR)
        ok = same & (o["flags"] == 0)
        rows.append(dict(max=float(rel[same].max()), median=float(np.median(rel[same])),
                         max_unflagged=float(rel[ok].max()) if ok.any() else 0.0,
                         code_changes=int((~same).sum()), flagged=int((o["flags"] != 0).sum())))
    return rows


@pytest.mark.parametrize("variant", ["default", "fp32_step", "all_fp32"])
def test_precision_variants_against_oracle(R, case, variant):
    cor, m, freqs, kw, pix, orc_res = case
    prm_kw = dict(all_fp32=variant == "all_fp32", fp32_step=variant == "fp32_step")
    print(f"case precision {variant}", flush=True)
    g = PU.gpu_trace([m], freqs, N_PIX, HALF, kw, **prm_kw)
    rows = _errors(g, orc_res, pix)
    for f, r in zip(freqs, rows):
        print(f"precision {variant} {f / 1e6:7.1f} MHz: max {r['max']:.2e} median {r['median']:.2e} "
              f"(unflagged max {r['max_unflagged']:.2e}; code changes {r['code_changes']}, flagged {r['flagged']})",
              flush=True)
    if variant == "default":
        for k, o in enumerate(orc_res):
            PU.compare(g["tb"][0, k].reshape(-1)[pix], g["info"][0, k].reshape(-1)[pix], o,
                       label=f"precision-default-{freqs[k] / 1e6:.0f}")
        return
    worst = max(r["max"] for r in rows)
    med = max(r["median"] for r in rows)
    assert med < 1e-3, (variant, med)
    assert worst < 5e-2, (variant, worst)


def test_precision_variants_are_distinct_kernels(R, case):
    """The three variants trace different arithmetic: their maps differ in the
    last bits (and the FP32 ones from each other)."""
    cor, m, freqs, kw, pix, orc_res = case
    print("case precision variants distinct", flush=True)
    maps = [PU.gpu_trace([m], freqs[:2], 32, HALF, kw, **v)["tb"] for v in
            (dict(), dict(fp32_step=True), dict(all_fp32=True))]
    assert not np.array_equal(maps[0], maps[1])
    assert not np.array_equal(maps[1], maps[2])


@pytest.mark.parametrize("variant", ["fp32_step", "all_fp32"])
def test_precision_variants_other_modes_and_grids(R, orc, variant):
    """The FP32 variants in the reduced tracing modes (straight lines of sight,
    refraction without the tube term) on a structured spherical model, and on a
    Cartesian grid (a linear slab, the exact parabola case), against the
    oracle: the same termination codes on every compared ray, and the loose
    bars of the variants above."""
    prm_kw = dict(all_fp32=variant == "all_fp32", fp32_step=variant == "fp32_step")
    cor = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=11, n_ar=4, n_feat=256)
    m = R.Model.from_corona(cor)
    pix = np.arange(0, 32 * 32, 2, dtype=np.int32)
    rels = []
    try:
        for refr, mag in ((False, False), (True, False)):
            kw = PU.step_kwargs(0.01, 0.1, refraction=refr, magnification=mag)
            print(f"case precision {variant} modes refraction={refr} magnification={mag}", flush=True)
            g = PU.gpu_trace([m], [60e6], 32, 2.0, kw, **prm_kw)
            o = PU.oracle_trace(orc, cor, 60e6, 32, 2.0, pix, kw)
            info = g["info"].reshape(-1)[pix]
            same = info["code"].astype(np.int32) == o["code"]
            assert np.all(same | (o["flags"] != 0)), (refr, mag, int((~same).sum()))
            tb = g["tb"].reshape(-1)[pix].astype(np.float64)
            rels.append(np.abs(tb - o["tb"])[same] / np.maximum(np.abs(o["tb"][same]), PU.TB_FLOOR))
            if not mag:
                assert np.all(g["info"]["ln_s_end"] == 0)
    finally:
        m.close()
    n = 25
    k = np.arange(n)
    ne = np.broadcast_to((1e6 + 5e4 * k)[None, None, :], (n, n, n)).astype(np.float32).copy()
    te = np.full((n, n, n), 1e6, np.float32)
    d = R.grid_desc(R.RT_GRID_CARTESIAN, (n, n, n), -1.0, 5.0, origin=(-6, -6, -6), spacing=(0.5, 0.5, 0.5))
    mc = R.Model(d, ne, te)
    try:
        kw = PU.step_kwargs(0.01, 1.0)
        print(f"case precision {variant} cartesian", flush=True)
        g = PU.gpu_trace([mc], [20e6], 16, 3.0, kw, **prm_kw)
    finally:
        mc.close()
    med = orc.OracleMedium(orc.GRID_CARTESIAN, shape=(n, n, n), r_in=-1.0, r_max=5.0, ne=ne, te=te,
                           origin=(-6, -6, -6), spacing=(0.5, 0.5, 0.5))
    o = orc.trace_pixels(med, orc.make_params(**kw), orc.make_image(16, 3.0), 20e6, np.arange(256, dtype=np.int32))
    info = g["info"].reshape(-1)
    same = info["code"].astype(np.int32) == o["code"]
    assert np.all(same | (o["flags"] != 0)), int((~same).sum())
    tb = g["tb"].reshape(-1).astype(np.float64)
    rels.append(np.abs(tb - o["tb"])[same] / np.maximum(np.abs(o["tb"][same]), PU.TB_FLOOR))
    for r, label in zip(rels, ("line of sight", "refraction without the tube term", "cartesian")):
        print(f"precision {variant} {label}: max {r.max():.2e} median {np.median(r):.2e} ({r.size} rays)", flush=True)
        assert np.median(r) < 1e-3, (variant, label)
        assert r.max() < 5e-2, (variant, label)
