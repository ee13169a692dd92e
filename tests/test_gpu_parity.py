"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Each case prints its label before the GPU call so that a failure names it.
"""
import numpy as np
import pytest

from paper_2606_02413_amd import corona
from tests import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun
    return rtsun


@pytest.fixture(scope="module")
def small_model(R):
    cor = corona.spherically_symmetric()
    return cor, R.Model.from_corona(cor)


@pytest.fixture(scope="module")
def structured_small(R):
    cor = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=11, n_ar=4, n_feat=256)
    return cor, R.Model.from_corona(cor)


def test_small_workload_full_map(R, orc, small_model):
    """Spherically symmetric Baumbach-Allen, 64x32x64, 64^2 image, 150 MHz, fixed dt = 0.005."""
    cor, m = small_model
    kw = PU.step_kwargs(0.005, 1.0)
    print("case small full map", flush=True)
    g = PU.gpu_trace([m], [150e6], 64, 2.5, kw, plain=True)
    pix = np.arange(64 * 64, dtype=np.int32)
    o = PU.oracle_trace(orc, cor, 150e6, 64, 2.5, pix, kw)
    s = PU.compare(g["tb"].reshape(-1), g["info"].reshape(-1), o, label="small")
    assert s["flagged"] < 0.05 * s["n"]
    st = g["stats"]
    assert st["ray_steps"] == int(g["info"]["n_steps"].sum())
    assert st["code_count"][3] == int((o["code"] == 3).sum())


@pytest.mark.parametrize("freq", [40e6, 80e6, 300e6])
def test_small_workload_frequencies(R, orc, small_model, freq):
    cor, m = small_model
    kw = PU.step_kwargs(0.005, 1.0)
    print(f"case small f={freq}", flush=True)
    g = PU.gpu_trace([m], [freq], 64, 2.5, kw)
    pix = np.arange(0, 64 * 64, 3, dtype=np.int32)
    o = PU.oracle_trace(orc, cor, freq, 64, 2.5, pix, kw)
    PU.compare(g["tb"].reshape(-1)[pix], g["info"].reshape(-1)[pix], o, label=f"small-{freq/1e6:.0f}MHz")


@pytest.mark.parametrize("variant", ["full", "no-magnification", "line-of-sight", "fp32-step", "all-fp32"])
def test_persistent_equals_plain_bitwise(R, structured_small, variant):
    """Both launch forms run the same per-ray code: bitwise equal maps, ray
    records and step totals in every tracing mode and precision variant."""
    cor, m = structured_small
    kw = PU.step_kwargs(0.01, 0.1, refraction=variant != "line-of-sight",
                        magnification=variant not in ("no-magnification", "line-of-sight"))
    extra = dict(fp32_step=variant == "fp32-step", all_fp32=variant == "all-fp32")
    freqs = corona.log_freqs(3)
    print(f"case persistent vs plain {variant}", flush=True)
    a = PU.gpu_trace([m, m], freqs, 45, 3.0, kw, plain=True, **extra)
    b = PU.gpu_trace([m, m], freqs, 45, 3.0, kw, plain=False, **extra)
    assert np.array_equal(a["tb"].view(np.uint32), b["tb"].view(np.uint32))
    assert np.array_equal(a["info"].view(np.uint8), b["info"].view(np.uint8))
    assert a["stats"]["ray_steps"] == b["stats"]["ray_steps"]


def test_two_different_models_in_one_call(R, orc, structured_small):
    """Two models with different random fields and active regions in one
    persistent launch: each image matches the oracle on its own model."""
    cor_a, m_a = structured_small
    cor_b = corona.structured(nr=64, nt=32, nph=64, r_in=1.0, r_max=30.0, seed=12, n_ar=4, n_feat=256)
    m_b = R.Model.from_corona(cor_b)
    kw = PU.step_kwargs(0.01, 0.1)
    freqs = [60e6, 240e6]
    n, half = 24, 2.0
    print("case two models", flush=True)
    g = PU.gpu_trace([m_a, m_b], freqs, n, half, kw)
    pix = np.arange(n * n, dtype=np.int32)
    for mi, cor in enumerate((cor_a, cor_b)):
        med = orc.OracleMedium.from_corona(cor)
        P = orc.make_params(twin_check=True, **kw)
        for k, f in enumerate(freqs):
            res = orc.trace_pixels(med, P, orc.make_image(n, half), f, pix)
            PU.compare(g["tb"][mi, k].reshape(-1), g["info"][mi, k].reshape(-1), res, label=f"model{mi}-{f/1e6:.0f}")
    assert not np.array_equal(g["tb"][0], g["tb"][1])
    m_b.close()


def test_every_launch_tuning_gives_the_same_maps(R, structured_small):
    """Every tuning the autotuner may choose (refill threshold, blocks per CU,
    die bands) traces the same bits as the plain per-image launch."""
    cor, m = structured_small
    kw = PU.step_kwargs(0.01, 0.1)
    freqs = corona.log_freqs(3)
    print("case launch tunings", flush=True)
    ref = PU.gpu_trace([m], freqs, 45, 3.0, kw, plain=True)
    try:
        for rf, bpc, bands in ((1, 1, 1), (8, 2, 8), (32, 1, 8), (16, 0, 1)):
            R.set_tuning(R.tuning(rf, bpc, bands), m.device)
            got = PU.gpu_trace([m], freqs, 45, 3.0, kw, plain=False)
            assert np.array_equal(ref["tb"].view(np.uint32), got["tb"].view(np.uint32)), (rf, bpc, bands)
            assert np.array_equal(ref["info"].view(np.uint8), got["info"].view(np.uint8)), (rf, bpc, bands)
    finally:
        R.set_tuning(R.tuning(), m.device)


def test_autotune_installs_a_tuning_and_caches_it(R, structured_small, tmp_path):
    import torch
    cor, m = structured_small
    freqs = corona.log_freqs(4)
    im = R.image_desc(45, 3.0)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    cache = str(tmp_path / "tuning.json")
    print("case autotune", flush=True)
    try:
        res = R.autotune([m], freqs, im, prm, max_freqs=2, cache=cache)
        assert not res["cached"] and res["best_ms"] > 0 and res["best_ms"] <= res["default_ms"]
        t = res["tuning"]
        assert 1 <= t["refill_min_idle"] <= 64 and t["xcd_bands"] in (1, 8) and t["blocks_per_cu"] >= 0
        assert R.get_tuning(m.device).as_dict() == t
        R.set_tuning(R.tuning(), m.device)
        again = R.autotune([m], freqs, im, prm, max_freqs=2, cache=cache)
        assert again["cached"] and again["tuning"] == t and R.get_tuning(m.device).as_dict() == t
        tuned = R.trace_maps([m], freqs, im, prm, info=False, stats=False)["tb"]
        plain = R.trace_maps([m], freqs, im, R.params(ds_max=0.01, n_floor=0.1, plain=True), info=False,
                             stats=False)["tb"]
        torch.cuda.synchronize()
        assert torch.equal(tuned, plain)
    finally:
        R.set_tuning(R.tuning(), m.device)


@pytest.mark.parametrize("adaptive", [False, True])
def test_structured_ragged_image(R, orc, structured_small, adaptive):
    """Random-field corona with active regions, r 1-30, ragged 37x29 image (tiles with a tail)."""
    cor, m = structured_small
    kw = PU.step_kwargs(0.01, 0.1 if adaptive else 1.0)
    freqs = [40e6, 150e6, 800e6]
    nu, nv = 37, 29
    im_g = R.image_desc(nu, 3.0, nv=nv, half_v=2.4)
    print(f"case structured ragged adaptive={adaptive}", flush=True)
    g = PU.gpu_trace([m], freqs, nu, 3.0, kw, image=im_g)
    im_o = orc.make_image(nu, 3.0, nv=nv, half_v=2.4)
    pix = np.arange(nu * nv, dtype=np.int32)
    for k, f in enumerate(freqs):
        o = PU.oracle_trace(orc, cor, f, nu, 3.0, pix, kw, image=im_o)
        PU.compare(g["tb"][0, k].reshape(-1), g["info"][0, k].reshape(-1), o, label=f"ragged-{f/1e6:.0f}")


@pytest.mark.parametrize("nu,nv", [(1, 1), (1, 9), (13, 1), (8, 8), (9, 8)])
def test_degenerate_and_single_tile_images(R, orc, structured_small, nu, nv):
    """Images of one pixel, one row or column (a tile that is mostly tail), one
    exact 8x8 tile and one tile plus a one-column tail, through both launch
    schedules, against the oracle on every pixel."""
    cor, m = structured_small
    kw = PU.step_kwargs(0.01, 0.1)
    im_g = R.image_desc(nu, 1.7, nv=nv, half_v=1.3)
    im_o = orc.make_image(nu, 1.7, nv=nv, half_v=1.3)
    pix = np.arange(nu * nv, dtype=np.int32)
    o = PU.oracle_trace(orc, cor, 90e6, nu, 1.7, pix, kw, image=im_o)
    maps = []
    for plain in (False, True):
        print(f"case image {nu}x{nv} plain={plain}", flush=True)
        g = PU.gpu_trace([m], [90e6], nu, 1.7, kw, image=im_g, plain=plain)
        assert g["tb"].shape == (1, 1, nv, nu)
        PU.compare(g["tb"].reshape(-1), g["info"].reshape(-1), o, label=f"image-{nu}x{nv}-{plain}")
        maps.append(g["tb"])
    assert np.array_equal(maps[0], maps[1])


@pytest.mark.parametrize("obs_dir,up", [((0.3, -0.8, 0.52), (0.0, 0.0, 1.0)),
                                         ((0.3420201433, 0.0, 0.9396926208), (0.0, 1.0, 0.0))])
def test_observer_directions(R, orc, structured_small, obs_dir, up):
    """An oblique observer, and one 20 degrees from the polar axis, whose chords
    have |t_z| > 0.9 and so take the y reference axis of Eq. 6."""
    cor, m = structured_small
    o = tuple(float(x) for x in np.asarray(obs_dir) / np.linalg.norm(obs_dir))
    kw = PU.step_kwargs(0.01, 0.1)
    n, half, freqs = 24, 2.0, [80e6, 300e6]
    print(f"case observer {o}", flush=True)
    g = PU.gpu_trace([m], freqs, n, half, kw, image=R.image_desc(n, half, obs_dir=o, up=up))
    im_o = orc.make_image(n, half, obs_dir=o, up=up)
    pix = np.arange(n * n, dtype=np.int32)
    for k, f in enumerate(freqs):
        res = PU.oracle_trace(orc, cor, f, n, half, pix, kw, image=im_o)
        s = PU.compare(g["tb"][0, k].reshape(-1), g["info"][0, k].reshape(-1), res, label=f"observer-{f/1e6:.0f}")
        # flagged rays keep the T_b bar and a conditioning-aware exit bar; the
        # share bound keeps the exact step-count and exit bars on most rays
        # (the low-frequency rays of this small random-field model cross many
        # caustics: 25-32 % are flagged at 80 MHz)
        assert s["flagged"] < 0.4 * s["n"]


def test_los_and_no_magnification_modes(R, orc, structured_small):
    cor, m = structured_small
    pix = np.arange(0, 32 * 32, 2, dtype=np.int32)
    for refr, mag in ((False, False), (True, False)):
        kw = PU.step_kwargs(0.01, 0.1, refraction=refr, magnification=mag)
        print(f"case modes refraction={refr} magnification={mag}", flush=True)
        g = PU.gpu_trace([m], [60e6], 32, 2.0, kw)
        o = PU.oracle_trace(orc, cor, 60e6, 32, 2.0, pix, kw)
        PU.compare(g["tb"].reshape(-1)[pix], g["info"].reshape(-1)[pix], o, label=f"modes-{refr}-{mag}")
        if not mag:
            assert np.all(g["info"]["ln_s_end"] == 0)


def test_flux_tube_identity_on_gpu(R, structured_small):
    """kappa = 0, equal boundary temperatures: T_b = T0 exp(ln S_end/S_0) (Eq. 1)."""
    cor, m = structured_small
    kw = PU.step_kwargs(0.01, 0.1, no_absorption=True, tb_inner=5e5, tb_sky=5e5)
    print("case flux tube", flush=True)
    g = PU.gpu_trace([m], [60e6], 32, 2.0, kw)
    info = g["info"].reshape(-1)
    hit = info["code"] != 3
    want = 5e5 * np.exp(info["ln_s_end"][hit].astype(np.float64))
    assert np.max(np.abs(g["tb"].reshape(-1)[hit] / want - 1)) < 1e-5


def test_max_steps_and_miss(R, orc, small_model):
    cor, m = small_model
    kw = PU.step_kwargs(0.005, 1.0, max_steps=37)
    print("case max_steps", flush=True)
    g = PU.gpu_trace([m], [150e6], 16, 2.5, kw)
    o = PU.oracle_trace(orc, cor, 150e6, 16, 2.5, np.arange(256, dtype=np.int32), kw)
    PU.compare(g["tb"].reshape(-1), g["info"].reshape(-1), o, label="max-steps")
    assert (g["info"]["code"] == 4).any() and (g["info"]["code"] == 3).any()
    assert g["info"]["n_steps"].max() == 37


def test_cartesian_grid_parabola(R, orc):
    """Linear slab on a Cartesian grid: GPU and oracle parity on the exact parabola case."""
    n = 25
    k = np.arange(n)
    ne = np.broadcast_to((1e6 + 5e4 * k)[None, None, :], (n, n, n)).astype(np.float32).copy()
    te = np.full((n, n, n), 1e6, np.float32)
    d = R.grid_desc(R.RT_GRID_CARTESIAN, (n, n, n), -1.0, 5.0, origin=(-6, -6, -6), spacing=(0.5, 0.5, 0.5))
    m = R.Model(d, ne, te)
    kw = PU.step_kwargs(0.01, 1.0)
    print("case cartesian", flush=True)
    g = PU.gpu_trace([m], [20e6], 16, 3.0, kw)
    med = orc.OracleMedium(orc.GRID_CARTESIAN, shape=(n, n, n), r_in=-1.0, r_max=5.0, ne=ne, te=te,
                           origin=(-6, -6, -6), spacing=(0.5, 0.5, 0.5))
    o = orc.trace_pixels(med, orc.make_params(**kw), orc.make_image(16, 3.0), 20e6, np.arange(256, dtype=np.int32))
    PU.compare(g["tb"].reshape(-1), g["info"].reshape(-1), o, label="cartesian")
    m.close()


def test_path_output_matches_oracle(R, orc, small_model):
    cor, m = small_model
    kw = PU.step_kwargs(0.005, 1.0)
    rays = [32 * 64 + 30, 10 * 64 + 12]
    print("case paths", flush=True)
    g = PU.gpu_trace([m], [80e6], 64, 2.5, kw, path_rays=rays, path_capacity=2000)
    med = orc.OracleMedium.from_corona(cor)
    for slot, ray in enumerate(sorted(rays)):
        res, path = orc.trace_pixel_path(med, orc.make_params(**kw), orc.make_image(64, 2.5), 80e6, ray)
        n = int(g["path_len"][slot])
        assert n == len(path) == res["n_steps"]
        gp = g["path"][slot, :n]
        assert np.max(np.abs(gp[:, :3] - path[:, :3])) < 1e-5
        assert np.max(np.abs(gp[:, 6] - path[:, 6]) / np.maximum(path[:, 6], 1e-6)) < 1e-3


def test_structured_workload_full_size_sampled(R, orc):
    """The benchmark workload at full size in the launch bench.py times: the
    256x128x256 structured model (r 1-30), one persistent launch over the
    512^2 x 8-frequency stack (40-800 MHz), ds_max 0.01, n_floor 0.1; the oracle
    on 48 seeded pixels per frequency."""
    import torch
    wl = corona.workload("structured")
    cor = wl.models(device="cuda")[0]
    m = R.Model.from_corona(cor)
    kw = PU.step_kwargs(wl.ds_max, wl.n_floor, max_steps=wl.max_steps)
    print("case structured full size, persistent", flush=True)
    g = PU.gpu_trace([m], wl.freqs, wl.n_pix, wl.half_width, kw)
    st = g["stats"]
    assert st["ray_steps"] == int(g["info"]["n_steps"].sum())
    pix = corona.seeded_pixels(wl.n_pix, 48, 3001)
    flagged = 0
    for k, f in enumerate(wl.freqs):
        o = PU.oracle_trace(orc, cor, f, wl.n_pix, wl.half_width, pix, kw)
        s = PU.compare(g["tb"][0, k].reshape(-1)[pix], g["info"][0, k].reshape(-1)[pix], o,
                       label=f"full-{f/1e6:.0f}MHz")
        flagged += s["flagged"]
    # (15 % flagged, mostly twin-sensitive rays at 40-94 MHz)
    assert flagged < 0.2 * len(pix) * len(wl.freqs)
    m.close()
    torch.cuda.empty_cache()


def test_batched_workload_sampled(R, orc):
    """The batched workload in the launch bench.py times: the structured model
    with seeds 0-3, every 8th of its 64 frequencies (40-800 MHz), 1024^2 image
    over +/-3 R_sun, all in one persistent launch; the oracle on 16 seeded
    pixels of every (model, frequency) map, and the launch's step statistics
    against the per-ray step counts."""
    wl = corona.workload("batched")
    freqs = wl.freqs[::8]
    cors = wl.models(device="cuda")
    models = [R.Model.from_corona(c) for c in cors]
    kw = PU.step_kwargs(wl.ds_max, wl.n_floor, max_steps=wl.max_steps)
    try:
        print(f"case batched workload: {len(models)} models x {len(freqs)} frequencies x {wl.n_pix}^2", flush=True)
        g = PU.gpu_trace(models, freqs, wl.n_pix, wl.half_width, kw)
        assert g["tb"].shape == (len(models), len(freqs), wl.n_pix, wl.n_pix)
        assert g["stats"]["ray_steps"] == int(g["info"]["n_steps"].astype(np.int64).sum())
        pix = corona.seeded_pixels(wl.n_pix, 16, 3002)
        n = flagged = 0
        for mi, cor in enumerate(cors):
            for k, f in enumerate(freqs):
                o = PU.oracle_trace(orc, cor, f, wl.n_pix, wl.half_width, pix, kw)
                s = PU.compare(g["tb"][mi, k].reshape(-1)[pix], g["info"][mi, k].reshape(-1)[pix], o,
                               label=f"batched-model{mi}-{f/1e6:.0f}MHz")
                n += s["n"]
                flagged += s["flagged"]
        assert flagged < 0.3 * n, (flagged, n)
    finally:
        for m in models:
            m.close()


def test_vacuum_model(R, orc):
    """n_e = 0 everywhere (a degenerate model the method allows): n = 1, so
    every ray is a straight chord with M = 1 at every step and no absorption;
    T_b is the boundary brightness behind it (tb_inner for chords that meet
    r_in, i.e. impact parameter b < r_in; tb_sky otherwise), ln S_end = 0, and
    the GPU matches the oracle ray by ray."""
    import torch
    nr, nt, nph = 16, 8, 16
    ne = np.zeros((nr, nt, nph), np.float32)
    te = np.full((nr, nt, nph), 1e6, np.float32)
    m = R.Model(R.grid_desc(R.RT_GRID_SPHERICAL_LOGR, (nr, nt, nph), 1.0, 3.0), ne, te)
    kw = PU.step_kwargs(0.01, 1.0, tb_inner=1e4, tb_sky=0.0)
    print("case vacuum model", flush=True)
    try:
        g = PU.gpu_trace([m], [100e6], 16, 2.5, kw)
    finally:
        m.close()
    tb = g["tb"].reshape(-1)
    info = g["info"].reshape(-1)
    u = -2.5 + (np.arange(16) + 0.5) * 5.0 / 16
    b = np.sqrt(u[None, :] ** 2 + u[:, None] ** 2).reshape(-1)
    hit = b < 1.0
    assert np.all(info["code"][hit] == 2) and np.all(tb[hit] == np.float32(1e4))
    traced = (~hit) & (b < 3.0)
    assert np.all(info["code"][traced] == 1) and np.all(tb[traced] == 0.0)
    assert np.max(np.abs(info["ln_s_end"][info["code"] != 3])) < 1e-9
    med = orc.OracleMedium(orc.GRID_SPHERICAL_LOGR, shape=(nr, nt, nph), r_in=1.0, r_max=3.0, ne=ne, te=te)
    o = orc.trace_pixels(med, orc.make_params(**kw), orc.make_image(16, 2.5), 100e6, np.arange(256, dtype=np.int32))
    PU.compare(tb, info, o, label="vacuum")


def test_call_capacity_limits(R, structured_small):
    """The largest call shapes: 16 models and 128 frequencies in one persistent
    launch give bitwise the maps of single-model, single-frequency calls; one
    model or frequency more is refused before any device work."""
    import torch
    cor, m = structured_small
    prm = R.params(ds_max=0.01, n_floor=0.1)
    im = R.image_desc(8, 2.0)
    freqs = corona.log_freqs(128)
    print("case 128 frequencies in one call", flush=True)
    many = R.trace_maps([m], freqs, im, prm, info=False, stats=False)["tb"]
    for k in (0, 37, 127):
        one = R.trace_maps([m], [freqs[k]], im, prm, info=False, stats=False)["tb"]
        assert torch.equal(many[0, k], one[0, 0]), k
    print("case 16 models in one call", flush=True)
    m16 = R.trace_maps([m] * 16, [90e6, 300e6], im, prm, info=False, stats=False)["tb"]
    one = R.trace_maps([m], [90e6, 300e6], im, prm, info=False, stats=False)["tb"]
    for j in range(16):
        assert torch.equal(m16[j], one[0]), j
    with pytest.raises(R.RtError) as e:
        R.trace_maps([m] * 17, [90e6], im, prm, info=False, stats=False)
    assert e.value.status == 6
    with pytest.raises(R.RtError) as e:
        R.trace_maps([m], corona.log_freqs(129), im, prm, info=False, stats=False)
    assert e.value.status == 6


def test_graph_replay_equals_eager(R, structured_small):
    """A captured trace call replayed several times, with eager work and
    synchronizations between replays, gives the eager maps every time."""
    import torch
    cor, m = structured_small
    freqs = [60e6, 240e6]
    im = R.image_desc(48, 2.5)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    print("case graph replay", flush=True)
    eager = R.trace_maps([m], freqs, im, prm, info=False, stats=True)
    torch.cuda.synchronize()
    ref = eager["tb"].clone()
    ref_stats = R.decode_stats(eager["stats"])
    graph, out = R.capture_trace_maps([m], freqs, im, prm)
    for k in range(4):
        out["tb"].fill_(-1.0)
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["tb"], ref), k
        st = R.decode_stats(out["stats"])
        assert st["ray_steps"] == ref_stats["ray_steps"], k
        assert float(junk) == float(junk)


def test_graph_refuses_replay_after_its_model_is_closed(R):
    """A captured trace keeps its models; once one is closed (its device arrays
    freed), replay raises instead of launching kernels that would read them."""
    import torch
    cor = corona.spherically_symmetric()
    m = R.Model.from_corona(cor)
    print("case graph after model close", flush=True)
    cap, out = R.capture_trace_maps([m], [150e6], R.image_desc(16, 2.5), R.params())
    cap.replay()
    torch.cuda.synchronize()
    m.close()
    with pytest.raises(RuntimeError, match="closed"):
        cap.replay()


def test_graph_survives_larger_calls_on_its_stream(R, structured_small):
    """Calls larger than a captured one grow the library's tables of that
    stream; the outgrown tables are retired, not freed, so the graph's replays
    still read valid memory and give the eager maps bit for bit.  Larger calls
    on the default stream in between use that stream's own tables."""
    import torch
    cor, m = structured_small
    freqs = [80e6, 200e6]
    im = R.image_desc(24, 2.0)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    print("case graph vs larger calls", flush=True)
    eager = R.trace_maps([m], freqs, im, prm, info=False, stats=False)
    torch.cuda.synchronize()
    ref = eager["tb"].clone()
    cap, out = R.capture_trace_maps([m], freqs, im, prm)
    big_im = R.image_desc(72, 2.5)
    big_ref = None
    for k, on_graph_stream in enumerate((True, False, True)):
        s = cap.stream if on_graph_stream else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            big = R.trace_maps([m, m], freqs + [120e6], R.image_desc(72 + 16 * k, 2.5), prm, info=False,
                               stats=False)
        s.synchronize()
        if k == 0:
            big_ref = big["tb"].clone()
        torch.cuda.synchronize()
        out["tb"].fill_(-1.0)
        cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["tb"], ref), k
    again = R.trace_maps([m, m], freqs + [120e6], big_im, prm, info=False, stats=False)
    torch.cuda.synchronize()
    assert torch.equal(again["tb"], big_ref)
