"""Stored oracle values (tests/golden/oracle_c0.json, written by
tests/golden/make_golden.py, which calls only the oracle): the oracle still
reproduces them (CPU), and the GPU path matches them at the parity bar."""
import json
import os

import numpy as np
import pytest

from paper_2606_02413_amd import corona
from tests import parity_util as PU

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_c0.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_oracle_reproduces_its_stored_values(orc):
    doc = _load()
    cor = corona.spherically_symmetric()
    med = orc.OracleMedium.from_corona(cor)
    P = orc.make_params(ds_max=doc["ds_max"], n_floor=doc["n_floor"])
    im = orc.make_image(doc["n_pix"], doc["half_width"])
    for st in doc["sets"]:
        pix = np.array([r["pixel"] for r in st["rays"]], dtype=np.int32)
        res = orc.trace_pixels(med, P, im, st["freq_hz"], pix)
        for r, g in zip(res, st["rays"]):
            assert int(r["code"]) == g["code"] and int(r["n_steps"]) == g["n_steps"]
            for key in ("tb", "tau", "ln_s_end"):
                assert abs(float(r[key]) - g[key]) <= 1e-10 * max(abs(g[key]), 1.0), (g["pixel"], key)
            assert np.max(np.abs(np.asarray(r["exit_pos"]) - np.asarray(g["exit_pos"]))) <= 1e-12


@pytest.mark.gpu
def test_gpu_matches_the_stored_values():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun as R
    doc = _load()
    m = R.Model.from_corona(corona.spherically_symmetric())
    kw = PU.step_kwargs(doc["ds_max"], doc["n_floor"])
    print("case golden", flush=True)
    for st in doc["sets"]:
        g = PU.gpu_trace([m], [st["freq_hz"]], doc["n_pix"], doc["half_width"], kw)
        tb, info = g["tb"].reshape(-1), g["info"].reshape(-1)
        for r in st["rays"]:
            p = r["pixel"]
            assert int(info["code"][p]) == r["code"] and int(info["n_steps"][p]) == r["n_steps"], p
            if r["flags"]:
                continue
            assert abs(float(tb[p]) - r["tb"]) <= PU.TB_REL_TOL * max(r["tb"], PU.TB_FLOOR), p
            assert np.linalg.norm(info["exit_pos"][p].astype(np.float64) - np.asarray(r["exit_pos"])) <= PU.EXIT_TOL, p
    m.close()
