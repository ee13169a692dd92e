"""Pins of the oracle's carried ray tube (two neighbour rays kept along the
whole ray): in a quadratic lens the neighbours are transverse harmonic
oscillators, so the RK4 tube area follows the powers of the RK4 propagator of
x'' = -beta x exactly; in a uniform medium the tube does not change; in a
Baumbach-Allen corona the carried ln S at the end of a ray tends to a finite
value as the step shrinks, while the step-wise estimate of Eqs. 5-11 is
proportional to the step."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def xf_of(f):
    return (8.98e3 / f) ** 2


@pytest.mark.parametrize("h", [0.05, 0.01])
def test_carried_tube_in_a_quadratic_lens(h):
    beta, f = 4.0, 100e6
    med = O.OracleMedium(O.ANALYTIC_LENS, r_in=-1.0, r_max=3.0, a0=beta / xf_of(f))
    P = O.make_params(ds_max=h, n_floor=1.0, carried_tube=True)
    res, path = O.trace_launch_path(med, P, f, [0, 0, -2.0], [0, 0, 1.0])
    # RK4 propagator of (x, p_x) for x'' = -beta x over one step h
    L = np.array([[0.0, 1.0], [-beta, 0.0]]) * h
    A = np.eye(2) + L + L @ L / 2 + L @ L @ L / 6 + L @ L @ L @ L / 24
    y = np.array([1.0, 0.0])
    want = []
    for _ in range(len(path)):
        y1 = A @ y
        want.append(2.0 * math.log(abs(y1[0] / y[0])))   # S = x^2 (the two neighbours alike)
        y = y1
    want = np.array(want)
    ok = np.abs(np.cumsum(want)) < 20          # stop before a caustic of the tube
    assert np.max(np.abs(path[:-1, 4][ok[:-1]] - want[:-1][ok[:-1]])) < 1e-9
    # continuum: S / S_0 = cos^2(sqrt(beta) t) at the first step points
    t = h * np.arange(1, 6)
    assert np.max(np.abs(np.cumsum(path[:5, 4]) - 2 * np.log(np.abs(np.cos(math.sqrt(beta) * t))))) < 5 * h ** 4
    # the smallest ln(S/S_0) over the step points (the last chord truncated at
    # the sphere): the tube is squeezed towards the focus at sqrt(beta) t = pi/2
    cum = np.cumsum(path[:, 4])
    cum[-1] = cum[-2] + res["lam_last"] * path[-1, 4]
    assert abs(res["ln_s_min"] - min(0.0, cum.min())) < 1e-9
    assert res["ln_s_min"] < 2 * math.log(abs(math.cos(math.sqrt(beta) * h * (int(math.pi / 2 / math.sqrt(beta) / h))))) + 1e-6


def test_carried_tube_is_constant_in_a_uniform_medium():
    med = O.OracleMedium(O.ANALYTIC_UNIFORM, r_in=-1.0, r_max=3.0, a0=2e7, t_const=1e6)
    P = O.make_params(ds_max=0.01, n_floor=0.1, carried_tube=True)
    res, path = O.trace_launch_path(med, P, 150e6, [2.9, 0.3, 0.2], [-1.0, 0.0, 0.0])
    assert np.max(np.abs(path[:, 4])) < 1e-12 and abs(res["ln_s_end"]) < 1e-10
    assert -1e-10 < res["ln_s_min"] <= 0.0


def test_carried_tube_converges_with_the_step_and_the_stepwise_area_does_not():
    med = O.OracleMedium(O.ANALYTIC_BA, r_in=1.0, r_max=3.0, t_const=1e6)
    r0, d = [[math.sqrt(9 - 1.3 ** 2), 0.0, 1.3]], [[-1.0, 0.0, 0.0]]
    carried, stepwise = [], []
    for h in (0.02, 0.01, 0.005):
        for flag, dst in ((True, carried), (False, stepwise)):
            P = O.make_params(ds_max=h, n_floor=1e-3, carried_tube=flag)
            dst.append(float(O.trace_launch(med, P, 80e6, np.array(r0), np.array(d))["ln_s_end"][0]))
    print("carried", carried, "step-wise", stepwise)
    # step-wise: proportional to the step
    assert abs(stepwise[0] / stepwise[1] - 2.0) < 0.02 and abs(stepwise[1] / stepwise[2] - 2.0) < 0.02
    # carried: a finite limit (ln S_end ~ 1.7 for this ray), approached at first
    # order only through the last, truncated step (its ln M is scaled by lambda)
    d1, d2 = abs(carried[0] - carried[1]), abs(carried[1] - carried[2])
    assert abs(carried[2]) > 1.0 and d2 < 1e-4 * abs(carried[2]) and d2 < 0.6 * d1
