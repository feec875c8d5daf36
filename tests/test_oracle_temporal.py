"""Pins of the oracle's temporal smoothing (Eq. 4 and the IR caches) against
closed forms: the smoothing factor's time constant, the exact step response,
fixed points, the variance of smoothed independent noise, and the
invalid-frame and Eq. 5/8 rules of the parameter smoothing.  CPU-only."""
import math

import numpy as np

from oracle import temporal as TC


def test_smoothing_factor_time_constant():
    assert TC.smoothing_alpha(0.1, 0.0) == 1.0 and TC.smoothing_alpha(0.1, -1.0) == 1.0
    for dt, tau in ((0.1, 1.0), (0.1, 3.0), (0.02, 0.5)):
        a = TC.smoothing_alpha(dt, tau)
        assert 0 < a < 1
        # n frames of a unit step cover 1 - exp(-n dt / tau) of it
        c = TC.ema(None, np.zeros(3), a, first=True)
        for n in range(1, 61):
            c = TC.ema(c, np.ones(3), a, first=False)
            assert np.allclose(c, 1 - math.exp(-n * dt / tau), rtol=0, atol=1e-12)
    assert TC.smoothing_alpha(0.1, 1.0) > TC.smoothing_alpha(0.1, 3.0)


def test_constant_input_is_a_fixed_point_and_first_frame_copies():
    x = np.random.default_rng(0).normal(size=(50, 4, 16))
    c = TC.ema(np.full_like(x, 123.0), x, 0.3, first=True)
    assert np.array_equal(c, x)
    for _ in range(20):
        c = TC.ema(c, x, 0.3, first=False)
    assert np.allclose(c, x, rtol=1e-14, atol=1e-14)


def test_smoothed_independent_noise_has_variance_alpha_over_2_minus_alpha():
    """Stationary variance of y_n = a x_n + (1-a) y_{n-1} for i.i.d. unit
    variance x: a^2 / (1 - (1-a)^2) = a / (2 - a)."""
    g = np.random.default_rng(1)
    for a in (TC.smoothing_alpha(0.1, 1.0), TC.smoothing_alpha(0.1, 3.0)):
        x = g.normal(size=(400, 2000))
        y = TC.ema(None, x[0], a, first=True)
        ys = []
        for n in range(1, 400):
            y = TC.ema(y, x[n], a, first=False)
            if n >= 200:
                ys.append(y)
        v = np.var(np.array(ys)[::25], axis=1).mean()  # frames 25 apart are nearly independent
        assert abs(v / (a / (2 - a)) - 1) < 0.03, (a, v)


def _fresh(rt, st, el, ed=(1e-3,) * 4, ee=(2e-3,) * 4, rng=(0,) * 4):
    return dict(rt60=np.array(rt, float), status=np.array(st), rt60_range=np.array(rng),
                e_direct=np.array(ed, float), e_early=np.array(ee, float), e_late=np.array(el, float),
                predelay_s=0.01)


def test_parameter_smoothing_rules():
    aE, aL = TC.smoothing_alpha(0.1, 1.0), TC.smoothing_alpha(0.1, 3.0)
    f1 = _fresh([1.0, 2.0, 0.0, 0.5], [0, 0, TC.ST_NO_ENERGY, 0], [1e-2, 2e-2, 0.0, 4e-3], rng=(0, 1, -1, 2))
    c = TC.smooth_params(None, f1, aE, aL, 4)
    assert np.array_equal(c["rt60"], f1["rt60"])  # the first frame is taken as it is
    f2 = _fresh([2.0, 0.0, 3.0, 0.7], [0, TC.ST_BAD_FIT, 0, 0], [2e-2, 2e-2, 1e-2, 4e-3], rng=(1, -1, 0, 0))
    c2 = TC.smooth_params(c, f2, aE, aL, 4)
    # Eq. 4 where both frames are valid; an invalid frame keeps the cache;
    # a valid frame after an invalid cache starts it
    assert math.isclose(c2["rt60"][0], aL * 2.0 + (1 - aL) * 1.0, rel_tol=1e-15)
    assert c2["rt60"][1] == 2.0 and c2["rt60_range"][1] == 1
    assert c2["rt60"][2] == 3.0 and c2["rt60_range"][2] == 0
    assert math.isclose(c2["rt60"][3], aL * 0.7 + (1 - aL) * 0.5, rel_tol=1e-15)
    assert np.allclose(c2["e_late"], aL * f2["e_late"] + (1 - aL) * f1["e_late"], rtol=1e-15)
    assert np.allclose(c2["e_direct"], f1["e_direct"], rtol=1e-15)  # equal frames stay
    # Eq. 5 with Eq. 8 on the smoothed values
    assert np.allclose(c2["g_reverb"], np.sqrt(c2["e_late"] * 6 * math.log(10) / c2["rt60"]), rtol=1e-15)
    assert c2["predelay_s"] == 0.01
