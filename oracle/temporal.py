"""Temporal coherence across frames, FP64 numpy (Section 4.2, Eq. 4; Section 5,
the early- and late-reflection caches with tau_ER = 1 s and tau_LR = 3 s).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library,
with which it shares no code.

Readings (the paper gives Eq. 4 and the two time constants, not the factor):
  * the smoothing factor of a frame of length dt is alpha = 1 - exp(-dt / tau),
    so that after n frames of a constant new value the cache has covered
    1 - exp(-n dt / tau) of the step; tau <= 0 means no smoothing (alpha = 1);
  * the first frame, or a reset, takes the new value as it is;
  * the IR cache is the same exponential smoothing applied to every histogram
    cell: the all-orders histogram with tau_ER, the late (orders >= 3)
    histogram with tau_LR;
  * Eq. 4 smooths the RT60 of every band with tau_LR; a frame whose estimate
    is invalid (status NO_ENERGY, BAD_FIT or NO_RANGE) leaves the cached value
    as it was; E_direct and E_early are smoothed with tau_ER, E_late with
    tau_LR, and g_reverb is recomputed from the smoothed E_late and RT60
    (Eq. 5 with Eq. 8); the other parameters are the frame's own.

Parity pins: tests/test_oracle_temporal.py (exact step response, fixed points,
the variance of smoothed independent noise, the invalid-frame rule).
"""
from __future__ import annotations

import math

import numpy as np

ST_NO_ENERGY = 1
ST_BAD_FIT = 2
ST_NO_RANGE = 4
INVALID = ST_NO_ENERGY | ST_BAD_FIT | ST_NO_RANGE
LN10_6 = 6.0 * math.log(10.0)


def smoothing_alpha(frame_dt: float, tau: float) -> float:
    """alpha = 1 - exp(-dt / tau); 1 when tau <= 0."""
    if tau <= 0.0:
        return 1.0
    return 1.0 - math.exp(-frame_dt / tau)


def ema(cache, fresh, alpha: float, first: bool):
    """One frame of exponential smoothing: alpha * fresh + (1 - alpha) * cache
    (fresh itself on the first frame)."""
    fresh = np.asarray(fresh, np.float64)
    if first:
        return fresh.copy()
    return alpha * fresh + (1.0 - alpha) * np.asarray(cache, np.float64)


def smooth_params(cached: dict | None, fresh: dict, alpha_early: float, alpha_late: float, n_bands: int) -> dict:
    """Eq. 4 and the energy smoothing for one IR.  `fresh` and `cached` hold
    rt60, status, e_direct, e_early, e_late (per band) and the frame's other
    parameters; returns the new cached (= output) parameters."""
    B = n_bands
    out = {k: (np.array(v, np.float64, copy=True) if isinstance(v, (list, np.ndarray)) else v)
           for k, v in fresh.items()}
    if cached is None:
        return out
    valid = (np.asarray(fresh["status"][:B]) & INVALID) == 0
    prev_valid = np.asarray(cached["rt60"][:B], np.float64) > 0
    rt_f = np.asarray(fresh["rt60"][:B], np.float64)
    rt_c = np.asarray(cached["rt60"][:B], np.float64)
    rt = np.where(valid & prev_valid, alpha_late * rt_f + (1 - alpha_late) * rt_c,
                  np.where(valid, rt_f, rt_c))
    out["rt60"] = rt
    # the status and fit range belong to the frame whose RT60 was taken in
    out["status"] = np.where(valid, np.asarray(fresh["status"][:B]), np.asarray(cached["status"][:B]))
    out["rt60_range"] = np.where(valid, np.asarray(fresh["rt60_range"][:B]), np.asarray(cached["rt60_range"][:B]))
    for key, a in (("e_direct", alpha_early), ("e_early", alpha_early), ("e_late", alpha_late)):
        out[key] = a * np.asarray(fresh[key][:B], np.float64) + (1 - a) * np.asarray(cached[key][:B], np.float64)
    g = np.zeros(B)
    ok = rt > 0
    g[ok] = np.sqrt(out["e_late"][ok] * LN10_6 / rt[ok])
    out["g_reverb"] = g
    return out
