"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them ray for ray."""
from __future__ import annotations

import math

import numpy as np

import oracle
import paper_1803_00430_amd as P

HIST_TOL = 1e-4   # relative, per bin-band-coefficient row sum (and per cell, scaled by that row)
RT60_TOL = 0.01   # relative


def gpu_trace(scene, sources, listener, radius, *, n_rays_total, ray_begin=0, ray_end=None, max_bounces,
              sh_order, n_bins, bin_width_s, seed, pair_base=0, want_hash=True, waves_per_cu=0):
    import torch
    if ray_end is None:
        ray_end = n_rays_total
    srcs = np.atleast_2d(np.asarray(sources, np.float32))
    nb = scene.n_bands
    hist, late, stats, rh = P.alloc_trace_outputs(len(srcs), n_bins, nb, sh_order, ray_end - ray_begin,
                                                  want_hash=want_hash)
    prm = P.trace_params(n_rays_total=n_rays_total, ray_begin=ray_begin, ray_end=ray_end,
                         max_bounces=max_bounces, sh_order=sh_order, n_bins=n_bins, bin_width_s=bin_width_s,
                         seed=seed, pair_base=pair_base, waves_per_cu=waves_per_cu)
    P.trace_ir(scene, srcs, listener, radius, prm, hist, late, stats, rh)
    torch.cuda.synchronize()
    return dict(hist=hist.double().cpu().numpy(), hist_late=late.double().cpu().numpy(),
                stats=P.stats_host(stats), ray_hash=None if rh is None else rh.cpu().numpy().view(np.uint32),
                _dev=(hist, late, stats))


def f32(x):
    """The value the C ABI carries for a scalar parameter (FP32)."""
    return float(np.float32(x))


def oracle_kw(kw):
    """Oracle arguments for the same inputs as the HIP path: the ABI passes the
    bin width as FP32, so the oracle gets that FP32 value (exact in FP64)."""
    o = {k: v for k, v in kw.items() if k not in ("want_hash", "waves_per_cu")}
    if "bin_width_s" in o:
        o["bin_width_s"] = f32(o["bin_width_s"])
    return o


def orc_trace(sd, sources, listener, radius, **kw):
    return oracle.trace_ir(sd, sources, listener, f32(radius), want_hash=True, **oracle_kw(kw))


def _stats_vec(st, nb):
    """Comparable stats of one IR as floats (GPU structured row or oracle dict)."""
    if isinstance(st, dict):
        g = lambda k: st[k]
    else:
        g = lambda k: st[k]
    return dict(
        n_segments=float(g("n_segments")), n_finite_segments=float(g("n_finite_segments")),
        n_escaped=float(g("n_escaped")), n_rays=float(g("n_rays")), seg_len_sum=float(g("seg_len_sum")),
        e_emitted=float(g("e_emitted")),
        e_class=np.asarray(g("e_class"))[:, :nb].astype(np.float64),
        e_escaped=np.asarray(g("e_escaped"))[:nb].astype(np.float64),
        e_alive_at_stop=np.asarray(g("e_alive_at_stop"))[:nb].astype(np.float64),
        e_alive_at_bounce_cap=np.asarray(g("e_alive_at_bounce_cap"))[:nb].astype(np.float64),
        e_absorbed=np.asarray(g("e_absorbed"))[:nb].astype(np.float64),
        first_arrival_bin=int(g("first_arrival_bin")), first_late_bin=int(g("first_late_bin")),
    )


def _removed_totals(side, one, s, nb):
    """Add ray `one`'s class energies (per class and band) to side[s]."""
    side[s] = side[s] + np.asarray(one["stats"][0]["e_class"])[:, :nb]


def traced_pair(scene, sd, sources, listener, radius, **kw):
    """Trace on both sides; rays whose discrete path (hit triangles and bounce
    kinds) differs between the HIP path and the oracle are traced again one
    by one on both sides and removed from both results.  Returns (gpu,
    oracle, divergent); gpu["removed"] and oracle["removed"] hold the class
    energies [source][class][band] of the removed rays on each side, and
    gpu["removed_sq"] their per-ray squares summed (for a Monte Carlo bound,
    see assert_removed_close)."""
    g = gpu_trace(scene, sources, listener, radius, **kw)
    o = orc_trace(sd, sources, listener, radius, **kw)
    srcs = np.atleast_2d(np.asarray(sources, np.float32))
    nb = scene.n_bands
    S = len(srcs)
    gs = [_stats_vec(g["stats"][s], nb) for s in range(S)]
    os_ = [_stats_vec(o["stats"][s], nb) for s in range(S)]
    div = np.argwhere(g["ray_hash"] != o["ray_hash"])
    rb = kw.get("ray_begin", 0)
    rem_g = [np.zeros((3, nb)) for _ in range(S)]
    rem_o = [np.zeros((3, nb)) for _ in range(S)]
    rem_sq = [np.zeros((3, nb)) for _ in range(S)]
    for (s, i) in div:
        one = dict(kw, ray_begin=rb + int(i), ray_end=rb + int(i) + 1, pair_base=kw.get("pair_base", 0) + int(s))
        g1 = gpu_trace(scene, srcs[s:s + 1], listener, radius, **one)
        o1 = orc_trace(sd, srcs[s:s + 1], listener, radius, **one)
        g["hist"][s] -= g1["hist"][0]
        g["hist_late"][s] -= g1["hist_late"][0]
        o["hist"][s] -= o1["hist"][0]
        o["hist_late"][s] -= o1["hist_late"][0]
        _removed_totals(rem_g, g1, s, nb)
        _removed_totals(rem_o, o1, s, nb)
        eg = np.asarray(g1["stats"][0]["e_class"])[:, :nb]
        eo = np.asarray(o1["stats"][0]["e_class"])[:, :nb]
        rem_sq[s] = rem_sq[s] + eg ** 2 + eo ** 2
        for side, one_res in ((gs, g1["stats"][0]), (os_, o1["stats"][0])):
            v1 = _stats_vec(one_res, nb)
            for key in ("n_segments", "n_finite_segments", "n_escaped", "n_rays", "seg_len_sum", "e_emitted",
                        "e_class", "e_escaped", "e_alive_at_stop", "e_alive_at_bounce_cap", "e_absorbed"):
                side[s][key] = side[s][key] - v1[key]
    g["cmp_stats"] = gs
    o["cmp_stats"] = os_
    g["removed"], o["removed"], g["removed_sq"] = rem_g, rem_o, rem_sq
    print(f"[parity] {len(div)} of {g['ray_hash'].size} rays took another discrete path on the two sides")
    return g, o, div


def assert_removed_close(g, o, sigmas=5.0):
    """The rays removed from the comparison (a different discrete path on the
    two sides) are two independent-looking samples of the same estimator:
    their summed class energies agree within `sigmas` Monte Carlo standard
    deviations, estimated from the removed rays' own contributions."""
    for s in range(len(g["removed"])):
        d = np.abs(g["removed"][s] - o["removed"][s])
        sd = np.sqrt(g["removed_sq"][s])
        assert np.all(d <= sigmas * sd + 1e-300), (s, d, sd)


def assert_hist_close(Hg, Ho, tol=HIST_TOL, what="hist", time_rel=0.0):
    """Row sums over bins agree within tol of sum|H_oracle|, and every cell
    within tol of that same absolute row sum.

    time_rel > 0 (for [T][B][NC] histograms of long FP32 paths): a cell may
    also differ by the energy that a relative path-length error of time_rel
    moves across its two bin edges, time_rel * t_m / dt * 2 * (the largest
    |H_oracle| among the cell and its two neighbours in time), t_m the end of
    bin m.  An FP32 path that keeps its discrete twin's hit sequence still
    drifts continuously from it; where one ray carries most of a row, the
    drift of its arrival time shows up at the 1e-4 level of that row, while
    a deposit in the wrong bin would still miss by a whole bin's energy."""
    Hg = np.asarray(Hg, np.float64)
    Ho = np.asarray(Ho, np.float64)
    assert Hg.shape == Ho.shape
    row_abs = np.abs(Ho).sum(axis=0)
    floor = 1e-30
    dr = np.abs(Hg.sum(0) - Ho.sum(0))
    assert np.all(dr <= tol * row_abs + floor), f"{what}: row-sum error {np.max(dr / (row_abs + floor)):.3e}"
    allow = tol * row_abs[None] + floor
    if time_rel > 0:
        a = np.abs(Ho)
        near = a.copy()
        near[1:] = np.maximum(near[1:], a[:-1])
        near[:-1] = np.maximum(near[:-1], a[1:])
        T = Ho.shape[0]
        t_end = np.arange(1, T + 1, dtype=np.float64).reshape((T,) + (1,) * (Ho.ndim - 1))  # in bins
        allow = allow + time_rel * t_end * 2.0 * near
    dc = np.abs(Hg - Ho)
    assert np.all(dc <= allow), f"{what}: cell error {np.max(dc / (row_abs[None] + floor)):.3e} of the row"


def assert_stats_close(sg, so, rel=1e-5):
    for k in ("n_segments", "n_finite_segments", "n_escaped", "n_rays"):
        assert abs(sg[k] - so[k]) <= max(1.0, 1e-5 * so[k]), (k, sg[k], so[k])
    for k in ("seg_len_sum", "e_emitted"):
        assert abs(sg[k] - so[k]) <= rel * abs(so[k]) + 1e-12, (k, sg[k], so[k])
    for k in ("e_escaped", "e_alive_at_stop", "e_alive_at_bounce_cap", "e_absorbed"):
        scale = max(np.abs(so[k]).max(), so["e_emitted"] * 1e-9)
        assert np.all(np.abs(sg[k] - so[k]) <= 1e-4 * scale + 1e-15), (k, sg[k], so[k])
    scale = np.abs(so["e_class"]).max(axis=0) + 1e-30
    assert np.all(np.abs(sg["e_class"] - so["e_class"]) <= HIST_TOL * scale[None]), (sg["e_class"], so["e_class"])


def gpu_trace_listener(scene, sources, listener, radius, *, n_rays_total, ray_begin=0, ray_end=None, max_bounces,
                       sh_order, n_bins, bin_width_s, seed, pair_base=0, want_hash=True):
    import torch
    if ray_end is None:
        ray_end = n_rays_total
    srcs = np.atleast_2d(np.asarray(sources, np.float32))
    nb = scene.n_bands
    hist, late, stats, _ = P.alloc_trace_outputs(len(srcs), n_bins, nb, sh_order)
    rh = torch.empty(ray_end - ray_begin, dtype=torch.int32, device="cuda") if want_hash else None
    prm = P.trace_params(n_rays_total=n_rays_total, ray_begin=ray_begin, ray_end=ray_end,
                         max_bounces=max_bounces, sh_order=sh_order, n_bins=n_bins, bin_width_s=bin_width_s,
                         seed=seed, pair_base=pair_base)
    P.trace_listener(scene, srcs, listener, radius, prm, hist, late, stats, rh)
    torch.cuda.synchronize()
    return dict(hist=hist.double().cpu().numpy(), hist_late=late.double().cpu().numpy(),
                stats=P.stats_host(stats), ray_hash=None if rh is None else rh.cpu().numpy().view(np.uint32),
                _dev=(hist, late, stats))


_RAYSET_KEYS = ("n_segments", "n_finite_segments", "n_escaped", "n_rays", "seg_len_sum", "e_emitted",
                "e_escaped", "e_alive_at_stop", "e_alive_at_bounce_cap", "e_absorbed")


def traced_listener_pair(scene, sd, sources, listener, radius, **kw):
    """trace_listener on both sides; rays whose discrete path (hit
    triangles, bounce kinds, occlusion outcomes) differs are traced again
    alone on both sides and removed from every source's result.  Returns
    (gpu, oracle, divergent ray indices)."""
    g = gpu_trace_listener(scene, sources, listener, radius, **kw)
    o = oracle.trace_listener(sd, sources, listener, f32(radius), want_hash=True, **oracle_kw(kw))
    srcs = np.atleast_2d(np.asarray(sources, np.float32))
    nb = scene.n_bands
    S = len(srcs)
    gs = [_stats_vec(g["stats"][s], nb) for s in range(S)]
    os_ = [_stats_vec(o["stats"][s], nb) for s in range(S)]
    div = np.flatnonzero(g["ray_hash"] != o["ray_hash"])
    print(f"[parity] {len(div)} of {g['ray_hash'].size} listener rays took another discrete path on the two sides")
    rb = kw.get("ray_begin", 0)
    for i in div:
        one = dict(kw, ray_begin=rb + int(i), ray_end=rb + int(i) + 1)
        g1 = gpu_trace_listener(scene, srcs, listener, radius, **one)
        o1 = oracle.trace_listener(sd, srcs, listener, f32(radius), **oracle_kw(one))
        for s in range(S):
            g["hist"][s] -= g1["hist"][s]
            g["hist_late"][s] -= g1["hist_late"][s]
            o["hist"][s] -= o1["hist"][s]
            o["hist_late"][s] -= o1["hist_late"][s]
            for side, res in ((gs, g1["stats"][s]), (os_, o1["stats"][s])):
                v1 = _stats_vec(res, nb)
                for key in _RAYSET_KEYS + ("e_class",):
                    side[s][key] = side[s][key] - v1[key]
    g["cmp_stats"] = gs
    o["cmp_stats"] = os_
    return g, o, div
