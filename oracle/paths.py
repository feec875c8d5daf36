"""Early-reflection paths: their records from the trace, the diffuse path
cache across frames and the prioritization for rendering, FP64 (Section 5:
the first two reflection orders with the diffuse path cache, augmented with
SH directivity per path; paths below the threshold of hearing discarded, the
N_ER = 100 strongest among all sources rendered, the rest added to the late
IR before it is analysed).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library,
with which it shares no code.

Readings (the paper gives the steps, not these details):
  * a path is identified by (source, reflection order, triangle of the first
    reflection, triangle of the second); every deposit of an order-1 or
    order-2 segment at the listener sphere is one record of its path: the
    band intensity the histogram received within the window, the midpoint of
    the chord's arrival-time interval clipped to the window, and the SH
    directivity e_total Y(arrival direction);
  * a frame's paths sum their records' intensities and directivities, and
    carry the intensity-weighted arrival time (kept as the sum of
    e_total * t);
  * the cache (temporal coherence of the early reflections with tau_ER):
    P <- (1 - alpha) P + alpha F per path, F = the frame's path (0 when
    absent), alpha = 1 - exp(-dt / tau_ER); a path whose total intensity
    falls below min_energy leaves the cache; the first frame takes F;
  * prioritization: paths with total intensity (sum over bands) below the
    threshold are discarded; the others are ranked by decreasing intensity
    over all sources (ties by key); the first N_ER are rendered; the rest
    join the late class: their band intensity moves from the early class
    (e_class[1]) to the late one (e_class[2]) and is added to the late
    histogram of their source at the bin of their mean arrival time.

Parity pins: tests/test_oracle_paths.py.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import IrStats, TraceParams, _dp, lib, stats_to_dict, SPEED_OF_SOUND

REC_W, REC_E, REC_T, REC_D = 29, 4, 12, 13


def trace_paths(scene, sources, listener, radius, *, n_rays_total, ray_begin=0, ray_end=None, max_bounces,
                sh_order, n_bins, bin_width_s, seed, pair_base=0, speed_of_sound=SPEED_OF_SOUND):
    """The FP64 trace with its path records: dict(hist, hist_late, stats,
    records [S, R, 2, 29])."""
    if ray_end is None:
        ray_end = n_rays_total
    verts = np.ascontiguousarray(scene["verts"], np.float64)
    tris = np.ascontiguousarray(scene["tris"], np.int32)
    tri_mat = np.ascontiguousarray(scene["tri_mat"], np.int32)
    ab = np.ascontiguousarray(scene["absorption"], np.float64)
    sc = np.ascontiguousarray(scene["scattering"], np.float64)
    M, B = ab.shape
    srcs = np.ascontiguousarray(np.atleast_2d(sources), np.float64)
    S = len(srcs)
    lst = np.ascontiguousarray([*np.asarray(listener, np.float64), float(radius)], np.float64)
    nc = (sh_order + 1) ** 2
    R = ray_end - ray_begin
    hist = np.zeros((S, n_bins, B, nc))
    hist_late = np.zeros((S, n_bins, B))
    stats = (IrStats * max(S, 1))()
    rec = np.zeros((S, max(R, 0), 2, REC_W))
    p = TraceParams(n_rays_total, ray_begin, ray_end, max_bounces, sh_order, n_bins, pair_base,
                    bin_width_s, speed_of_sound, seed)
    rc = lib().orc_trace_ir_paths(_dp(verts), len(verts), tris.ctypes.data_as(C.POINTER(C.c_int32)), len(tris),
                                  tri_mat.ctypes.data_as(C.POINTER(C.c_int32)), _dp(ab), _dp(sc), M, B,
                                  _dp(srcs), S, _dp(lst), C.byref(p), _dp(hist), _dp(hist_late), stats, _dp(rec))
    if rc != 0:
        raise ValueError("oracle trace_paths: invalid arguments")
    return dict(hist=hist, hist_late=hist_late, stats=[stats_to_dict(stats[s], B) for s in range(S)], records=rec)


def aggregate(records, n_bands, n_coeffs):
    """Paths of one frame: {(source, order, tri1, tri2): dict(e [B], et, d [NC])},
    each the sum of its records (et: the sum of e_total * t)."""
    rec = np.asarray(records, np.float64)
    S = rec.shape[0]
    src = np.broadcast_to(np.arange(S)[:, None, None], rec.shape[:3])
    ok = rec[..., 0] == 1.0
    x, s = rec[ok], src[ok]
    keys = np.stack([s, x[:, 1].astype(np.int64), x[:, 2].astype(np.int64), x[:, 3].astype(np.int64)], axis=1)
    if len(keys) == 0:
        return {}
    uk, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    e = np.zeros((len(uk), n_bands))
    et = np.zeros(len(uk))
    d = np.zeros((len(uk), n_coeffs))
    ev = x[:, REC_E:REC_E + n_bands]
    np.add.at(e, inv, ev)
    np.add.at(et, inv, ev.sum(axis=1) * x[:, REC_T])
    np.add.at(d, inv, x[:, REC_D:REC_D + n_coeffs])
    return {tuple(int(v) for v in uk[i]): dict(e=e[i], et=float(et[i]), d=d[i]) for i in range(len(uk))}


def cache_update(cache, fresh, alpha, min_energy, first):
    """One frame of the path cache."""
    if first or cache is None:
        merged = {k: dict(e=v["e"].copy(), et=v["et"], d=v["d"].copy()) for k, v in fresh.items()}
    else:
        merged = {}
        for k in set(cache) | set(fresh):
            c, f = cache.get(k), fresh.get(k)
            tmpl = c if c is not None else f
            e = np.zeros_like(tmpl["e"])
            et = 0.0
            d = np.zeros_like(tmpl["d"])
            if c is not None:
                e += (1 - alpha) * c["e"]
                et += (1 - alpha) * c["et"]
                d += (1 - alpha) * c["d"]
            if f is not None:
                e += alpha * f["e"]
                et += alpha * f["et"]
                d += alpha * f["d"]
            merged[k] = dict(e=e, et=et, d=d)
    return {k: v for k, v in merged.items() if v["e"].sum() >= min_energy}


def select(paths, threshold, n_er, hist_late, e_class, bin_width_s):
    """Prioritization.  hist_late [S][T][B] and e_class [S][3][B] are updated
    in place with the culled paths; returns the rendered paths, strongest
    first, as a list of (key, path)."""
    items = [(k, v) for k, v in paths.items() if v["e"].sum() >= threshold]
    items.sort(key=lambda kv: (-kv[1]["e"].sum(), kv[0]))
    T = hist_late.shape[1]
    for k, v in items[n_er:]:
        s = k[0]
        et = v["e"].sum()
        m = min(int(np.floor(v["et"] / et / bin_width_s)), T - 1) if et > 0 else 0
        hist_late[s, m] += v["e"]
        e_class[s][1] -= v["e"]
        e_class[s][2] += v["e"]
    return items[:n_er]
