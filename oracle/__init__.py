"""CPU FP64 oracle for ray-parameterized reverberation (arXiv 1803.00430).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the HIP path (`paper_1803_00430_amd`), and neither imports the other.

Contents
  * ctypes wrapper of `rpr_oracle.c` (Philox4x32-10, real SH, brute-force
    closest hit, the stochastic tracer with the listener-sphere deposit);
  * `estimate_reverb`: the reverberation-parameter estimation of Section 4.2
    in numpy FP64 (Schroeder backward integration and least squares for RT60,
    Eq. 5-8 for the reverb gain, the predelay, the mean free path and the
    energy-weighted directivity of Eq. 1);
  * `oracle.mlp` (its own module): FP64 featurisation, forward / backward of
    the learned estimator's MLP, its Gaussian negative log-likelihood, Adam,
    and the decoding of the network output, for gradient checks.

Parity pins (what each function is checked against) are listed in the tests;
functions with none say "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "librpr_oracle.so")

MAX_BANDS = 8
INT32_MAX = 2**31 - 1
SPEED_OF_SOUND = 343.0


def build(force: bool = True) -> str:
    """Compile rpr_oracle.c with gcc (OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class TraceParams(C.Structure):
    _fields_ = [("n_rays_total", C.c_int64), ("ray_begin", C.c_int64), ("ray_end", C.c_int64),
                ("max_bounces", C.c_int32), ("sh_order", C.c_int32), ("n_bins", C.c_int32),
                ("pair_base", C.c_int32), ("bin_width_s", C.c_double),
                ("speed_of_sound", C.c_double), ("seed", C.c_uint64)]


class IrStats(C.Structure):
    _fields_ = [("n_segments", C.c_int64), ("n_finite_segments", C.c_int64),
                ("n_escaped", C.c_int64), ("n_rays", C.c_int64), ("seg_len_sum", C.c_double),
                ("e_emitted", C.c_double), ("first_arrival_bin", C.c_int32),
                ("first_late_bin", C.c_int32), ("e_class", (C.c_double * MAX_BANDS) * 3),
                ("e_escaped", C.c_double * MAX_BANDS), ("e_alive_at_stop", C.c_double * MAX_BANDS),
                ("e_alive_at_bounce_cap", C.c_double * MAX_BANDS),
                ("e_absorbed", C.c_double * MAX_BANDS), ("n_next_event", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_sh_eval.argtypes = [C.c_int, dp, dp]
        L.orc_emission_dir.argtypes = [dp, dp]
        L.orc_diffuse_dir.argtypes = [dp, dp, dp]
        L.orc_emission_batch.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, dp]
        L.orc_diffuse_batch.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, dp, C.c_int64, dp]
        L.orc_closest_hit_batch.argtypes = [dp, C.POINTER(C.c_int32), C.c_int64, dp, dp, C.c_int64,
                                            dp, C.POINTER(C.c_int64)]
        L.orc_trace_ir.argtypes = [dp, C.c_int64, C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int32),
                                   dp, dp, C.c_int32, C.c_int32, dp, C.c_int32, dp,
                                   C.POINTER(TraceParams), dp, dp, C.POINTER(IrStats),
                                   C.POINTER(C.c_uint32)]
        L.orc_trace_ir.restype = C.c_int
        L.orc_trace_ir_paths.argtypes = L.orc_trace_ir.argtypes[:-1] + [dp]
        L.orc_trace_ir_paths.restype = C.c_int
        L.orc_trace_listener.argtypes = L.orc_trace_ir.argtypes
        L.orc_trace_listener.restype = C.c_int
        L.orc_cone_dir.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_cone_batch.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, dp, C.c_double,
                                     C.c_int64, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_surface_offset.argtypes = [C.c_double]
        L.orc_get_surface_offset.restype = C.c_double
        L.orc_trace_path.argtypes = [dp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp, dp,
                                     C.c_int32, dp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_double,
                                     C.c_int32, dp, dp, dp, C.POINTER(C.c_int64)]
        L.orc_trace_path.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------- primitives

def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter under a 2-word key."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(x: int) -> float:
    return float(lib().orc_uniform(int(x) & 0xFFFFFFFF))


def sh_eval(order: int, dirs) -> np.ndarray:
    """Real SH of order <= `order` at each direction; [N, (order+1)^2]."""
    d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    nc = (order + 1) ** 2
    out = np.zeros((len(d), 16), np.float64)
    for i in range(len(d)):
        lib().orc_sh_eval(order, _dp(d[i]), _dp(out[i]))
    return out[:, :nc]


def emission_dir(u) -> np.ndarray:
    u = np.ascontiguousarray(u, np.float64)
    o = np.zeros(3)
    lib().orc_emission_dir(_dp(u), _dp(o))
    return o


def diffuse_dir(nf, u) -> np.ndarray:
    nf = np.ascontiguousarray(nf, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    o = np.zeros(3)
    lib().orc_diffuse_dir(_dp(nf), _dp(u), _dp(o))
    return o


def emission_batch(seed: int, pair: int, n: int) -> np.ndarray:
    """Emission directions of rays 0..n-1 of one pair, [n, 3]."""
    out = np.zeros((n, 3))
    lib().orc_emission_batch(seed, pair, n, _dp(out))
    return out


def diffuse_batch(seed: int, pair: int, order: int, nf, n: int) -> np.ndarray:
    """Diffuse bounce directions about nf for rays 0..n-1 at one order, [n, 3]."""
    nf = np.ascontiguousarray(nf, np.float64)
    out = np.zeros((n, 3))
    lib().orc_diffuse_batch(seed, pair, order, _dp(nf), n, _dp(out))
    return out


def closest_hit(verts, tris, orig, dirs):
    """Brute-force closest hit of each ray; returns (t [N], tri [N]) with
    t = inf and tri = -1 for misses."""
    v = np.ascontiguousarray(verts, np.float64)
    t = np.ascontiguousarray(tris, np.int32)
    o = np.ascontiguousarray(orig, np.float64)
    d = np.ascontiguousarray(dirs, np.float64)
    n = len(o)
    tout = np.zeros(n)
    iout = np.zeros(n, np.int64)
    lib().orc_closest_hit_batch(_dp(v), t.ctypes.data_as(C.POINTER(C.c_int32)), len(t), _dp(o), _dp(d), n,
                                _dp(tout), iout.ctypes.data_as(C.POINTER(C.c_int64)))
    return tout, iout


def stats_to_dict(st: IrStats, nb: int) -> dict:
    return dict(
        n_segments=int(st.n_segments), n_finite_segments=int(st.n_finite_segments),
        n_escaped=int(st.n_escaped), n_rays=int(st.n_rays), seg_len_sum=float(st.seg_len_sum),
        e_emitted=float(st.e_emitted), first_arrival_bin=int(st.first_arrival_bin),
        first_late_bin=int(st.first_late_bin),
        e_class=np.array([[st.e_class[c][b] for b in range(nb)] for c in range(3)]),
        e_escaped=np.array(st.e_escaped[:nb]), e_alive_at_stop=np.array(st.e_alive_at_stop[:nb]),
        e_alive_at_bounce_cap=np.array(st.e_alive_at_bounce_cap[:nb]),
        e_absorbed=np.array(st.e_absorbed[:nb]), n_next_event=int(st.n_next_event),
    )


class surface_offset:
    """Context manager: trace with the reflected segment's start `metres` off
    the surface instead of the 1 mm reading, then restore it.  For the tests
    that follow the oracle to the limit of a vanishing offset."""

    def __init__(self, metres: float):
        self.metres = float(metres)

    def __enter__(self):
        self.prev = lib().orc_get_surface_offset()
        lib().orc_set_surface_offset(self.metres)
        return self

    def __exit__(self, *exc):
        lib().orc_set_surface_offset(self.prev)
        return False


def trace_ir(scene, sources, listener, radius, *, n_rays_total, ray_begin=0, ray_end=None,
             max_bounces, sh_order, n_bins, bin_width_s, seed, pair_base=0,
             speed_of_sound=SPEED_OF_SOUND, want_hash=False):
    """Run the FP64 tracer.  Returns dict(hist [S,T,B,NC], hist_late [S,T,B],
    stats [list of dict], ray_hash [S,R] or None)."""
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
    rh = np.zeros((S, max(R, 0)), np.uint32) if want_hash else None
    p = TraceParams(n_rays_total, ray_begin, ray_end, max_bounces, sh_order, n_bins, pair_base,
                    bin_width_s, speed_of_sound, seed)
    rc = lib().orc_trace_ir(_dp(verts), len(verts), tris.ctypes.data_as(C.POINTER(C.c_int32)), len(tris),
                            tri_mat.ctypes.data_as(C.POINTER(C.c_int32)), _dp(ab), _dp(sc), M, B,
                            _dp(srcs), S, _dp(lst), C.byref(p), _dp(hist), _dp(hist_late), stats,
                            rh.ctypes.data_as(C.POINTER(C.c_uint32)) if rh is not None else None)
    if rc != 0:
        raise ValueError("oracle trace_ir: invalid arguments")
    return dict(hist=hist, hist_late=hist_late, stats=[stats_to_dict(stats[s], B) for s in range(S)],
                ray_hash=rh)


def trace_listener(scene, sources, listener, radius, *, n_rays_total, ray_begin=0, ray_end=None,
                   max_bounces, sh_order, n_bins, bin_width_s, seed, pair_base=0,
                   speed_of_sound=SPEED_OF_SOUND, want_hash=False):
    """Listener-origin trace with next-event estimation toward each source
    ball of radius `radius` (`orc_trace_listener`).  Returns dict(hist
    [S,T,B,NC], hist_late [S,T,B], stats [list of dict], ray_hash [R] or
    None)."""
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
    rh = np.zeros(max(R, 0), np.uint32) if want_hash else None
    p = TraceParams(n_rays_total, ray_begin, ray_end, max_bounces, sh_order, n_bins, pair_base,
                    bin_width_s, speed_of_sound, seed)
    rc = lib().orc_trace_listener(_dp(verts), len(verts), tris.ctypes.data_as(C.POINTER(C.c_int32)), len(tris),
                                  tri_mat.ctypes.data_as(C.POINTER(C.c_int32)), _dp(ab), _dp(sc), M, B,
                                  _dp(srcs), S, _dp(lst), C.byref(p), _dp(hist), _dp(hist_late), stats,
                                  rh.ctypes.data_as(C.POINTER(C.c_uint32)) if rh is not None else None)
    if rc != 0:
        raise ValueError("oracle trace_listener: invalid arguments")
    return dict(hist=hist, hist_late=hist_late, stats=[stats_to_dict(stats[s], B) for s in range(S)],
                ray_hash=rh)


def cone_batch(seed: int, pair: int, order: int, w3: int, axis, cos_half_angle: float, n: int) -> np.ndarray:
    """Directions uniform in a cone about `axis` from counters (i, pair,
    order, w3), i < n; [n, 3]."""
    a = np.ascontiguousarray(axis, np.float64)
    out = np.zeros((n, 3))
    lib().orc_cone_batch(seed, pair, order, w3, _dp(a), float(cos_half_angle), n, _dp(out))
    return out


def trace_path(scene, source, *, seed, ray, pair, max_bounces, window_len, max_seg=4096):
    """Segments of one ray: dict(orig [n,3], dir [n,3], t [n], tri [n]) (diagnostics)."""
    verts = np.ascontiguousarray(scene["verts"], np.float64)
    tris = np.ascontiguousarray(scene["tris"], np.int32)
    tm = np.ascontiguousarray(scene["tri_mat"], np.int32)
    ab = np.ascontiguousarray(scene["absorption"], np.float64)
    sc = np.ascontiguousarray(scene["scattering"], np.float64)
    src = np.ascontiguousarray(source, np.float64)
    o = np.zeros((max_seg, 3)); d = np.zeros((max_seg, 3)); t = np.zeros(max_seg); tri = np.zeros(max_seg, np.int64)
    n = lib().orc_trace_path(_dp(verts), len(tris), tris.ctypes.data_as(C.POINTER(C.c_int32)),
                             tm.ctypes.data_as(C.POINTER(C.c_int32)), _dp(ab), _dp(sc), ab.shape[1],
                             _dp(src), seed, ray, pair, max_bounces, window_len, max_seg, _dp(o), _dp(d), _dp(t),
                             tri.ctypes.data_as(C.POINTER(C.c_int64)))
    return dict(orig=o[:n], dir=d[:n], t=t[:n], tri=tri[:n])


# ----------------------------------------------------------------- estimation

RANGES = ((-5.0, -35.0), (-5.0, -25.0), (-5.0, -15.0), (0.0, -10.0))  # T30, T20, T10, EDT
ST_OK = 0
ST_NO_ENERGY = 1
ST_BAD_FIT = 2
ST_NO_RANGE = 4
ST_TRUNCATED_BY_BOUNCES = 8
ST_TAIL_COMPENSATED = 16


def _fit(I, dt, C0, m_last, W):
    """One Schroeder fit.  S[m] = C0 + sum_{j=m}^{m_last} I[j] (backward
    integration, the energy remaining after the left edge of bin m, plus the
    tail constant C0), y = 10 log10(S/S[0]) at t_m = m dt; the first of the
    ranges T30, T20, T10, EDT whose bottom level is reached at some
    m <= m_last - W is fitted by ordinary least squares over the points with
    lo <= y <= hi (at least 3).  Returns (rt60, range index, status)."""
    Sb = np.cumsum(I[: m_last + 1][::-1])[::-1]
    S = C0 + Sb
    y = 10.0 * np.log10(S / S[0])
    t = np.arange(m_last + 1) * dt
    top = m_last - W
    if top < 0:
        return 0.0, -1, ST_NO_RANGE
    for r, (hi, lo) in enumerate(RANGES):
        if not np.any(y[: top + 1] <= lo):
            continue
        sel = (y <= hi) & (y >= lo)
        if sel.sum() < 3:
            continue
        tt, yy = t[sel], y[sel]
        n = float(len(tt))
        st_, sy = tt.sum(), yy.sum()
        stt, sty = (tt * tt).sum(), (tt * yy).sum()
        den = n * stt - st_ * st_
        if den <= 0:
            continue
        slope = (n * sty - st_ * sy) / den
        if slope >= 0:
            return 0.0, r, ST_BAD_FIT
        return -60.0 / slope, r, ST_OK
    return 0.0, -1, ST_NO_RANGE


def rt60_schroeder(I, dt, tail_iters=3):
    """RT60 of one band from its intensity histogram I[m] (Section 4.2,
    "Reverberation Time": estimated by the standard Schroeder method).
    Reading: the fit range falls back T30 -> T20 -> T10 -> EDT; W = max(1,
    floor(T/20)) bins at the end must lie below the fitted range; if the
    energy reaches the last W bins the IR was cut by the window, and the
    missing tail is added to the backward integral, refitting `tail_iters`
    times: with tau = RT60 / (6 ln 10) (the intensity decay constant), the mean
    of I over the last W bins up to m_last, which stands for the intensity
    (W-1)/2 bins before the end, is extrapolated to the window end and
    integrated to infinity, C = mean * exp(-(W+1) dt / (2 tau)) * tau / dt.
    Returns (rt60, range, status)."""
    I = np.asarray(I, np.float64)
    T = len(I)
    W = max(1, T // 20)
    nz = np.nonzero(I > 0)[0]
    if len(nz) == 0:
        return 0.0, -1, ST_NO_ENERGY
    m_last = int(nz[-1])
    rt, rng_, st = _fit(I, dt, 0.0, m_last, W)
    if st == ST_OK and m_last >= T - W:
        tail = I[m_last - W + 1: m_last + 1].mean()
        for _ in range(tail_iters):
            tau = rt / (6.0 * math.log(10.0))
            C0 = tail * math.exp(-(W + 1) * dt / (2.0 * tau)) * tau / dt
            rt2, rng2, st2 = _fit(I, dt, C0, m_last, W)
            if st2 != ST_OK:
                break
            rt, rng_, st = rt2, rng2, ST_OK | ST_TAIL_COMPENSATED
    return rt, rng_, st


def estimate_reverb(hist, hist_late, stats, bin_width_s, rt60_source=None, tail_iters=3):
    """Reverb parameters of one IR (Section 4.2).
      hist      [T, B, NC]  SH x band histogram, I[m] = sqrt(4 pi) H[m][b][0]
      hist_late [T, B]      orders >= 3 only, or None
      rt60_source  1: RT60 from hist_late (Section 4.2: the IR the parameters
                   are estimated from holds only the higher-order
                   reflections); 0: from the all-orders intensity.  Default:
                   1 when hist_late is given, else 0.
      stats     dict from trace_ir
    Returns a dict of per-band arrays and scalars."""
    if rt60_source is None:
        rt60_source = 0 if hist_late is None else 1
    H = np.asarray(hist, np.float64)
    T, B, NC = H.shape
    dt = float(bin_width_s)
    I_all = math.sqrt(4.0 * math.pi) * H[:, :, 0]
    I_fit = I_all if rt60_source == 0 else np.asarray(hist_late, np.float64)
    out = dict(rt60=np.zeros(B), rt60_range=np.full(B, -1, np.int32), status=np.zeros(B, np.int32),
               e_direct=np.zeros(B), e_early=np.zeros(B), e_late=np.zeros(B), g_reverb=np.zeros(B),
               dir_loudness=np.zeros((B, NC)))
    for b in range(B):
        rt, rg, st = rt60_schroeder(I_fit[:, b], dt, tail_iters)
        e_late = float(stats["e_class"][2][b])
        if stats["e_alive_at_bounce_cap"][b] > 1e-3 * stats["e_emitted"]:
            st |= ST_TRUNCATED_BY_BOUNCES
        out["rt60"][b] = rt
        out["rt60_range"][b] = rg
        out["status"][b] = st
        out["e_direct"][b] = stats["e_class"][0][b]
        out["e_early"][b] = stats["e_class"][1][b]
        out["e_late"][b] = e_late
        # Eq. 5 with Eq. 8: g = sqrt(I_total / I_reverb), I_reverb = RT60 / (6 ln 10)
        out["g_reverb"][b] = math.sqrt(e_late * 6.0 * math.log(10.0) / rt) if rt > 0 else 0.0
        tot = I_all[:, b].sum()
        # Eq. 1: energy-weighted directivity, sum_t X_lm I / sum_t I with X_lm I = H_lm
        out["dir_loudness"][b] = H[:, b, :].sum(axis=0) / tot if tot > 0 else 0.0
    fl, fa = stats["first_late_bin"], stats["first_arrival_bin"]
    out["predelay_s"] = fl * dt if fl != INT32_MAX else -1.0
    out["first_arrival_s"] = fa * dt if fa != INT32_MAX else -1.0
    nf = stats["n_finite_segments"]
    out["mean_free_path_m"] = stats["seg_len_sum"] / nf if nf > 0 else 0.0
    return out
