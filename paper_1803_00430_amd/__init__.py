"""Python binding of librpr.so: ray-parameterized reverberation propagation
(arXiv 1803.00430) on MI355X.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory and streams; tensors are passed to the C ABI
(include/rpr.h) as raw pointers.  Importing this module does not need a GPU;
calling into the library does, and fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rpr.h")

RPR_OK = 0
MAX_BANDS = 8
MAX_COEFFS = 16
INT32_MAX = 2**31 - 1

ST_OK = 0
ST_NO_ENERGY = 1
ST_BAD_FIT = 2
ST_NO_RANGE = 4
ST_TRUNCATED_BY_BOUNCES = 8
ST_TAIL_COMPENSATED = 16


class RprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rpr error {code}: {msg}")
        self.code = code


class Source(C.Structure):
    _fields_ = [("pos", C.c_float * 3)]


class Listener(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("radius", C.c_float)]


class TraceParams(C.Structure):
    _fields_ = [("n_rays_total", C.c_int64), ("ray_begin", C.c_int64), ("ray_end", C.c_int64),
                ("max_bounces", C.c_int32), ("sh_order", C.c_int32), ("n_bins", C.c_int32),
                ("pair_base", C.c_int32), ("bin_width_s", C.c_float), ("speed_of_sound", C.c_float),
                ("seed", C.c_uint64), ("flags", C.c_int32), ("waves_per_cu", C.c_int32),
                ("segment_budget", C.c_int64), ("max_rays", C.c_int64)]


TRACE_COUNT_VISITS = 1
TRACE_DETERMINISTIC = 2


class EstimateParams(C.Structure):
    _fields_ = [("rt60_source", C.c_int32), ("tail_iters", C.c_int32)]


class SceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_nodes", C.c_int64), ("max_depth", C.c_int32),
                ("n_bands", C.c_int32), ("n_materials", C.c_int32), ("n_degenerate", C.c_int32),
                ("bounds_lo", C.c_float * 3), ("bounds_hi", C.c_float * 3), ("stack_need", C.c_int32),
                ("reserved", C.c_int32)]


class Pair(C.Structure):
    _fields_ = [("scene", C.c_int32), ("pair_id", C.c_int32), ("src", C.c_float * 3), ("lst", C.c_float * 3),
                ("radius", C.c_float), ("max_bounces", C.c_int32), ("n_rays", C.c_int64), ("seed", C.c_uint64)]


class BatchParams(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("sh_order", C.c_int32), ("bin_width_s", C.c_float),
                ("speed_of_sound", C.c_float), ("rt60_source", C.c_int32), ("tail_iters", C.c_int32),
                ("autotune", C.c_int32), ("use_graph", C.c_int32), ("waves_per_cu", C.c_int32),
                ("order", C.c_int32), ("method", C.c_int32), ("chunk_rays", C.c_int32),
                ("deterministic", C.c_int32)]


METHODS = {"source": 0, "listener": 1}


class BatchInfo(C.Structure):
    _fields_ = [("total_rays", C.c_int64), ("n_pairs", C.c_int32), ("waves_per_cu", C.c_int32),
                ("order", C.c_int32), ("stack_need", C.c_int32), ("graph", C.c_int32),
                ("n_candidates", C.c_int32), ("best_ms", C.c_float), ("worst_ms", C.c_float),
                ("chunk_rays", C.c_int32), ("from_cache", C.c_int32), ("stack_entries", C.c_int32),
                ("fixed_point", C.c_int32)]


# Host views of the device structs (same layout as include/rpr.h).
class ReverbDesc(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("sh_order", C.c_int32), ("sample_rate", C.c_float),
                ("speed_of_sound", C.c_float), ("max_comb_delay_s", C.c_float), ("reserved", C.c_int32)]


class PathCacheInfo(C.Structure):
    _fields_ = [("max_paths", C.c_int32), ("n_paths", C.c_int32), ("overflow", C.c_int32), ("table_size", C.c_int32)]


class ModelInfo(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("n_layers", C.c_int32), ("dims", C.c_int32 * 9), ("max_batch", C.c_int32),
                ("step", C.c_int64)]


class AdamParams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float), ("reserved", C.c_float)]


ST_LEARNED = 32
ST_UNCERTAIN = 64


IR_STATS_DTYPE = np.dtype([
    ("n_segments", "<i8"), ("n_finite_segments", "<i8"), ("n_escaped", "<i8"), ("n_rays", "<i8"),
    ("seg_len_sum", "<f8"), ("e_emitted", "<f8"), ("first_arrival_bin", "<i4"), ("first_late_bin", "<i4"),
    ("e_class", "<f8", (3, MAX_BANDS)), ("e_escaped", "<f8", (MAX_BANDS,)),
    ("e_alive_at_stop", "<f8", (MAX_BANDS,)), ("e_alive_at_bounce_cap", "<f8", (MAX_BANDS,)),
    ("e_absorbed", "<f8", (MAX_BANDS,)), ("n_node_visits", "<i8"), ("n_tri_tests", "<i8"),
    ("n_next_event", "<i8"), ("n_deposit_rows", "<i8"),
])
REVERB_PARAMS_DTYPE = np.dtype([
    ("rt60", "<f4", (MAX_BANDS,)), ("rt60_range", "<i4", (MAX_BANDS,)), ("status", "<i4", (MAX_BANDS,)),
    ("e_direct", "<f4", (MAX_BANDS,)), ("e_early", "<f4", (MAX_BANDS,)), ("e_late", "<f4", (MAX_BANDS,)),
    ("g_reverb", "<f4", (MAX_BANDS,)), ("predelay_s", "<f4"), ("first_arrival_s", "<f4"),
    ("mean_free_path_m", "<f4"), ("reserved", "<f4"), ("dir_loudness", "<f4", (MAX_BANDS, MAX_COEFFS)),
])
REVERB_COMBS = 8
REVERB_ALLPASS = 4
REVERB_SETUP_DTYPE = np.dtype([
    ("t_comb", "<f4", (REVERB_COMBS,)), ("m_comb", "<i4", (REVERB_COMBS,)), ("mfp_drawn", "<f4"),
    ("predelay_samples", "<i4"), ("n_bands", "<i4"), ("sh_order", "<i4"),
    ("g_comb", "<f4", (MAX_BANDS, REVERB_COMBS)), ("g_reverb", "<f4", (MAX_BANDS,)),
    ("dir", "<f4", (REVERB_COMBS, 4)), ("a", "<f4", (REVERB_COMBS, MAX_COEFFS)),
    ("J", "<f4", (REVERB_COMBS, MAX_COEFFS, MAX_COEFFS)), ("D", "<f4", (MAX_BANDS, MAX_COEFFS, MAX_COEFFS)),
])
assert IR_STATS_DTYPE.itemsize == 536 and REVERB_PARAMS_DTYPE.itemsize == 752
assert REVERB_SETUP_DTYPE.itemsize == 17392
PATH_RECORD_WORDS = 32
EARLY_PATH_DTYPE = np.dtype([
    ("source", "<i4"), ("order", "<i4"), ("tri", "<i4", (2,)), ("e", "<f4", (MAX_BANDS,)), ("t", "<f4"),
    ("d", "<f4", (MAX_COEFFS,)), ("reserved", "<f4", (3,)),
])
assert EARLY_PATH_DTYPE.itemsize == 128

_vp = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32

# name -> (restype, argtypes); every entry point of include/rpr.h
SIGNATURES = {
    "scene_create": (C.c_int, [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _i32, _vp, C.POINTER(_vp)]),
    "scene_rebuild": (C.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _i32, _vp]),
    "scene_wait": (C.c_int, [_vp]),
    "scene_destroy": (C.c_int, [_vp]),
    "scene_info": (C.c_int, [_vp, C.POINTER(SceneInfo)]),
    "trace_ir": (C.c_int, [_vp, C.POINTER(Source), _i32, C.POINTER(Listener), C.POINTER(TraceParams), _vp, _vp,
                           _vp, _vp, _vp]),
    "trace_ir_noalloc": (C.c_int, [_vp, C.POINTER(Source), _i32, C.POINTER(Listener), C.POINTER(TraceParams), _vp,
                                   _vp, _vp, _vp, _vp]),
    "trace_listener": (C.c_int, [_vp, C.POINTER(Source), _i32, C.POINTER(Listener), C.POINTER(TraceParams), _vp,
                                 _vp, _vp, _vp, _vp]),
    "estimate_reverb": (C.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _i32, C.c_float, C.POINTER(EstimateParams),
                                  _vp, _vp]),
    "temporal_alpha": (C.c_float, [C.c_float, C.c_float]),
    "budget_ray_count": (_i64, [_i64, _i64, _i64, _i64, _i64, _i64]),
    "ir_cache_update": (C.c_int, [_vp, _vp, _i64, C.c_float, _i32, _vp]),
    "reverb_params_smooth": (C.c_int, [_vp, _vp, _i32, _i32, C.c_float, C.c_float, _i32, _vp]),
    "trace_ir_paths": (C.c_int, [_vp, C.POINTER(Source), _i32, C.POINTER(Listener), C.POINTER(TraceParams), _vp,
                                 _vp, _vp, _vp, _vp, _i32, _vp]),
    "path_cache_create": (C.c_int, [_i32, C.POINTER(_vp)]),
    "path_cache_destroy": (C.c_int, [_vp]),
    "path_cache_update": (C.c_int, [_vp, _vp, _vp, _i32, C.c_float, _i32, C.c_float, _vp]),
    "path_cache_select": (C.c_int, [_vp, C.c_float, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _i32, C.c_float, _vp]),
    "path_cache_info": (C.c_int, [_vp, C.POINTER(PathCacheInfo)]),
    "reverb_state_bytes": (C.c_int, [C.POINTER(ReverbDesc), C.POINTER(_i64)]),
    "reverb_state_reset": (C.c_int, [_vp, _i32, C.POINTER(ReverbDesc), _vp]),
    "reverb_setup": (C.c_int, [_vp, _vp, _i32, _i32, C.c_float, _vp, _vp, _i32, C.POINTER(ReverbDesc), _vp, _vp]),
    "reverb_render": (C.c_int, [_vp, _i32, _vp, _i32, _vp, _vp, C.POINTER(ReverbDesc), _vp]),
    "scene_closest_hit": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "debug_philox": (C.c_int, [_vp, _i64, _vp, _vp]),
    "debug_sh_eval": (C.c_int, [_vp, _i64, _i32, _vp, _vp]),
    "memory_probe": (C.c_int, [_vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp]),
    "batch_create": (C.c_int, [C.POINTER(_vp), _i32, C.POINTER(Pair), _i32, C.POINTER(BatchParams), _vp, _vp,
                               _vp, _vp, _vp, C.POINTER(_vp)]),
    "batch_run": (C.c_int, [_vp, _vp]),
    "batch_info": (C.c_int, [_vp, C.POINTER(BatchInfo)]),
    "batch_destroy": (C.c_int, [_vp]),
    "reverb_model_create": (C.c_int, [C.POINTER(_i32), _i32, _i32, C.c_uint64, _vp, C.POINTER(_vp)]),
    "reverb_model_destroy": (C.c_int, [_vp]),
    "reverb_model_info": (C.c_int, [_vp, C.POINTER(ModelInfo)]),
    "reverb_model_load": (C.c_int, [_vp, _vp, _i64, _vp]),
    "reverb_model_save": (C.c_int, [_vp, _vp, _i64, _vp]),
    "reverb_model_featurize": (C.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "reverb_model_targets": (C.c_int, [_vp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "reverb_model_forward": (C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "reverb_model_backward": (C.c_int, [_vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp]),
    "reverb_model_grads": (C.c_int, [_vp, _vp, _i64, _vp]),
    "reverb_model_adam": (C.c_int, [_vp, C.POINTER(AdamParams), _vp]),
    "reverb_model_set_tower": (C.c_int, [_vp, _i32, _i32, _vp]),
    "reverb_model_train_step": (C.c_int, [_vp, _vp, _i64, _vp, _i32, _vp, _vp, C.POINTER(AdamParams), _vp, _vp]),
    "reverb_model_decode": (C.c_int, [_vp, _vp, _i64, _i32, C.c_float, _vp, _vp, _vp, _vp]),
    "reverb_params_scatter": (C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "reverb_model_feature_stats": (C.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "reverb_model_normalize": (C.c_int, [_vp, _i64, _i32, _vp, _vp, _vp]),
    "reverb_model_ood_gate": (C.c_int, [_vp, _i64, _i32, _i32, _i32, C.c_float, _i32, _vp, _vp, _vp]),
    "last_error": (C.c_char_p, []),
    "rpr_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load librpr.so (built in-tree by paper_1803_00430_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1803_00430_amd.build`"
                               " (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != RPR_OK:
        raise RprError(rc, lib().last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f32(x, device):
    import torch
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, np.float32), device=device)


def _dev_i32(x, device):
    import torch
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, np.int32), device=device)


class Scene:
    """A triangle scene with per-band materials and its BVH on the GPU."""

    def __init__(self, verts, tris, tri_mat, absorption, scattering, device="cuda", stream=None):
        import torch
        self.device = torch.device(device)
        v = _dev_f32(verts, self.device).reshape(-1, 3)
        t = _dev_i32(tris, self.device).reshape(-1, 3)
        m = None if tri_mat is None else _dev_i32(tri_mat, self.device).reshape(-1)
        a = _dev_f32(absorption, self.device)
        s = _dev_f32(scattering, self.device)
        if a.dim() != 2 or a.shape != s.shape:
            raise ValueError("absorption and scattering must both be [materials, bands]")
        self.n_materials, self.n_bands = int(a.shape[0]), int(a.shape[1])
        h = C.c_void_p()
        _check(lib().scene_create(_ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(m), _ptr(a), _ptr(s),
                                  self.n_materials, self.n_bands, _stream(stream), C.byref(h)))
        self._h = h

    @classmethod
    def from_dict(cls, d, **kw):
        return cls(d["verts"], d["tris"], d.get("tri_mat"), d["absorption"], d["scattering"], **kw)

    def rebuild(self, verts, tris, tri_mat, absorption, scattering, stream=None):
        """Rebuild this scene in place from new geometry and materials
        (scene_rebuild: enqueued on the stream without waiting; no allocation
        when they fit what the scene holds).  What the device finds wrong with
        the inputs is raised by the next call that uses the scene, or wait()."""
        v = _dev_f32(verts, self.device).reshape(-1, 3)
        t = _dev_i32(tris, self.device).reshape(-1, 3)
        m = None if tri_mat is None else _dev_i32(tri_mat, self.device).reshape(-1)
        a = _dev_f32(absorption, self.device)
        s = _dev_f32(scattering, self.device)
        if a.dim() != 2 or a.shape != s.shape:
            raise ValueError("absorption and scattering must both be [materials, bands]")
        nm, nb = int(a.shape[0]), int(a.shape[1])
        import torch
        if stream is not None and stream != torch.cuda.current_stream(self.device):
            for x in (v, t, m, a, s):
                if x is not None:
                    x.record_stream(stream)
        rc = lib().scene_rebuild(self.handle, _ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(m), _ptr(a), _ptr(s),
                                 nm, nb, _stream(stream))
        # the scene's band count follows the call even when the build fails
        self.n_materials, self.n_bands = nm, nb
        # the inputs stay referenced until the build has run (the next rebuild waits for it)
        self._inputs = (v, t, m, a, s)
        _check(rc)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("scene is closed")
        return self._h

    def info(self) -> dict:
        si = SceneInfo()
        _check(lib().scene_info(self.handle, C.byref(si)))
        return dict(n_tris=si.n_tris, n_nodes=si.n_nodes, max_depth=si.max_depth, n_bands=si.n_bands,
                    n_materials=si.n_materials, n_degenerate=si.n_degenerate,
                    bounds_lo=list(si.bounds_lo), bounds_hi=list(si.bounds_hi), stack_need=si.stack_need)

    def wait(self):
        """Wait for the last rebuild and raise what it found wrong, if anything."""
        _check(lib().scene_wait(self.handle))

    def closest_hit(self, orig, dirs, stream=None):
        import torch
        o = _dev_f32(orig, self.device).reshape(-1, 3)
        d = _dev_f32(dirs, self.device).reshape(-1, 3)
        n = o.shape[0]
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        tri = torch.empty(n, dtype=torch.int32, device=self.device)
        _check(lib().scene_closest_hit(self.handle, _ptr(o), _ptr(d), n, _ptr(t), _ptr(tri), _stream(stream)))
        return t, tri

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_params(*, n_rays_total, max_bounces, sh_order, n_bins, bin_width_s, seed, ray_begin=0, ray_end=None,
                 pair_base=0, speed_of_sound=343.0, flags=0, waves_per_cu=0, segment_budget=0,
                 max_rays=0) -> TraceParams:
    return TraceParams(int(n_rays_total), int(ray_begin), int(n_rays_total if ray_end is None else ray_end),
                       int(max_bounces), int(sh_order), int(n_bins), int(pair_base), float(bin_width_s),
                       float(speed_of_sound), int(seed), int(flags), int(waves_per_cu), int(segment_budget),
                       int(max_rays))


def alloc_trace_outputs(n_src, n_bins, n_bands, sh_order, n_rays=0, device="cuda", late=True, want_hash=False):
    import torch
    nc = (sh_order + 1) ** 2
    hist = torch.empty((n_src, n_bins, n_bands, nc), dtype=torch.float32, device=device)
    hist_late = torch.empty((n_src, n_bins, n_bands), dtype=torch.float32, device=device) if late else None
    stats = torch.empty((n_src, IR_STATS_DTYPE.itemsize), dtype=torch.uint8, device=device)
    ray_hash = torch.empty((n_src, n_rays), dtype=torch.int32, device=device) if want_hash else None
    return hist, hist_late, stats, ray_hash


def trace_ir(scene: Scene, sources, listener, radius, params: TraceParams, hist, hist_late, stats, ray_hash=None,
             stream=None):
    """Enqueue trace_ir on `stream` into caller-allocated tensors."""
    srcs = np.ascontiguousarray(np.atleast_2d(sources), np.float32)
    n = len(srcs)
    src_arr = (Source * max(n, 1))()
    for i in range(n):
        src_arr[i].pos[:] = [float(x) for x in srcs[i]]
    lp = np.asarray(listener, np.float32)
    lst = Listener((C.c_float * 3)(*[float(x) for x in lp]), float(radius))
    _check(lib().trace_ir(scene.handle, src_arr, n, C.byref(lst), C.byref(params), _ptr(hist), _ptr(hist_late),
                          _ptr(stats), _ptr(ray_hash), _stream(stream)))


def trace_ir_noalloc(scene: Scene, sources, listener, radius, params: TraceParams, hist, hist_late, stats,
                     ray_hash=None, stream=None):
    """Enqueue trace_ir_noalloc (trace_ir with the library's static scratch,
    no allocation; at most 1024 sources) on `stream`."""
    srcs = np.ascontiguousarray(np.atleast_2d(sources), np.float32)
    n = len(srcs)
    src_arr = (Source * max(n, 1))()
    for i in range(n):
        src_arr[i].pos[:] = [float(x) for x in srcs[i]]
    lp = np.asarray(listener, np.float32)
    lst = Listener((C.c_float * 3)(*[float(x) for x in lp]), float(radius))
    _check(lib().trace_ir_noalloc(scene.handle, src_arr, n, C.byref(lst), C.byref(params), _ptr(hist),
                                  _ptr(hist_late), _ptr(stats), _ptr(ray_hash), _stream(stream)))


def trace_listener(scene: Scene, sources, listener, radius, params: TraceParams, hist, hist_late, stats,
                   ray_hash=None, stream=None):
    """Enqueue trace_listener (listener point, source balls of `radius`) on
    `stream` into caller-allocated tensors; `ray_hash` is [n_rays] (one per
    ray) or None."""
    srcs = np.ascontiguousarray(np.atleast_2d(sources), np.float32)
    n = len(srcs)
    src_arr = (Source * max(n, 1))()
    for i in range(n):
        src_arr[i].pos[:] = [float(x) for x in srcs[i]]
    lp = np.asarray(listener, np.float32)
    lst = Listener((C.c_float * 3)(*[float(x) for x in lp]), float(radius))
    _check(lib().trace_listener(scene.handle, src_arr, n, C.byref(lst), C.byref(params), _ptr(hist),
                                _ptr(hist_late), _ptr(stats), _ptr(ray_hash), _stream(stream)))


def estimate_reverb(hist, hist_late, stats, n_bins, n_bands, sh_order, bin_width_s, out, rt60_source=None,
                    tail_iters=3, stream=None):
    """Enqueue estimate_reverb; `out` is a uint8 tensor [n_ir, 752].
    rt60_source: 1 late-only (orders >= 3), 0 all orders; default 1 when
    hist_late is given."""
    n_ir = int(stats.shape[0])
    if rt60_source is None:
        rt60_source = 0 if hist_late is None else 1
    ep = EstimateParams(int(rt60_source), int(tail_iters))
    _check(lib().estimate_reverb(_ptr(hist), _ptr(hist_late), _ptr(stats), n_ir, int(n_bins), int(n_bands),
                                 int(sh_order), float(bin_width_s), C.byref(ep), _ptr(out), _stream(stream)))


def budget_ray_count(budget_segments, prev_segments, prev_rays, min_rays, max_rays, nominal) -> int:
    """Rays of the next frame under a segment budget (see include/rpr.h)."""
    return int(lib().budget_ray_count(int(budget_segments), int(prev_segments), int(prev_rays), int(min_rays),
                                      int(max_rays), int(nominal)))


def temporal_alpha(frame_dt_s: float, tau_s: float) -> float:
    """Smoothing factor of one frame: 1 - exp(-dt / tau) (1 when tau <= 0)."""
    return float(lib().temporal_alpha(float(frame_dt_s), float(tau_s)))


def ir_cache_update(cache, fresh, alpha: float, first: bool, stream=None):
    """cache = alpha * fresh + (1 - alpha) * cache over all cells (fresh on
    the first frame); both float32 device tensors of the same size."""
    assert cache.numel() == fresh.numel() and cache.dtype == fresh.dtype
    _check(lib().ir_cache_update(_ptr(cache), _ptr(fresh), int(cache.numel()), float(alpha), int(bool(first)),
                                 _stream(stream)))


def reverb_params_smooth(cache, fresh, n_bands, alpha_early: float, alpha_late: float, first: bool, stream=None):
    """Eq. 4 and the energy smoothing, in place in `cache` ([n_ir, 752] uint8)."""
    n_ir = int(cache.shape[0])
    assert int(fresh.shape[0]) == n_ir
    _check(lib().reverb_params_smooth(_ptr(cache), _ptr(fresh), n_ir, int(n_bands), float(alpha_early),
                                      float(alpha_late), int(bool(first)), _stream(stream)))


def alloc_params(n_ir, device="cuda"):
    import torch
    return torch.empty((n_ir, REVERB_PARAMS_DTYPE.itemsize), dtype=torch.uint8, device=device)


def stats_host(stats) -> np.ndarray:
    """Device stats tensor -> numpy structured array (IR_STATS_DTYPE)."""
    return stats.cpu().numpy().view(IR_STATS_DTYPE).reshape(-1)


def params_host(params) -> np.ndarray:
    return params.cpu().numpy().view(REVERB_PARAMS_DTYPE).reshape(-1)


def debug_philox(ctr_key, stream=None):
    """ctr_key: uint32-valued [n, 6] (ctr0..3, key0..1) -> [n, 4] device outputs."""
    import torch
    a = np.ascontiguousarray(ctr_key, np.uint32).view(np.int32)
    t = torch.as_tensor(a, device="cuda")
    out = torch.empty((a.shape[0], 4), dtype=torch.int32, device="cuda")
    _check(lib().debug_philox(_ptr(t), a.shape[0], _ptr(out), _stream(stream)))
    return out


def memory_probe(buf, pattern, iters, grid, block, sink, stream=None):
    """Enqueue one memory-probe launch over the device tensor `buf` (see
    include/rpr.h); returns the bytes it reads."""
    nbytes = buf.numel() * buf.element_size()
    _check(lib().memory_probe(_ptr(buf), int(nbytes), int(pattern), int(iters), int(grid), int(block), _ptr(sink),
                              _stream(stream)))
    return int(iters) * nbytes if pattern == 0 else int(grid) * int(block) * int(iters) * 128


def device_cus():
    """Compute units of the current device."""
    import torch
    return int(torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count)


def debug_sh_eval(dirs, order, stream=None):
    import torch
    d = _dev_f32(dirs, "cuda").reshape(-1, 3)
    out = torch.empty((d.shape[0], MAX_COEFFS), dtype=torch.float32, device="cuda")
    _check(lib().debug_sh_eval(_ptr(d), d.shape[0], int(order), _ptr(out), _stream(stream)))
    return out


class Batch:
    """A planned batch of source-listener pairs over several scenes; `run()`
    enqueues reset + trace + estimate (a graph replay when use_graph).
    method "source" traces each pair from its source to the listener sphere;
    "listener" from its listener point with next-event queries toward its
    source, a ball of the pair's radius."""

    def __init__(self, scenes, pairs, *, n_bins, sh_order, bin_width_s, speed_of_sound=343.0, rt60_source=None,
                 tail_iters=3, autotune=True, use_graph=True, waves_per_cu=0, order=0, late=True, device="cuda",
                 stream=None, method="source", chunk_rays=0, deterministic=False):
        import torch
        if rt60_source is None:
            rt60_source = 1 if late else 0
        self.scenes = list(scenes)  # kept alive for the batch's lifetime
        n = len(pairs)
        arr = (Pair * n)()
        for i, p in enumerate(pairs):
            arr[i].scene = int(p["scene"])
            arr[i].pair_id = int(p.get("pair_id", i))
            arr[i].src[:] = [float(x) for x in p["source"]]
            arr[i].lst[:] = [float(x) for x in p["listener"]]
            arr[i].radius = float(p["radius"])
            arr[i].max_bounces = int(p["max_bounces"])
            arr[i].n_rays = int(p["n_rays"])
            arr[i].seed = int(p["seed"])
        nb = self.scenes[0].n_bands
        self.n_pairs, self.n_bins, self.n_bands, self.sh_order = n, n_bins, nb, sh_order
        self.hist, self.hist_late, self.stats, _ = alloc_trace_outputs(n, n_bins, nb, sh_order, device=device,
                                                                       late=late)
        self.params = alloc_params(n, device=device)
        bp = BatchParams(int(n_bins), int(sh_order), float(bin_width_s), float(speed_of_sound), int(rt60_source),
                         int(tail_iters), int(bool(autotune)), int(bool(use_graph)), int(waves_per_cu), int(order),
                         METHODS[method], int(chunk_rays), int(bool(deterministic)))
        handles = (C.c_void_p * len(self.scenes))(*[sc.handle.value for sc in self.scenes])
        h = C.c_void_p()
        _check(lib().batch_create(handles, len(self.scenes), arr, n, C.byref(bp), _ptr(self.hist),
                                  _ptr(self.hist_late), _ptr(self.stats), _ptr(self.params), _stream(stream),
                                  C.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().batch_run(self._h, _stream(stream)))

    def info(self) -> dict:
        bi = BatchInfo()
        _check(lib().batch_info(self._h, C.byref(bi)))
        return {k: getattr(bi, k) for k, _ in BatchInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ learned estimator
STAT_FEATURES = 64
# input: 200 bins x 4 bands x 16 SH coefficients + 64 trace statistics -> 16 means + 16 log-variances
LEARN_DIMS = (12800 + STAT_FEATURES, 512, 512, 512, 32)
# two-tower variant: the 12,800 histogram features through a 64-unit tower, the 64 statistics
# passed through as +s and -s (reverb_model_set_tower), then 512 -> 512 -> 32
LEARN_TOWER = 64
LEARN_DIMS_TOWER = (12800 + STAT_FEATURES, LEARN_TOWER + 2 * STAT_FEATURES, 512, 512, 32)


class Model:
    """The learned reverb-parameter estimator (an MLP trained by the library's
    own BF16 matrix-core kernels).  Parameters are an FP32 vector in the
    layout of include/rpr.h (W_l row-major then b_l, per layer)."""

    def __init__(self, dims=LEARN_DIMS, *, max_batch=256, seed=0, stream=None):
        arr = (C.c_int32 * len(dims))(*[int(d) for d in dims])
        h = C.c_void_p()
        _check(lib().reverb_model_create(arr, len(dims) - 1, int(max_batch), int(seed), _stream(stream), C.byref(h)))
        self._h = h
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        self.input_norm = None  # (shift, scale) device tensors, set when the model is trained
        self.tower = None  # (n_hist, tower_width) when layer 0 is a two-tower layer

    def info(self) -> dict:
        mi = ModelInfo()
        _check(lib().reverb_model_info(self._h, C.byref(mi)))
        return dict(n_params=mi.n_params, n_layers=mi.n_layers, dims=list(mi.dims[:mi.n_layers + 1]),
                    max_batch=mi.max_batch, step=mi.step)

    @property
    def n_params(self) -> int:
        return self.info()["n_params"]

    def load(self, params, stream=None):
        _check(lib().reverb_model_load(self._h, _ptr(params), params.numel(), _stream(stream)))

    def save(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().reverb_model_save(self._h, _ptr(out), out.numel(), _stream(stream)))
        return out

    def grads(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().reverb_model_grads(self._h, _ptr(out), out.numel(), _stream(stream)))
        return out

    def forward(self, features, out=None, stream=None):
        import torch
        n = features.shape[0]
        if out is None:
            out = torch.empty((n, self.dims[-1]), dtype=torch.float32, device=features.device)
        _check(lib().reverb_model_forward(self._h, _ptr(features), n, _ptr(out), _stream(stream)))
        return out

    def backward(self, features, t, w, rows=None, m=None, loss=None, stream=None):
        import torch
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=features.device)
        m = int(rows.shape[0] if rows is not None else features.shape[0]) if m is None else int(m)
        _check(lib().reverb_model_backward(self._h, _ptr(features), features.shape[0], _ptr(rows), m, _ptr(t),
                                           _ptr(w), _ptr(loss), _stream(stream)))
        return loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, stream=None):
        ap = AdamParams(lr, beta1, beta2, eps, weight_decay, 0.0)
        _check(lib().reverb_model_adam(self._h, C.byref(ap), _stream(stream)))

    def set_tower(self, n_hist, tower_width, stream=None):
        """Two-tower layer 0 (see reverb_model_set_tower); (0, 0) restores a dense one."""
        _check(lib().reverb_model_set_tower(self._h, int(n_hist), int(tower_width), _stream(stream)))
        self.tower = (int(n_hist), int(tower_width)) if tower_width else None

    def train_step(self, features, t, w, rows, loss, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
                   m=None, stream=None):
        ap = AdamParams(lr, beta1, beta2, eps, weight_decay, 0.0)
        m = int(rows.shape[0]) if m is None else int(m)
        _check(lib().reverb_model_train_step(self._h, _ptr(features), features.shape[0], _ptr(rows), m, _ptr(t),
                                             _ptr(w), C.byref(ap), _ptr(loss), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().reverb_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def featurize(hist, n_bins, n_bands, n_coeffs, stats=None, stream=None):
    """BF16 features [n][T*B*NC + 64] (raw uint16 in an int16 tensor) and e_in [n]."""
    import torch
    n = hist.shape[0]
    f = torch.empty((n, n_bins * n_bands * n_coeffs + STAT_FEATURES), dtype=torch.int16, device=hist.device)
    e = torch.empty(n, dtype=torch.float32, device=hist.device)
    _check(lib().reverb_model_featurize(_ptr(hist), _ptr(stats), n, int(n_bins), int(n_bands), int(n_coeffs),
                                        _ptr(f), _ptr(e), _stream(stream)))
    return f, e


def targets(ref_params, e_in, n_bands, stream=None):
    import torch
    n = e_in.shape[0]
    t = torch.empty((n, 4 * n_bands), dtype=torch.float32, device=e_in.device)
    w = torch.empty((n, 4 * n_bands), dtype=torch.float32, device=e_in.device)
    _check(lib().reverb_model_targets(_ptr(ref_params), _ptr(e_in), n, int(n_bands), _ptr(t), _ptr(w),
                                      _stream(stream)))
    return t, w


def decode(out, e_in, n_bands, kappa, stream=None):
    """(params [n] ReverbParams, sigma [n][B], uncertain [n] i32) from network outputs."""
    import torch
    n = out.shape[0]
    params = alloc_params(n, device=out.device)
    sigma = torch.empty((n, n_bands), dtype=torch.float32, device=out.device)
    unc = torch.empty(n, dtype=torch.int32, device=out.device)
    _check(lib().reverb_model_decode(_ptr(out), _ptr(e_in), n, int(n_bands), float(kappa), _ptr(params),
                                     _ptr(sigma), _ptr(unc), _stream(stream)))
    return params, sigma, unc


def feature_stats(features, n_hist, stream=None):
    """(mean [F], scale [F]) of the input normalisation fitted on `features`."""
    import torch
    n, F = features.shape
    mean = torch.empty(F, dtype=torch.float32, device=features.device)
    scale = torch.empty(F, dtype=torch.float32, device=features.device)
    _check(lib().reverb_model_feature_stats(_ptr(features), n, F, int(n_hist), _ptr(mean), _ptr(scale),
                                            _stream(stream)))
    return mean, scale


def normalize(features, shift, scale, stream=None):
    """In place: features = (features - shift) * scale (BF16)."""
    n, F = features.shape
    _check(lib().reverb_model_normalize(_ptr(features), n, F, _ptr(shift), _ptr(scale), _stream(stream)))
    return features


def ood_gate(features, c0, c1, zmax, n_bands, params=None, uncertain=None, stream=None):
    """Mark rows whose normalised features in [c0, c1) exceed +-zmax as uncertain (in place)."""
    n, F = features.shape
    _check(lib().reverb_model_ood_gate(_ptr(features), n, F, int(c0), int(c1), float(zmax), int(n_bands),
                                       _ptr(params), _ptr(uncertain), _stream(stream)))


def params_scatter(src, idx, dst, stream=None):
    _check(lib().reverb_params_scatter(_ptr(src), _ptr(idx), idx.shape[0], _ptr(dst), _stream(stream)))


def trace_ir_paths(scene: Scene, sources, listener, radius, params: TraceParams, hist, hist_late, stats, records,
                   n_records, stream=None):
    """trace_ir plus the early-reflection path records: records
    [max_records, 32] float32, n_records [1] int32/uint32 (device)."""
    srcs = np.ascontiguousarray(np.atleast_2d(sources), np.float32)
    n = len(srcs)
    src_arr = (Source * max(n, 1))()
    for i in range(n):
        src_arr[i].pos[:] = [float(x) for x in srcs[i]]
    lp = np.asarray(listener, np.float32)
    lst = Listener((C.c_float * 3)(*[float(x) for x in lp]), float(radius))
    assert records.shape[1] == PATH_RECORD_WORDS and records.is_contiguous()
    _check(lib().trace_ir_paths(scene.handle, src_arr, n, C.byref(lst), C.byref(params), _ptr(hist),
                                _ptr(hist_late), _ptr(stats), _ptr(records), _ptr(n_records), int(records.shape[0]),
                                _stream(stream)))


class PathCache:
    """The diffuse path cache and the prioritization of early paths (see
    include/rpr.h)."""

    def __init__(self, max_paths=65536):
        h = _vp()
        _check(lib().path_cache_create(int(max_paths), C.byref(h)))
        self._h = h

    def close(self):
        if self._h is not None and self._h.value:
            lib().path_cache_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, records, n_records, alpha, first, min_energy=0.0, stream=None):
        _check(lib().path_cache_update(self._h, _ptr(records), _ptr(n_records), int(records.shape[0]), float(alpha),
                                       int(bool(first)), float(min_energy), _stream(stream)))

    def select(self, threshold, n_er, out, n_out, hist_late=None, stats=None, n_src=0, n_bins=1, n_bands=4,
               bin_width_s=1e-3, stream=None):
        _check(lib().path_cache_select(self._h, float(threshold), int(n_er), _ptr(out), _ptr(n_out), _ptr(hist_late),
                                       _ptr(stats), int(n_src), int(n_bins), int(n_bands), float(bin_width_s),
                                       _stream(stream)))

    def info(self):
        i = PathCacheInfo()
        _check(lib().path_cache_info(self._h, C.byref(i)))
        return dict(max_paths=i.max_paths, n_paths=i.n_paths, overflow=i.overflow, table_size=i.table_size)


def early_paths_host(out, n) -> np.ndarray:
    return out.cpu().numpy().view(EARLY_PATH_DTYPE).reshape(-1)[:n]


def reverb_desc(n_bands=4, sh_order=1, sample_rate=44100.0, speed_of_sound=343.0, max_comb_delay_s=0.3):
    return ReverbDesc(int(n_bands), int(sh_order), float(sample_rate), float(speed_of_sound),
                      float(max_comb_delay_s), 0)


def reverb_state_bytes(desc: ReverbDesc) -> int:
    """Bytes of rendering state per source (delay lines + header)."""
    b = _i64(0)
    _check(lib().reverb_state_bytes(C.byref(desc), C.byref(b)))
    return int(b.value)


def reverb_state(n_src, desc: ReverbDesc, device="cuda", stream=None):
    """Zeroed rendering state of n_src sources ([n_src, bytes] uint8)."""
    import torch
    st = torch.empty((n_src, reverb_state_bytes(desc)), dtype=torch.uint8, device=device)
    reverb_state_reset(st, desc, stream)
    return st


def reverb_state_reset(state, desc: ReverbDesc, stream=None):
    _check(lib().reverb_state_reset(_ptr(state), int(state.shape[0]), C.byref(desc), _stream(stream)))


def alloc_reverb_setup(n, device="cuda"):
    import torch
    return torch.zeros((n, REVERB_SETUP_DTYPE.itemsize), dtype=torch.uint8, device=device)


def reverb_setup(params, hist, bin_width_s, z, angles, desc: ReverbDesc, setup=None, first=True, stream=None):
    """Reverberator parameters of each IR (see include/rpr.h).  params [n, 752]
    uint8 (REVERB_PARAMS_DTYPE), hist [n, T, B, NC] f32, z [n, 8] f32 standard
    normals, angles [n, 8, 3] f32 radians; setup [n, 17392] uint8 (read when
    first is False).  Returns setup."""
    n = int(params.shape[0])
    assert hist.shape[0] == n and hist.dtype.is_floating_point and hist.is_contiguous()
    assert hist.shape[2] == desc.n_bands and hist.shape[3] == (desc.sh_order + 1) ** 2
    assert tuple(z.shape) == (n, REVERB_COMBS) and tuple(angles.shape) == (n, REVERB_COMBS, 3)
    if setup is None:
        setup = alloc_reverb_setup(n, params.device)
    assert setup.shape[0] == n and setup.shape[1] == REVERB_SETUP_DTYPE.itemsize
    _check(lib().reverb_setup(_ptr(params), _ptr(hist), n, int(hist.shape[1]), float(bin_width_s), _ptr(z),
                              _ptr(angles), int(bool(first)), C.byref(desc), _ptr(setup), _stream(stream)))
    return setup


def reverb_render(setup, x, state, desc: ReverbDesc, out=None, stream=None):
    """Render x [n_src, n_bands, n] f32 (band audio at the predelay tap) into
    out [n_src, (sh_order+1)^2, n] f32, continuing each source's state."""
    import torch
    n_src, nb, n = x.shape
    nc = (desc.sh_order + 1) ** 2
    assert nb == desc.n_bands and x.dtype == torch.float32 and x.is_contiguous()
    assert setup.shape[0] >= n_src and state.shape[0] >= n_src
    assert state.shape[1] == reverb_state_bytes(desc)
    if out is None:
        out = torch.empty((n_src, nc, n), dtype=torch.float32, device=x.device)
    assert tuple(out.shape) == (n_src, nc, n) and out.is_contiguous()
    _check(lib().reverb_render(_ptr(setup), n_src, _ptr(x), n, _ptr(state), _ptr(out), C.byref(desc),
                               _stream(stream)))
    return out


def reverb_setup_host(setup) -> np.ndarray:
    return setup.cpu().numpy().view(REVERB_SETUP_DTYPE).reshape(-1)


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/rpr.h."""
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))
