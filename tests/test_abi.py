"""CPU checks of the C ABI: the library loads, exports every function that
include/rpr.h declares, and the binding's struct layouts match the header's
(checked by compiling the header with gcc).  No GPU calls."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import paper_1803_00430_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_function():
    names = P.header_functions()
    assert {"scene_create", "scene_destroy", "trace_ir", "estimate_reverb", "last_error"} <= set(names)
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(P.SIGNATURES) == set(names)
    assert L.rpr_version().startswith(b"rpr")


def test_invalid_arguments_fail_before_any_launch():
    L = P.lib()
    out = C.c_void_p()
    # n_bands out of range: rejected on the host, nothing launched
    rc = L.scene_create(None, 0, None, 0, None, None, None, 1, 9, None, C.byref(out))
    assert rc == -1 and out.value is None
    assert b"n_bands" in L.last_error()
    assert L.scene_rebuild(None, None, 0, None, 0, None, None, None, 1, 4, None) == -1
    assert b"scene is null" in L.last_error()
    assert L.trace_ir(None, None, 0, None, None, None, None, None, None, None) == -1
    ep = P.EstimateParams(0, 3)
    assert L.estimate_reverb(None, None, None, 1, 10, 4, 4, 1e-3, C.byref(ep), None, None) == -1
    assert L.estimate_reverb(None, None, None, 0, 10, 4, 2, 1e-3, C.byref(ep), None, None) == 0  # empty: no-op
    # learned estimator: shapes are checked on the host
    dims = (C.c_int32 * 3)(100, 64, 32)  # 100 is not a multiple of 32
    assert L.reverb_model_create(dims, 2, 16, 0, None, C.byref(out)) == -1 and out.value is None
    assert b"multiple of 32" in L.last_error()
    dims = (C.c_int32 * 3)(64, 64, 32)
    assert L.reverb_model_create(dims, 2, 0, 0, None, C.byref(out)) == -1
    assert L.reverb_model_featurize(None, None, 1, 0, 4, 16, None, None, None) == -1
    assert L.reverb_model_featurize(None, None, 0, 10, 4, 16, None, None, None) == 0  # empty: no-op
    assert L.reverb_model_decode(None, None, 1, 9, 1.0, None, None, None, None) == -1
    assert L.reverb_model_forward(None, None, 1, None, None) == -1


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "rpr.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("RprIrStats %zu\nRprReverbParams %zu\nRprTraceParams %zu\nRprSceneInfo %zu\n",
         sizeof(RprIrStats), sizeof(RprReverbParams), sizeof(RprTraceParams), sizeof(RprSceneInfo));
  printf("RprPair %zu\nRprBatchParams %zu\nRprBatchInfo %zu\n", sizeof(RprPair), sizeof(RprBatchParams),
         sizeof(RprBatchInfo));
  printf("RprModelInfo %zu\nRprAdamParams %zu\n", sizeof(RprModelInfo), sizeof(RprAdamParams));
  printf("RprReverbDesc %zu\nRprReverbSetup %zu\n", sizeof(RprReverbDesc), sizeof(RprReverbSetup));
  P(RprReverbSetup, g_comb); P(RprReverbSetup, dir); P(RprReverbSetup, J); P(RprReverbSetup, D);
  P(RprReverbDesc, max_comb_delay_s);
  P(RprModelInfo, max_batch); P(RprModelInfo, step); P(RprAdamParams, weight_decay);
  P(RprPair, n_rays); P(RprPair, seed); P(RprBatchInfo, best_ms);
  P(RprIrStats, seg_len_sum); P(RprIrStats, first_arrival_bin); P(RprIrStats, e_class);
  P(RprIrStats, e_escaped); P(RprIrStats, e_absorbed); P(RprIrStats, n_tri_tests);
  P(RprReverbParams, g_reverb); P(RprReverbParams, predelay_s); P(RprReverbParams, dir_loudness);
  P(RprTraceParams, bin_width_s); P(RprTraceParams, seed);
  return 0;
}''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["RprIrStats"]) == P.IR_STATS_DTYPE.itemsize
    assert int(got["RprReverbParams"]) == P.REVERB_PARAMS_DTYPE.itemsize
    assert int(got["RprTraceParams"]) == C.sizeof(P.TraceParams)
    assert int(got["RprSceneInfo"]) == C.sizeof(P.SceneInfo)
    assert int(got["RprPair"]) == C.sizeof(P.Pair) and int(got["RprPair.n_rays"]) == P.Pair.n_rays.offset
    assert int(got["RprPair.seed"]) == P.Pair.seed.offset
    assert int(got["RprBatchParams"]) == C.sizeof(P.BatchParams)
    assert int(got["RprBatchInfo"]) == C.sizeof(P.BatchInfo)
    assert int(got["RprBatchInfo.best_ms"]) == P.BatchInfo.best_ms.offset
    assert int(got["RprModelInfo"]) == C.sizeof(P.ModelInfo) and int(got["RprAdamParams"]) == C.sizeof(P.AdamParams)
    assert int(got["RprModelInfo.max_batch"]) == P.ModelInfo.max_batch.offset
    assert int(got["RprModelInfo.step"]) == P.ModelInfo.step.offset
    assert int(got["RprAdamParams.weight_decay"]) == P.AdamParams.weight_decay.offset
    for name in ("seg_len_sum", "first_arrival_bin", "e_class", "e_escaped", "e_absorbed", "n_tri_tests"):
        assert int(got[f"RprIrStats.{name}"]) == P.IR_STATS_DTYPE.fields[name][1], name
    for name in ("g_reverb", "predelay_s", "dir_loudness"):
        assert int(got[f"RprReverbParams.{name}"]) == P.REVERB_PARAMS_DTYPE.fields[name][1], name
    assert int(got["RprReverbDesc"]) == C.sizeof(P.ReverbDesc)
    assert int(got["RprReverbDesc.max_comb_delay_s"]) == P.ReverbDesc.max_comb_delay_s.offset
    assert int(got["RprReverbSetup"]) == P.REVERB_SETUP_DTYPE.itemsize
    for name in ("g_comb", "dir", "J", "D"):
        assert int(got[f"RprReverbSetup.{name}"]) == P.REVERB_SETUP_DTYPE.fields[name][1], name
    assert int(got["RprTraceParams.bin_width_s"]) == P.TraceParams.bin_width_s.offset
    assert int(got["RprTraceParams.seed"]) == P.TraceParams.seed.offset


def test_binding_has_no_cpu_path():
    # the binding module must not import the oracle
    src = open(os.path.join(ROOT, "paper_1803_00430_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no fallback", "")


def test_temporal_alpha_is_host_side_and_matches_oracle():
    """temporal_alpha is plain host arithmetic (no device call)."""
    import math
    from oracle import temporal as TC
    for dt, tau in ((0.1, 1.0), (0.1, 3.0), (0.02, 0.5)):
        assert math.isclose(P.temporal_alpha(dt, tau), TC.smoothing_alpha(dt, tau), rel_tol=1e-6)
    assert P.temporal_alpha(0.1, 0.0) == 1.0 and P.temporal_alpha(0.1, -2.0) == 1.0


def test_budget_ray_count_is_host_side_and_matches_oracle():
    from oracle.budget import budget_ray_count as ref
    g = np.random.default_rng(0)
    for _ in range(200):
        args = (int(g.integers(1, 10**12)), int(g.integers(0, 10**10)), int(g.integers(0, 10**7)),
                int(g.integers(1, 1000)), int(g.integers(1000, 10**9)), int(g.integers(1, 10**6)))
        assert P.budget_ray_count(*args) == ref(*args), args


def test_reverb_state_bytes_and_description_checks_are_host_side():
    """The reverberator's state size (header, comb lines with channels padded
    to 4 from order 1 on, all-pass lines) and its description checks need no
    GPU."""
    import math
    for nb, order, fs, tmax in ((4, 1, 44100.0, 0.3), (1, 0, 8000.0, 0.005), (8, 3, 192000.0, 2.0),
                                (3, 2, 48000.0, 0.1)):
        nc = (order + 1) ** 2
        pad = 1 if nc == 1 else (nc + 3) // 4 * 4
        m_cap = math.floor(float(np.float32(tmax)) * float(np.float32(fs)) + 0.5)
        a_cap = max(math.floor(t * float(np.float32(fs)) + 0.5) for t in (4.9e-3, 4.1e-3, 3.4e-3, 2.9e-3))
        want = 64 + 4 * nb * (8 * m_cap * pad + 4 * nc * a_cap)
        got = P.reverb_state_bytes(P.reverb_desc(nb, order, fs, 343.0, tmax))
        assert got == (want + 255) // 256 * 256, (nb, order, fs, tmax, got, want)
    for bad in (P.reverb_desc(0, 1), P.reverb_desc(9, 1), P.reverb_desc(4, -1), P.reverb_desc(4, 4),
                P.reverb_desc(4, 1, 7999.0), P.reverb_desc(4, 1, 200000.0), P.reverb_desc(4, 1, 44100.0, 0.0),
                P.reverb_desc(4, 1, 44100.0, 343.0, 0.004), P.reverb_desc(4, 1, 44100.0, 343.0, 2.5),
                P.reverb_desc(4, 1, float("nan"))):
        with pytest.raises(P.RprError):
            P.reverb_state_bytes(bad)
    L = P.lib()
    d = P.reverb_desc()
    # bad arguments are refused before any launch; empty calls are no-ops
    assert L.reverb_setup(None, None, 1, 10, 0.01, None, None, 1, C.byref(d), None, None) == -1
    assert L.reverb_setup(None, None, 1, 0, 0.01, None, None, 1, C.byref(d), None, None) == -1
    assert L.reverb_setup(None, None, 0, 10, 0.01, None, None, 1, C.byref(d), None, None) == 0
    assert L.reverb_render(None, 2, None, 16, None, None, C.byref(d), None) == -1
    assert L.reverb_render(None, -1, None, 0, None, None, C.byref(d), None) == -1
    assert L.reverb_render(None, 0, None, 0, None, None, C.byref(d), None) == 0
    assert L.reverb_render(None, 2, None, 0, None, None, C.byref(d), None) == 0  # no samples: no launch
    assert L.reverb_state_reset(None, 3, C.byref(d), None) == -1
    assert L.reverb_state_reset(None, 0, C.byref(d), None) == 0
    assert L.reverb_state_reset(C.c_void_p(16), 1, None, None) == -1
