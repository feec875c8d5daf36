"""trace_ir_noalloc (the allocation-free variant of trace_ir, scratch in a
static device array) against trace_ir through the C ABI: two calls in a row,
the second with fewer sources, rays and bins than the first, so that the
second must not see what the first left in the shared scratch.  trace_ir
hands its queue slots out in the order of the rays' first directions and
trace_ir_noalloc in ray order, so equal ray hashes also show that the order
changes no ray's path (3,001 rays per source: three blocks of the sort and a
ragged last one)."""
import numpy as np
import pytest

import paper_1803_00430_amd as P
import rpr_scenes as R
from parity import assert_hist_close

pytestmark = pytest.mark.gpu


def _run(fn, sc, srcs, lst, radius, kw):
    import torch
    hist, late, stats, rh = P.alloc_trace_outputs(len(srcs), kw["n_bins"], sc.n_bands, kw["sh_order"],
                                                  kw["n_rays_total"], want_hash=True)
    fn(sc, srcs, lst, radius, P.trace_params(**kw), hist, late, stats, rh)
    torch.cuda.synchronize()
    return (hist.double().cpu().numpy(), late.double().cpu().numpy(), P.stats_host(stats),
            rh.cpu().numpy().view(np.uint32))


def _same(a, b, n_src):
    Ha, La, Sa, ha = a
    Hb, Lb, Sb, hb = b
    # per-ray decisions are identical: the same kernel, the same rays
    assert np.array_equal(ha, hb)
    for s in range(n_src):
        assert_hist_close(Ha[s], Hb[s])
        assert_hist_close(La[s], Lb[s], what="hist_late")
        for k in ("n_segments", "n_finite_segments", "n_escaped", "n_rays", "first_arrival_bin", "first_late_bin"):
            assert Sa[s][k] == Sb[s][k], (s, k, Sa[s][k], Sb[s][k])
        for k in ("seg_len_sum", "e_emitted"):
            assert abs(Sa[s][k] - Sb[s][k]) <= 1e-9 * abs(Sb[s][k]) + 1e-15, (s, k)
        for k in ("e_class", "e_escaped", "e_alive_at_stop", "e_absorbed"):
            d = np.abs(np.asarray(Sa[s][k], np.float64) - np.asarray(Sb[s][k], np.float64))
            assert np.all(d <= 1e-4 * np.abs(np.asarray(Sb[s][k], np.float64)).max() + 1e-15), (s, k)


def test_noalloc_matches_trace_ir_on_consecutive_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    d = R.batch_scene(104, n_pairs=6)  # box-cluster interior
    sc = P.Scene.from_dict(d)
    srcs = np.asarray([p["source"] for p in d["pairs"]], np.float32)
    lst, radius = d["pairs"][0]["listener"], 0.75
    first = dict(n_rays_total=3001, max_bounces=60, sh_order=3, n_bins=700, bin_width_s=1e-3, seed=11, pair_base=2)
    second = dict(n_rays_total=517, max_bounces=25, sh_order=2, n_bins=150, bin_width_s=2e-3, seed=12, pair_base=9)
    print("noalloc: call 1, 6 sources x 3001 rays", flush=True)
    a1 = _run(P.trace_ir_noalloc, sc, srcs, lst, radius, first)
    b1 = _run(P.trace_ir, sc, srcs, lst, radius, first)
    _same(a1, b1, len(srcs))
    assert a1[2]["n_segments"].sum() > 6 * 3001
    print("noalloc: call 2, 2 sources x 517 rays", flush=True)
    a2 = _run(P.trace_ir_noalloc, sc, srcs[:2], lst, radius, second)
    b2 = _run(P.trace_ir, sc, srcs[:2], lst, radius, second)
    _same(a2, b2, 2)
    assert a2[2]["n_rays"].sum() == 2 * 517


def test_noalloc_rejects_too_many_sources():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    sc = P.Scene.from_dict(R.tiny_config())
    srcs = np.tile(np.asarray([[2.0, 2.0, 1.5]], np.float32), (1025, 1))
    kw = dict(n_rays_total=64, max_bounces=2, sh_order=0, n_bins=10, bin_width_s=1e-3, seed=0)
    hist, late, stats, _ = P.alloc_trace_outputs(len(srcs), kw["n_bins"], 4, kw["sh_order"])
    with pytest.raises(P.RprError) as e:
        P.trace_ir_noalloc(sc, srcs, (7.0, 5.0, 1.5), 0.5, P.trace_params(**kw), hist, late, stats)
    assert e.value.code == -1 and "1024" in str(e.value)
