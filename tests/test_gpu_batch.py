"""Batched persistent launch: every pair of a batch equals the same pair traced
alone by trace_ir (itself checked against the oracle), whatever the launch
shape; graph replays equal eager runs."""
import numpy as np
import pytest

import paper_1803_00430_amd as P
import rpr_scenes as R
from parity import assert_hist_close, gpu_trace

pytestmark = pytest.mark.gpu

T, NSH, DT = 400, 3, 1e-3


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    tiny = R.tiny_config()
    b1 = R.batch_scene(103, n_pairs=3)  # shoebox
    b2 = R.batch_scene(104, n_pairs=3)  # L-room
    b3 = R.batch_scene(105, n_pairs=3)  # cluttered interior
    dicts = [tiny, b1, b2, b3]
    scenes = [P.Scene.from_dict(d) for d in dicts]
    pairs = [dict(scene=0, source=tiny["sources"][0], listener=tiny["listener"], radius=0.5, n_rays=1500,
                  max_bounces=40, seed=1000, pair_id=0)]
    g = R.rng(5)
    k = 1
    for si, d in enumerate(dicts[1:], start=1):
        for p in d["pairs"]:
            pairs.append(dict(scene=si, source=p["source"], listener=p["listener"], radius=p["radius"],
                              n_rays=int(g.integers(500, 2500)), max_bounces=int(g.integers(20, 80)),
                              seed=1000 + k, pair_id=k))
            k += 1
    return scenes, pairs


def _alone(scenes, p):
    return gpu_trace(scenes[p["scene"]], np.asarray(p["source"])[None], p["listener"], p["radius"],
                     n_rays_total=p["n_rays"], max_bounces=p["max_bounces"], sh_order=NSH, n_bins=T,
                     bin_width_s=DT, seed=p["seed"], pair_base=p["pair_id"], want_hash=False)


def _host(b):
    return (b.hist.double().cpu().numpy(), b.hist_late.double().cpu().numpy(), P.stats_host(b.stats),
            P.params_host(b.params))


@pytest.mark.parametrize("order,wpc", [(0, 0), (1, 2)])
def test_batch_equals_pairs_alone(setup, order, wpc):
    import torch
    scenes, pairs = setup
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False,
                order=order, waves_per_cu=wpc)
    b.run()
    torch.cuda.synchronize()
    H, HL, st, prm = _host(b)
    for i, p in enumerate(pairs):
        a = _alone(scenes, p)
        assert_hist_close(H[i], a["hist"][0], tol=1e-5, what=f"pair {i}")
        assert_hist_close(HL[i], a["hist_late"][0], tol=1e-5, what=f"pair {i} late")
        for key in ("n_segments", "n_finite_segments", "n_escaped", "n_rays"):
            assert st[i][key] == a["stats"][0][key], (i, key)
        assert st[i]["first_arrival_bin"] == a["stats"][0]["first_arrival_bin"]
    info = b.info()
    assert info["n_pairs"] == len(pairs) and info["total_rays"] == sum(p["n_rays"] for p in pairs)
    assert info["order"] == order and info["graph"] == 0
    b.close()


def test_graph_replays_match_eager(setup):
    import torch
    scenes, pairs = setup
    eager = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False)
    eager.run()
    torch.cuda.synchronize()
    He, HLe, ste, pre = _host(eager)
    g = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=True, use_graph=True)
    info = g.info()
    assert info["graph"] == 1 and info["n_candidates"] >= 2 and info["best_ms"] <= info["worst_ms"]
    for rep in range(3):
        g.run()
        torch.cuda.synchronize()
        Hg, HLg, stg, prg = _host(g)
        for i in range(len(pairs)):
            assert_hist_close(Hg[i], He[i], tol=1e-5, what=f"replay {rep} pair {i}")
            assert stg[i]["n_segments"] == ste[i]["n_segments"]
        # the replay's estimation step equals an eager estimate of the replay's
        # own histograms (RT60 of two runs may differ where FP32 atomic order
        # moves a point of a sparse decay across a fit-range boundary)
        ref = P.alloc_params(len(pairs))
        P.estimate_reverb(g.hist, g.hist_late, g.stats, T, 4, NSH, DT, ref)
        pr = P.params_host(ref)
        assert np.array_equal(prg["rt60"], pr["rt60"]) and np.array_equal(prg["status"], pr["status"])
        assert np.array_equal(prg["g_reverb"], pr["g_reverb"])
        # eager work between replays
        eager.run()
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
    g.close()
    eager.close()


def test_batch_rejects_bad_pairs(setup):
    scenes, pairs = setup
    bad = [dict(pairs[0], scene=7)]
    with pytest.raises(P.RprError):
        P.Batch(scenes, bad, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False)
    bad = [dict(pairs[0], n_rays=0)]
    with pytest.raises(P.RprError):
        P.Batch(scenes, bad, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False)
