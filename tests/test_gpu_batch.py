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


@pytest.mark.parametrize("order,wpc,chunk", [(0, 0, 0), (1, 2, 0), (2, 0, 256), (2, 5, 4096)])
def test_batch_equals_pairs_alone(setup, order, wpc, chunk):
    import torch
    scenes, pairs = setup
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False,
                order=order, waves_per_cu=wpc, chunk_rays=chunk)
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
    assert info["order"] == order and info["graph"] == 0 and info["chunk_rays"] == (chunk or 1024)
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
    assert info["graph"] == 1
    assert info["from_cache"] == 1 or (info["n_candidates"] >= 2 and info["best_ms"] <= info["worst_ms"])
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


_CACHED_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import torch
import paper_1803_00430_amd as P
import test_gpu_batch as TB
scenes, pairs = TB._tune_case()
b = P.Batch(scenes, pairs, n_bins=TB.T, sh_order=TB.NSH, bin_width_s=TB.DT, autotune=True, use_graph=False)
print(json.dumps(b.info()))
"""


def _tune_case():
    """A small batch over the tiny room, with a tuning key no other test uses."""
    tiny = R.tiny_config()
    scenes = [P.Scene.from_dict(tiny)]
    pairs = [dict(scene=0, source=tiny["sources"][0], listener=tiny["listener"], radius=0.5, n_rays=700 + 300 * k,
                  max_bounces=20, seed=77 + k, pair_id=k) for k in range(3)]
    return scenes, pairs


def test_autotune_cache_file(setup, tmp_path, monkeypatch):
    """With RPR_AUTOTUNE_CACHE set, a tuned shape (width, queue order, chunk
    size, stack variant, deposit mode) is written to the file (one line per
    key) and a new process takes it from there without timing any candidate."""
    import json
    import os
    import subprocess
    import sys
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("RPR_AUTOTUNE_CACHE", str(path))
    scenes, pairs = _tune_case()
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=True, use_graph=False)
    info = b.info()
    b.close()
    # 4 widths x (1 + 1 + 3 chunk sizes), then the deeper stack variants and fixed-point deposits
    assert info["from_cache"] == 1 or info["n_candidates"] >= 8
    assert info["stack_entries"] in (32, 48, 64) and info["stack_need"] < info["stack_entries"]
    assert info["fixed_point"] in (0, 1)
    lines = [l.split() for l in path.read_text().splitlines()]
    assert lines and all(len(l) == 6 for l in lines)
    mine = [l for l in lines if l[1:4] == [str(info["waves_per_cu"]), str(info["order"]), str(info["chunk_rays"])]
            and l[5] == str(info["fixed_point"])]
    assert mine, (lines, info)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _CACHED_CHILD, root], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, RPR_AUTOTUNE_CACHE=str(path)))
    assert out.returncode == 0, out.stderr[-2000:]
    child = json.loads(out.stdout.strip().splitlines()[-1])
    assert child["from_cache"] == 1 and child["n_candidates"] == 0
    keys = ("waves_per_cu", "order", "chunk_rays", "stack_entries", "fixed_point")
    assert tuple(child[k] for k in keys) == tuple(info[k] for k in keys)


def test_deterministic_graph_replays_equal_eager(setup):
    """With deterministic accumulation a graph replay and an eager run of the
    batch give bit-identical histograms and RT60 (FP32 atomics would let the
    order of the adds move a point of a sparse decay across a fit-range edge)."""
    import torch
    scenes, pairs = setup
    eager = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False,
                    deterministic=True, waves_per_cu=3)
    eager.run()
    torch.cuda.synchronize()
    He, HLe, ste, pre = _host(eager)
    g = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=True, use_graph=True,
                deterministic=True)
    assert eager.info()["fixed_point"] == 1 and g.info()["fixed_point"] == 1
    for rep in range(3):
        g.run()
        torch.cuda.synchronize()
        Hg, HLg, stg, prg = _host(g)
        assert np.array_equal(Hg, He) and np.array_equal(HLg, HLe), rep
        assert np.array_equal(prg["rt60"], pre["rt60"]) and np.array_equal(prg["status"], pre["status"])
        assert np.array_equal(prg["rt60_range"], pre["rt60_range"])
        eager.run()
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
    # the same pairs accumulated in FP32 agree within 1e-5 of each row
    f = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=False)
    f.run()
    torch.cuda.synchronize()
    Hf = f.hist.double().cpu().numpy()
    for i in range(len(pairs)):
        assert_hist_close(He[i], Hf[i], tol=1e-5, what=f"pair {i}")
    for b in (g, eager, f):
        b.close()
