"""The batched persistent launch against the FP64 oracle, pair by pair.

A batch of pairs over four scenes (the tiny shoebox, an L-shaped room, a
cluttered box-cluster interior and a tessellated shoebox; 12 to 19,332
triangles) with ragged ray counts and bounce limits is traced in one launch,
in every queue order, by both methods, and each pair's histogram, statistics
and reverb parameters are compared with the oracle tracing that pair alone:
histograms within 1e-4 of each (band, coefficient) row, RT60 within 1%.

The batch writes no per-ray path hashes, so the rays whose discrete path
differs between the two sides are found by tracing the pair alone through
trace_ir / trace_listener with hashes (the batch equals those per pair, see
test_gpu_batch.py) and are then traced one by one on both sides and removed
from the batch's and the oracle's results."""
import numpy as np
import pytest

import oracle
import paper_1803_00430_amd as P
import rpr_scenes as R
from parity import (HIST_TOL, RT60_TOL, assert_hist_close, f32, gpu_trace, gpu_trace_listener, oracle_kw)

pytestmark = pytest.mark.gpu

T, NSH, DT = 400, 3, 1e-3


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    tiny = R.tiny_config()
    dicts = [tiny, R.batch_scene(103, n_pairs=2), R.batch_scene(107, n_pairs=2), R.batch_scene(108, n_pairs=2)]
    scenes = [P.Scene.from_dict(d) for d in dicts]
    g = R.rng(11)
    pairs = [dict(scene=0, source=tiny["sources"][0], listener=tiny["listener"], radius=0.5, n_rays=1111,
                  max_bounces=50, seed=2000, pair_id=0)]
    for si, d in enumerate(dicts[1:], start=1):
        for p in d["pairs"]:
            k = len(pairs)
            pairs.append(dict(scene=si, source=p["source"], listener=p["listener"], radius=p["radius"],
                              n_rays=int(g.integers(300, 1700)), max_bounces=int(g.integers(50, 201)),
                              seed=2000 + 7 * k, pair_id=k))
    return dicts, scenes, pairs


def _kw(p):
    return dict(n_rays_total=p["n_rays"], max_bounces=p["max_bounces"], sh_order=NSH, n_bins=T, bin_width_s=DT,
                seed=p["seed"], pair_base=p["pair_id"])


def _one_ray(kw, i):
    return dict(kw, ray_begin=i, ray_end=i + 1)


@pytest.fixture(scope="module")
def reference(setup):
    """Per pair and method: the oracle's result, and the divergent rays'
    single-ray traces on both sides."""
    dicts, scenes, pairs = setup
    out = {}
    for method in ("source", "listener"):
        refs = []
        for p in pairs:
            sd, sc, kw = dicts[p["scene"]], scenes[p["scene"]], _kw(p)
            src = np.asarray(p["source"], np.float32)[None]
            if method == "source":
                g = gpu_trace(sc, src, p["listener"], p["radius"], **kw)
                o = oracle.trace_ir(sd, src, p["listener"], f32(p["radius"]), want_hash=True, **oracle_kw(kw))
                gone = lambda i: gpu_trace(sc, src, p["listener"], p["radius"], **_one_ray(kw, i))
                oone = lambda i: oracle.trace_ir(sd, src, p["listener"], f32(p["radius"]),
                                                 **oracle_kw(_one_ray(kw, i)))
                div = np.flatnonzero(g["ray_hash"][0] != o["ray_hash"][0])
            else:
                g = gpu_trace_listener(sc, src, p["listener"], p["radius"], **kw)
                o = oracle.trace_listener(sd, src, p["listener"], f32(p["radius"]), want_hash=True,
                                          **oracle_kw(kw))
                gone = lambda i: gpu_trace_listener(sc, src, p["listener"], p["radius"], **_one_ray(kw, i))
                oone = lambda i: oracle.trace_listener(sd, src, p["listener"], f32(p["radius"]),
                                                       **oracle_kw(_one_ray(kw, i)))
                div = np.flatnonzero(g["ray_hash"] != o["ray_hash"])
            rm_g = [gone(int(i)) for i in div]
            rm_o = [oone(int(i)) for i in div]
            refs.append(dict(o=o, div=div, rm_g=rm_g, rm_o=rm_o))
        n_div = sum(len(r["div"]) for r in refs)
        n_all = sum(p["n_rays"] for p in pairs)
        print(f"[parity] batch {method}: {n_div} of {n_all} rays took another discrete path on the two sides")
        out[method] = refs
    return out


def _run_batch(scenes, pairs, method, order, wpc, chunk=0, use_graph=False):
    import torch
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=False, use_graph=use_graph,
                order=order, waves_per_cu=wpc, method=method, chunk_rays=chunk)
    b.run()
    torch.cuda.synchronize()
    res = (b.hist.double().cpu().numpy(), b.hist_late.double().cpu().numpy(), P.stats_host(b.stats),
           P.params_host(b.params))
    b.close()
    return res


@pytest.mark.parametrize("method,order,wpc,chunk", [("source", 0, 0, 0), ("source", 1, 2, 0), ("source", 2, 0, 256),
                                                    ("listener", 0, 0, 0), ("listener", 2, 3, 4096)])
def test_batch_pairs_match_oracle(setup, reference, method, order, wpc, chunk):
    dicts, scenes, pairs = setup
    H, HL, st, prm = _run_batch(scenes, pairs, method, order, wpc, chunk)
    refs = reference[method]
    # the source-origin trace follows the oracle's paths (FP64 ray state); the
    # listener-origin trace keeps an FP32 ray state and splits more often
    max_div = 1e-3 if method == "source" else 5e-3
    assert sum(len(r["div"]) for r in refs) <= max_div * sum(p["n_rays"] for p in pairs)
    for i, (p, r) in enumerate(zip(pairs, refs)):
        o = r["o"]
        Hg, HLg, Ho, HLo = H[i].copy(), HL[i].copy(), o["hist"][0].copy(), o["hist_late"][0].copy()
        for g1, o1 in zip(r["rm_g"], r["rm_o"]):
            Hg -= g1["hist"][0]
            HLg -= g1["hist_late"][0]
            Ho -= o1["hist"][0]
            HLo -= o1["hist_late"][0]
        assert_hist_close(Hg, Ho, what=f"{method} order {order} pair {i}")
        assert_hist_close(HLg, HLo, what=f"{method} order {order} pair {i} late")
        os_ = o["stats"][0]
        assert st[i]["n_rays"] == os_["n_rays"] == p["n_rays"]
        if len(r["div"]) == 0:
            for key in ("n_segments", "n_finite_segments", "n_escaped"):
                assert st[i][key] == os_[key], (i, key, st[i][key], os_[key])
            assert abs(st[i]["seg_len_sum"] - os_["seg_len_sum"]) <= 1e-5 * os_["seg_len_sum"]
            scale = np.abs(np.asarray(os_["e_class"])).max(axis=0)[:4] + 1e-30
            assert np.all(np.abs(np.asarray(st[i]["e_class"])[:, :4] - np.asarray(os_["e_class"])[:, :4])
                          <= HIST_TOL * scale)
            # RT60 of the batch's estimate step against the oracle's estimate of
            # the oracle's histogram: within 1%, from the same fit range
            po = oracle.estimate_reverb(o["hist"][0], o["hist_late"][0], os_, f32(DT))
            ok = po["rt60"] > 0
            assert np.array_equal(prm[i]["rt60_range"][:4][ok], po["rt60_range"][ok]), i
            assert np.all(np.abs(prm[i]["rt60"][:4][ok] - po["rt60"][ok]) <= RT60_TOL * po["rt60"][ok]), \
                (i, prm[i]["rt60"][:4], po["rt60"])


def test_batch_graph_replay_matches_oracle(setup, reference):
    """A graph replay of the source-origin batch (the launch the benchmark
    times), autotuned, against the oracle on every pair."""
    import torch
    dicts, scenes, pairs = setup
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=NSH, bin_width_s=DT, autotune=True, use_graph=True)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    H = b.hist.double().cpu().numpy()
    for i, r in enumerate(reference["source"]):
        Hg, Ho = H[i].copy(), r["o"]["hist"][0].copy()
        for g1, o1 in zip(r["rm_g"], r["rm_o"]):
            Hg -= g1["hist"][0]
            Ho -= o1["hist"][0]
        assert_hist_close(Hg, Ho, what=f"replay pair {i}")
    b.close()
