"""GPU parity of the listener-origin trace with next-event estimation
(`trace_listener`) against the FP64 oracle, through the C ABI.

Tolerances as for the source-origin trace: histograms within 1e-4 of each
bin-band-coefficient row's absolute sum, RT60 within 1%.  At the city's full
size one ray can carry most of a row (a reflection close to a source ball),
and its FP32 arrival time drifts from the FP64 one by about 6e-6 relative
(0.7 mm over 124 m and 8 segments, measured) without any change of its hit
sequence; there cells also get the timing allowance of
`assert_hist_close(time_rel=1e-5)`, while row sums keep the 1e-4 bar.  These
kernels keep an FP32 ray state; the closest hit of each segment is still
decided by the FP64 triangle test.  Rays whose discrete path differs between
the two sides (hit triangles, bounce kinds, and here also the outcome of
every occlusion query) are traced again alone on both sides and removed;
each test allows 0.5% and states what was measured."""
import math

import numpy as np
import pytest

import oracle
import paper_1803_00430_amd as P
import rpr_scenes as R
from parity import RT60_TOL, assert_hist_close, assert_stats_close, gpu_trace_listener, traced_listener_pair
from test_gpu_trace import _cluttered_room

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


def _tiny_kw(c, **over):
    kw = dict(n_rays_total=c["n_rays"], max_bounces=c["max_bounces"], sh_order=c["sh_order"],
              n_bins=c["n_bins"], bin_width_s=c["bin_width_s"], seed=c["seed"])
    kw.update(over)
    return kw


def test_listener_tiny_parity(torch_cuda):
    """The tiny shoebox (4096 rays, 50 bounces, 2000 x 1 ms, SH order 2),
    traced from the listener point with the source as a 0.5 m ball."""
    c = R.tiny_config()
    sc = P.Scene.from_dict(c)
    kw = _tiny_kw(c)
    g, o, div = traced_listener_pair(sc, c, c["sources"], c["listener"], c["radius"], **kw)
    print(f"divergent rays: {len(div)} of {c['n_rays']}")
    assert len(div) <= 0.005 * c["n_rays"], len(div)  # measured 4 of 4096
    assert_hist_close(g["hist"][0], o["hist"][0])
    assert_hist_close(g["hist_late"][0], o["hist_late"][0], what="hist_late")
    assert_stats_close(g["cmp_stats"][0], o["cmp_stats"][0])
    assert int(g["stats"][0]["n_next_event"]) > 0
    out = P.alloc_params(1)
    hist, late, stats = g["_dev"]
    P.estimate_reverb(hist, late, stats, c["n_bins"], 4, c["sh_order"], c["bin_width_s"], out)
    pg = P.params_host(out)[0]
    po = oracle.estimate_reverb(o["hist"][0], o["hist_late"][0], o["stats"][0], c["bin_width_s"])
    assert np.all(np.abs(pg["rt60"][:4] - po["rt60"]) <= RT60_TOL * po["rt60"])
    assert np.array_equal(pg["rt60_range"][:4], po["rt60_range"])


def test_listener_ragged_multisource_parity(torch_cuda):
    """Cluttered room (thousands of triangles, 3 materials), three sources
    of which boxes hide parts, a ray count that is not a multiple of the
    wave, SH order 3, a 250 ms window."""
    sd = _cluttered_room(7, n_boxes=25, edge=1.1)
    sc = P.Scene.from_dict(sd)
    srcs = np.array([[1.0, 1.0, 1.2], [6.0, 4.5, 2.0], [10.5, 8.0, 3.1]], np.float32)
    lst = np.array([5.0, 5.0, 1.6], np.float32)
    kw = dict(n_rays_total=1000, max_bounces=100, sh_order=3, n_bins=250, bin_width_s=1e-3, seed=78,
              pair_base=9)
    g, o, div = traced_listener_pair(sc, sd, srcs, lst, 0.6, **kw)
    print(f"divergent rays: {len(div)} of 1000")
    assert len(div) <= 0.005 * 1000, len(div)  # measured 0 of 1000
    for s in range(3):
        assert_hist_close(g["hist"][s], o["hist"][s], what=f"hist[{s}]")
        assert_hist_close(g["hist_late"][s], o["hist_late"][s], what=f"hist_late[{s}]")
        assert_stats_close(g["cmp_stats"][s], o["cmp_stats"][s])
        assert g["stats"][s]["first_arrival_bin"] == o["stats"][s]["first_arrival_bin"]


def test_listener_subsets_and_statistics(torch_cuda):
    """Disjoint ray ranges add up and keep their hashes; the path statistics
    are the same in every source's record."""
    sd = _cluttered_room(7, n_boxes=25, edge=1.1)
    sc = P.Scene.from_dict(sd)
    srcs = np.array([[1.0, 1.0, 1.2], [10.5, 8.0, 3.1]], np.float32)
    lst = np.array([5.0, 5.0, 1.6], np.float32)
    kw = dict(n_rays_total=3000, max_bounces=40, sh_order=1, n_bins=300, bin_width_s=1e-3, seed=5)
    full = gpu_trace_listener(sc, srcs, lst, 0.6, **kw)
    a = gpu_trace_listener(sc, srcs, lst, 0.6, ray_end=1111, **kw)
    b = gpu_trace_listener(sc, srcs, lst, 0.6, ray_begin=1111, **kw)
    assert np.array_equal(np.concatenate([a["ray_hash"], b["ray_hash"]]), full["ray_hash"])
    for s in range(2):
        assert_hist_close(a["hist"][s] + b["hist"][s], full["hist"][s], tol=1e-6)
    st = full["stats"]
    for k in ("n_segments", "n_escaped", "n_rays", "n_next_event", "seg_len_sum"):
        assert st[0][k] == st[1][k], k
    assert st[0]["n_rays"] == 3000


@pytest.mark.parametrize("scat", [[0.5, 0.5, 0.5, 0.5], [0.05, 0.35, 0.65, 0.95]])
def test_listener_zero_absorption_late_field(torch_cuda, scat):
    """Closed room without absorption: dt / V per bin in every band."""
    c = R.tiny_config()
    sd = dict(c, absorption=np.zeros((1, 4), np.float32), scattering=np.array([scat], np.float32))
    sc = P.Scene.from_dict(sd)
    g = gpu_trace_listener(sc, c["sources"], c["listener"], c["radius"],
                           **_tiny_kw(c, n_rays_total=65536, max_bounces=100000, sh_order=0), want_hash=False)
    I = math.sqrt(4 * math.pi) * g["hist"][0][:, :, 0]
    late = I[300:].mean(axis=0)
    assert np.all(np.abs(late / (1e-3 / 210.0) - 1) < 0.02), late


def test_listener_rejects_bad_arguments(torch_cuda):
    c = R.tiny_config()
    sc = P.Scene.from_dict(c)
    hist, late, stats, _ = P.alloc_trace_outputs(300, 100, 4, 1)
    prm = P.trace_params(n_rays_total=64, max_bounces=3, sh_order=1, n_bins=100, bin_width_s=1e-3, seed=0)
    with pytest.raises(P.RprError):
        P.trace_listener(sc, np.zeros((257, 3)), c["listener"], 0.5, prm, hist, late, stats)
    with pytest.raises(P.RprError):
        P.trace_listener(sc, c["sources"], c["listener"], 0.0, prm, hist, late, stats)
    bad = P.trace_params(n_rays_total=64, max_bounces=3, sh_order=1, n_bins=100, bin_width_s=1e-3, seed=0,
                         flags=1)
    with pytest.raises(P.RprError):
        P.trace_listener(sc, c["sources"], c["listener"], 0.5, bad, hist, late, stats)


def test_listener_batch_matches_single_pairs(torch_cuda):
    """A batch with method "listener" (one persistent launch over pairs in
    several scenes, replayed from a graph) gives every pair the histogram of
    trace_listener on that pair alone, up to the order of the FP32 atomic
    additions; one pair is also checked against the oracle."""
    rooms = [R.learn_room(200000 + i) for i in range(4)]
    scenes = [P.Scene.from_dict(r) for r in rooms]
    pairs = []
    for i, r in enumerate(rooms):
        for j in range(2 if i < 2 else 1):
            pairs.append(dict(scene=i, pair_id=10 + len(pairs), source=r["sources"][0] + 0.1 * j,
                              listener=r["listener"], radius=0.5, max_bounces=100 + 50 * j,
                              n_rays=333 + 250 * len(pairs), seed=(1 << 33) + 7 * len(pairs)))
    T, dt, n = 300, 1e-3, 3
    b = P.Batch(scenes, pairs, n_bins=T, sh_order=n, bin_width_s=dt, autotune=False, use_graph=True,
                method="listener")
    for _ in range(2):
        b.run()
    torch_cuda.cuda.synchronize()
    Hb = b.hist.double().cpu().numpy()
    stb = P.stats_host(b.stats)
    for k, p in enumerate(pairs):
        g = gpu_trace_listener(scenes[p["scene"]], p["source"][None], p["listener"], p["radius"],
                               n_rays_total=p["n_rays"], max_bounces=p["max_bounces"], sh_order=n, n_bins=T,
                               bin_width_s=dt, seed=p["seed"], pair_base=p["pair_id"], want_hash=False)
        assert_hist_close(Hb[k], g["hist"][0], tol=1e-5, what=f"pair {k}")
        for key in ("n_segments", "n_escaped", "n_rays", "n_next_event", "first_arrival_bin"):
            assert stb[k][key] == g["stats"][0][key], (k, key)
    p = pairs[0]
    kw = dict(n_rays_total=p["n_rays"], max_bounces=p["max_bounces"], sh_order=n, n_bins=T, bin_width_s=dt,
              seed=p["seed"], pair_base=p["pair_id"])
    g, o, div = traced_listener_pair(scenes[0], rooms[0], p["source"][None], p["listener"], p["radius"], **kw)
    assert len(div) <= 0.005 * p["n_rays"]  # measured 0 of 333
    assert_hist_close(g["hist"][0], o["hist"][0])
    b.close()


def test_listener_city_full_size_ray_subset(torch_cuda):
    """The city at full size (99,996 triangles, its 8 sources as 1 m balls
    heard at the listener point, 100 bounces, SH order 3, 3000 bins) traced
    from the listener, on a subset of absolute ray ids that the brute-force
    oracle can follow (every segment and every query against every
    triangle)."""
    c = R.city_config()
    sc = P.Scene.from_dict(c)
    kw = dict(n_rays_total=c["n_rays"], ray_begin=2000, ray_end=4048, max_bounces=c["max_bounces"],
              sh_order=c["sh_order"], n_bins=c["n_bins"], bin_width_s=c["bin_width_s"], seed=c["seed"])
    g, o, div = traced_listener_pair(sc, c, c["sources"], c["listener"], c["radius"], **kw)
    print(f"divergent rays: {len(div)} of 2048")
    assert len(div) <= 0.005 * 2048, len(div)  # measured 0 of 2048
    for s in range(8):
        Hg, Ho = g["hist"][s], o["hist"][s]
        row = np.abs(Ho).sum(0)
        rel = np.abs(Hg - Ho) / (row[None] + 1e-30)
        m, b, k = np.unravel_index(np.argmax(rel), rel.shape)
        print(f"source {s}: worst cell bin {m} band {b} coeff {k}: error {rel[m, b, k]:.2e} of the row; "
              f"that cell holds {abs(Ho[m, b, k]) / (row[b, k] + 1e-30):.2e} of it")
        assert_hist_close(Hg, Ho, what=f"hist[{s}]", time_rel=1e-5)
        assert_stats_close(g["cmp_stats"][s], o["cmp_stats"][s])
    assert sum(int(o["stats"][s]["first_arrival_bin"] < 3000) for s in range(8)) >= 4  # most sources heard


def test_listener_city_full_trace_invariants(torch_cuda):
    """The complete city traced from the listener (32,768 rays for all 8
    sources): the ray set's statistics repeat in every record, every
    histogram's energy equals its class energies, and the path statistics
    count every ray."""
    c = R.city_config()
    sc = P.Scene.from_dict(c)
    g = gpu_trace_listener(sc, c["sources"], c["listener"], c["radius"], n_rays_total=c["n_rays"],
                           max_bounces=c["max_bounces"], sh_order=c["sh_order"], n_bins=c["n_bins"],
                           bin_width_s=c["bin_width_s"], seed=c["seed"], want_hash=False)
    st = g["stats"]
    for s in range(8):
        assert st[s]["n_rays"] == c["n_rays"] and abs(st[s]["e_emitted"] - 1.0) < 1e-9
        assert st[s]["n_segments"] == st[s]["n_finite_segments"] + st[s]["n_escaped"]
        assert st[s]["n_next_event"] == st[0]["n_next_event"] > 0
        I = math.sqrt(4 * math.pi) * g["hist"][s][:, :, 0]
        assert np.allclose(I.sum(0), st[s]["e_class"][:, :4].sum(0), rtol=1e-4, atol=1e-15)
