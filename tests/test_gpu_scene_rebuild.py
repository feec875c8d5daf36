"""scene_rebuild against scene_create: a scene rebuilt in place from new
geometry must be the scene that scene_create makes from it.  Checked through
every closest hit of 20,000 random rays (distance and triangle, exactly), the
scene information and a deterministic trace (histograms bit for bit, every
ray's path hash), over a sequence of rebuilds that grows the scene, shrinks
it within its arrays, empties it, fails on a bad vertex index (reported by the
next call that uses the scene; the scene is then empty) and fills it again.
The rebuild is asynchronous: the first call after it (a closest-hit query, a
trace, scene_wait) waits for it."""
import numpy as np
import pytest

import paper_1803_00430_amd as P
import rpr_scenes as R

pytestmark = pytest.mark.gpu


def _soup(n, seed, spread=20.0):
    g = np.random.default_rng(seed)
    c = g.uniform(-spread, spread, (n, 3)).astype(np.float32)
    v = (c[:, None, :] + g.normal(0, 0.7, (n, 3, 3))).astype(np.float32).reshape(-1, 3)
    nm = 3
    return dict(verts=v, tris=np.arange(3 * n, dtype=np.int32).reshape(n, 3),
                tri_mat=g.integers(0, nm, n).astype(np.int32),
                absorption=g.uniform(0.05, 0.6, (nm, 4)).astype(np.float32),
                scattering=g.uniform(0.0, 0.9, (nm, 4)).astype(np.float32))


def _args(d):
    return d["verts"], d["tris"], d.get("tri_mat"), d["absorption"], d["scattering"]


def _hits(scene, rays):
    t, tri = scene.closest_hit(*rays)
    return t.cpu().numpy(), tri.cpu().numpy()


def _trace(scene, src, lst):
    import torch
    T, n = 200, 2
    hist, late, stats, rh = P.alloc_trace_outputs(1, T, scene.n_bands, n, 4096, want_hash=True)
    prm = P.trace_params(n_rays_total=4096, max_bounces=30, sh_order=n, n_bins=T, bin_width_s=2e-3, seed=77,
                         flags=P.TRACE_DETERMINISTIC)
    P.trace_ir(scene, np.asarray([src], np.float32), lst, 1.0, prm, hist, late, stats, rh)
    torch.cuda.synchronize()
    return hist.cpu().numpy(), late.cpu().numpy(), rh.cpu().numpy()


def _same_scene(rebuilt, d, rays, src, lst):
    fresh = P.Scene(*_args(d))
    try:
        (t0, i0), (t1, i1) = _hits(rebuilt, rays), _hits(fresh, rays)
        assert rebuilt.info() == fresh.info()
        assert np.array_equal(i0, i1)
        assert np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
        if len(d["tris"]):
            assert (i0 >= 0).any()
        for a, b in zip(_trace(rebuilt, src, lst), _trace(fresh, src, lst)):
            assert np.array_equal(a, b)
    finally:
        fresh.close()


def test_rebuild_in_place_equals_a_fresh_scene():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    rays = R.random_rays(5, 20000, [-22, -22, -22], [22, 22, 22])
    src, lst = [0.5, -1.0, 2.0], [-3.0, 2.0, 1.0]
    small, big, tiny = _soup(2000, 1), _soup(6000, 2), R.tiny_config()
    sc = P.Scene(*_args(small))
    try:
        _same_scene(sc, small, rays, src, lst)
        sc.rebuild(*_args(big))                 # grows its arrays
        _same_scene(sc, big, rays, src, lst)
        sc.rebuild(*_args(tiny))                # fits: no allocation
        _same_scene(sc, tiny, rays, src, lst)
        sc.rebuild(*_args(big))                 # a trace is the first call after the rebuild
        fresh = P.Scene(*_args(big))
        for a, b in zip(_trace(sc, src, lst), _trace(fresh, src, lst)):
            assert np.array_equal(a, b)
        fresh.close()
        sc.rebuild(*_args(small))               # two rebuilds in a row: the second replaces the first
        sc.rebuild(*_args(tiny))
        _same_scene(sc, tiny, rays, src, lst)
        empty = dict(big, tris=np.zeros((0, 3), np.int32), tri_mat=np.zeros(0, np.int32))
        sc.rebuild(*_args(empty))
        info = sc.info()
        assert info["n_tris"] == 0 and info["n_nodes"] == 0
        assert (_hits(sc, rays)[1] == -1).all()
        bad = dict(big, tris=big["tris"].copy())
        bad["tris"][123, 2] = 10 ** 7
        sc.rebuild(*_args(bad))                 # enqueued: the device finds the bad index
        with pytest.raises(RuntimeError, match="scene_rebuild: vertex index out of range"):
            sc.wait()
        sc.wait()                               # reported once
        assert sc.info()["n_tris"] == 0
        assert (_hits(sc, rays)[1] == -1).all()
        sc.rebuild(*_args(bad))
        with pytest.raises(RuntimeError, match="scene_rebuild: vertex index out of range"):
            _hits(sc, rays)                     # or by the next call that uses the scene
        sc.rebuild(*_args(big))                 # fits again
        _same_scene(sc, big, rays, src, lst)
    finally:
        sc.close()


def test_pipelined_rebuilds_match_serial():
    """The benchmark's step pattern: three streams, one scene per stream
    rebuilt in place each step, step i+1's rebuild enqueued before step i's
    trace.  In deterministic accumulation every step's histograms and path
    hashes equal those of a scene built and traced alone, bit for bit, and its
    counts are equal."""
    import torch
    cfg = R.city_config()
    n_rays, S = 4096, len(cfg["sources"])
    T, n, B = cfg["n_bins"], cfg["sh_order"], cfg["absorption"].shape[1]
    prm = P.trace_params(n_rays_total=n_rays, max_bounces=cfg["max_bounces"], sh_order=n, n_bins=T,
                         bin_width_s=cfg["bin_width_s"], seed=cfg["seed"], flags=P.TRACE_DETERMINISTIC)
    dev = torch.device("cuda:0")
    inputs = [torch.as_tensor(np.asarray(cfg[k]), device=dev)
              for k in ("verts", "tris", "tri_mat", "absorption", "scattering")]

    def outputs():
        h, l_, s, rh = P.alloc_trace_outputs(S, T, B, n, n_rays, want_hash=True)
        return h, l_, s, rh

    ref_sc = P.Scene(*inputs)
    ref = outputs()
    P.trace_ir(ref_sc, cfg["sources"], cfg["listener"], cfg["radius"], prm, *ref)
    torch.cuda.synchronize()
    ref_np = [x.cpu().numpy() for x in (ref[0], ref[1], ref[3])]
    ref_st = P.stats_host(ref[2])
    ref_sc.close()

    n_pipe, steps = 3, 7
    streams = [torch.cuda.Stream() for _ in range(n_pipe)]
    scenes = [P.Scene(*inputs) for _ in range(n_pipe)]
    outs = [outputs() for _ in range(steps)]
    torch.cuda.synchronize()  # inputs and outputs made on the default stream, used on the others

    def rebuild(i):
        with torch.cuda.stream(streams[i % n_pipe]):
            scenes[i % n_pipe].rebuild(*inputs)

    rebuild(0)
    for i in range(steps):
        if i + 1 < steps:
            rebuild(i + 1)
        with torch.cuda.stream(streams[i % n_pipe]):
            P.trace_ir(scenes[i % n_pipe], cfg["sources"], cfg["listener"], cfg["radius"], prm, *outs[i])
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        got = [x.cpu().numpy() for x in (o[0], o[1], o[3])]
        for a, b in zip(got, ref_np):
            assert np.array_equal(a, b), i
        st = P.stats_host(o[2])
        for s in range(S):
            for key in ("n_segments", "n_finite_segments", "n_escaped", "n_rays", "first_arrival_bin"):
                assert st[s][key] == ref_st[s][key], (i, s, key)
    for sc in scenes:
        sc.close()
