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
