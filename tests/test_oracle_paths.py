"""Pins of the oracle's early-reflection paths (Section 5: orders 1-2 with
the diffuse path cache and SH directivity per path; the prioritization that
renders the N_ER strongest paths and adds the rest to the late IR) against
facts fixed outside them: the records hold exactly the early class of the
trace, a specular shoebox's order-1 and order-2 paths are its image sources
(energy, arrival time and direction per wall), the cache follows the closed
form of exponential smoothing per path, and the selection keeps the
strongest paths and conserves the energy it moves.  CPU-only."""
import math

import numpy as np
import pytest

import rpr_scenes as R
from oracle import paths as OP
from test_oracle_pins import C_SOUND, _direct_energy, _mean_se

FACES = ("x0", "x1", "y0", "y1", "z0", "z1")


def _trace(orc, scene, n, seed, **kw):
    c = R.tiny_config()
    args = dict(max_bounces=2, sh_order=1, n_bins=200, bin_width_s=1e-3, seed=seed)
    args.update(kw)
    return OP.trace_paths(scene, c["sources"], c["listener"], c["radius"], n_rays_total=n, **args)


def test_records_hold_the_early_class_exactly(orc):
    """Scattering box, K = 5: the records' band intensities sum to the
    trace's early class (orders 1-2), per source, and their directivity to
    the early part of the histogram's SH coefficients; no record comes from
    the direct or late segments."""
    c = R.tiny_config()
    r = _trace(orc, c, 8192, 3, max_bounces=5)
    for s in range(len(c["sources"])):
        paths = OP.aggregate(r["records"][s:s + 1], 4, 4)
        e = sum(p["e"] for p in paths.values())
        assert np.allclose(e, r["stats"][s]["e_class"][1], rtol=1e-12, atol=0)
        assert all(k[1] in (1, 2) for k in paths)
        assert all((k[1] == 1) == (k[3] == -1) for k in paths)
    rec = r["records"]
    assert np.all(rec[..., 0][rec[..., 0] != 0] == 1)
    assert set(np.unique(rec[..., 1][rec[..., 0] == 1])) <= {1.0, 2.0}
    # the same rays with K = 2 and K = 0: the difference of the histograms is
    # the early part, whose SH coefficients summed over time and bands are
    # the records' directivities
    r2 = _trace(orc, c, 8192, 3, max_bounces=2)
    r0 = _trace(orc, c, 8192, 3, max_bounces=0)
    early = (r2["hist"] - r0["hist"]).sum(axis=(1, 2))  # [S][NC]
    d = np.array([sum((p["d"] for p in OP.aggregate(r2["records"][s:s + 1], 4, 4).values()), np.zeros(4))
                  for s in range(len(c["sources"]))])
    assert np.allclose(d, early, rtol=1e-10, atol=1e-14 * np.abs(early).max())


def _face_of(tri):
    return FACES[tri // 2]


def _image(src, face, dims):
    p = np.array(src, np.float64)
    a = "xyz".index(face[0])
    p[a] = -p[a] if face[1] == "0" else 2 * dims[a] - p[a]
    return p


def test_specular_shoebox_paths_are_image_sources(orc):
    """Scattering 0: the order-1 paths off each wall (its two triangles) carry
    the energy of that wall's image source, (1 - alpha) times the direct
    energy of a ball at the image distance; they arrive at the image
    distance over c (within the ball's radius) from the image's direction.
    The order-2 paths off each ordered pair of walls carry the energy of the
    corresponding second-order image."""
    c = R.tiny_config()
    sc = dict(c, scattering=np.zeros((1, 4), np.float32))
    dims = np.array([10.0, 7.0, 3.0])
    src, lp, rad = c["sources"][0].astype(np.float64), c["listener"].astype(np.float64), c["radius"]
    alpha = c["absorption"][0].astype(np.float64)
    n, nb = 2**20, 16
    runs = [OP.trace_paths(sc, src[None], lp, rad, n_rays_total=n, ray_begin=i * (n // nb),
                           ray_end=(i + 1) * (n // nb), max_bounces=2, sh_order=1, n_bins=200, bin_width_s=1e-3,
                           seed=31) for i in range(nb)]
    per_run = [OP.aggregate(r["records"], 4, 4) for r in runs]
    for f in FACES:
        img = _image(src, f, dims)
        dist = float(np.linalg.norm(img - lp))
        es = [sum((p["e"] for k, p in P.items() if k[1] == 1 and _face_of(k[2]) == f), np.zeros(4)) for P in per_run]
        e, se = _mean_se(es)
        ref = (1 - alpha) * _direct_energy(dist, rad)
        assert np.all(np.abs(e - ref) < 5 * se + 1e-12 * ref), (f, e, ref, se)
        tot = {k: p for P in per_run for k, p in P.items() if k[1] == 1 and _face_of(k[2]) == f}
        et = sum(p["et"] for p in tot.values()) / sum(p["e"].sum() for p in tot.values())
        assert abs(et - dist / C_SOUND) < rad / C_SOUND, (f, et, dist / C_SOUND)
        d = sum(p["d"] for p in tot.values())
        v = np.array([-d[3], -d[1], d[2]])  # (-X_11, -X_1-1, X_10) points at the arrival
        u = (img - lp) / dist
        assert np.dot(v / np.linalg.norm(v), u) > 1 - 2 * (rad / dist) ** 2, f
    # second order.  Two parallel walls give two images, one per order of the
    # walls; two perpendicular walls give one image (both orders land on the
    # same point), reached in the one order the geometry allows, so the pair's
    # paths in both orders together carry its energy.
    for i1, f1 in enumerate(FACES):
        for f2 in FACES[i1 + 1:]:
            orders = [(f1, f2), (f2, f1)] if f1[0] == f2[0] else [((f1, f2), (f2, f1))]
            for o in orders:
                seqs = o if isinstance(o[0], tuple) else (o,)
                img = _image(_image(src, seqs[0][0], dims), seqs[0][1], dims)
                dist = float(np.linalg.norm(img - lp))
                es = [sum((p["e"] for k, p in P.items()
                           if k[1] == 2 and (_face_of(k[2]), _face_of(k[3])) in seqs), np.zeros(4)) for P in per_run]
                e, se = _mean_se(es)
                ref = (1 - alpha) ** 2 * _direct_energy(dist, rad)
                assert np.all(np.abs(e - ref) < 5 * se + 1e-12 * ref), (seqs, e, ref, se)
                assert np.all(se < 0.25 * ref), (seqs, se, ref)  # enough hits for the test to bite


def _p(e, t, d):
    e = np.asarray(e, np.float64)
    return dict(e=e, et=e.sum() * t, d=np.asarray(d, np.float64))


def test_cache_is_exponential_smoothing_per_path():
    """A path seen every frame is a fixed point; one seen once decays by
    (1 - alpha) per frame and leaves the cache below min_energy; a path
    appearing later grows as 1 - (1 - alpha)^n; the first frame copies."""
    a, emin = 0.3, 1e-3
    A = (0, 1, 5, -1)
    Bk = (0, 2, 5, 7)
    Ck = (1, 1, 9, -1)
    f1 = {A: _p([1.0, 2.0], 0.01, [1.0, 0.5]), Bk: _p([0.5, 0.5], 0.02, [1.0, 0.0])}
    c = OP.cache_update({A: _p([9, 9], 1, [9, 9])}, f1, a, emin, first=True)
    assert set(c) == {A, Bk} and np.array_equal(c[A]["e"], f1[A]["e"])
    for n in range(1, 25):
        fresh = {A: f1[A], Ck: _p([0.2, 0.1], 0.03, [0.3, 0.0])}
        c = OP.cache_update(c, fresh, a, emin, first=False)
        assert np.allclose(c[A]["e"], [1.0, 2.0], rtol=1e-14) and abs(c[A]["et"] - 0.03) < 1e-15
        assert np.allclose(c[Ck]["e"], np.array([0.2, 0.1]) * (1 - (1 - a) ** n), rtol=1e-12)
        if 1.0 * (1 - a) ** n >= emin:
            assert np.allclose(c[Bk]["e"], np.array([0.5, 0.5]) * (1 - a) ** n, rtol=1e-12)
            assert np.allclose(c[Bk]["d"], np.array([1.0, 0.0]) * (1 - a) ** n, rtol=1e-12)
        else:
            assert Bk not in c
    # the arrival time of a cached path is its intensity-weighted mean
    assert abs(c[Ck]["et"] / c[Ck]["e"].sum() - 0.03) < 1e-14


def test_selection_keeps_the_strongest_and_moves_the_rest_to_the_late_class():
    """The N_ER strongest paths over all sources are rendered, strongest
    first; paths below the threshold are dropped; the others join the late
    class of their source at the bin of their mean arrival time, and the
    total intensity of each source's early + late classes is unchanged."""
    rng = np.random.default_rng(7)
    S, T, B, dt = 3, 50, 4, 0.01
    paths = {}
    for i in range(40):
        s = int(rng.integers(0, S))
        key = (s, int(rng.integers(1, 3)), i, -1)
        paths[key] = _p(rng.uniform(0, 1, B) * 10.0 ** rng.uniform(-4, 0), rng.uniform(0, (T - 0.5) * dt), np.zeros(4))
    hl = rng.uniform(0, 1, (S, T, B))
    ec = rng.uniform(1, 2, (S, 3, B))
    hl0, ec0 = hl.copy(), ec.copy()
    thr, n_er = 1e-3, 12
    out = OP.select(paths, thr, n_er, hl, ec, dt)
    tot = {k: v["e"].sum() for k, v in paths.items()}
    eligible = sorted((k for k in paths if tot[k] >= thr), key=lambda k: -tot[k])
    assert [k for k, _ in out] == eligible[:n_er]
    assert all(tot[out[i][0]] >= tot[out[i + 1][0]] for i in range(len(out) - 1))
    culled = eligible[n_er:]
    want = hl0.copy()
    moved = np.zeros((S, B))
    for k in culled:
        m = int(paths[k]["et"] / tot[k] / dt)
        want[k[0], m] += paths[k]["e"]
        moved[k[0]] += paths[k]["e"]
    assert np.allclose(hl, want, rtol=1e-14)
    assert np.allclose(ec[:, 1], ec0[:, 1] - moved) and np.allclose(ec[:, 2], ec0[:, 2] + moved)
    assert np.allclose(ec[:, 1] + ec[:, 2], ec0[:, 1] + ec0[:, 2])
    # fewer eligible paths than N_ER: all rendered, nothing moved
    hl2, ec2 = hl0.copy(), ec0.copy()
    out2 = OP.select(paths, thr, 1000, hl2, ec2, dt)
    assert len(out2) == len(eligible) and np.array_equal(hl2, hl0) and np.array_equal(ec2, ec0)
