"""Pins of the segment-budget rule against facts of the traced scenes: in a
closed box every ray lives to the bounce limit, so N' = budget / (K + 1)
exactly; in an open box the measured segments per ray fall, N' rises, and the
next frame's segments land on the budget within the sampling spread of the
per-ray segment count.  CPU-only (the oracle tracer counts the segments)."""
import math

import numpy as np

import oracle
import rpr_scenes as R
from oracle.budget import budget_ray_count


def _segments(sd, src, lst, n, K, seed):
    r = oracle.trace_ir(sd, src, lst, 0.5, n_rays_total=n, max_bounces=K, sh_order=0, n_bins=4000,
                        bin_width_s=1e-3, seed=seed)
    return sum(s["n_segments"] for s in r["stats"]), n


def test_closed_box_gives_budget_over_k_plus_one():
    c = R.tiny_config()
    K = 20
    segs, rays = _segments(c, c["sources"], c["listener"], 512, K, 1)
    assert segs == rays * (K + 1)  # closed room, long window: no escapes
    budget = 100_000
    assert budget_ray_count(budget, segs, rays, 1, 10**9, 512) == budget // (K + 1)


def test_open_box_budget_is_met_by_the_next_frame():
    verts, tris, tm = R.merge(R.box_surfaces((0, 0, 0), (10, 7, 3), faces=("x0", "x1", "y0", "z0")), [0] * 4)
    sd = dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.full((1, 4), 0.1, np.float32),
              scattering=np.full((1, 4), 0.5, np.float32))
    src, lst, K, budget = np.array([[2.0, 2.0, 1.5]]), np.array([7.0, 5.0, 1.5]), 30, 60_000
    segs0, rays0 = _segments(sd, src, lst, 2048, K, 2)
    assert segs0 < rays0 * (K + 1)  # rays escape
    n1 = budget_ray_count(budget, segs0, rays0, 64, 10**9, 2048)
    assert n1 > budget // (K + 1)  # escaped rays leave room for more primary rays
    r = oracle.trace_ir(sd, src, lst, 0.5, n_rays_total=n1, max_bounces=K, sh_order=0, n_bins=4000,
                        bin_width_s=1e-3, seed=3, want_hash=False)
    segs1 = r["stats"][0]["n_segments"]
    # segments per ray have a spread of at most K + 1; the frame's total is within 5 standard errors
    per = segs0 / rays0
    sd_bound = (K + 1) / 2
    assert abs(segs1 - budget) <= 5 * sd_bound * math.sqrt(n1) + per, (segs1, budget)


def test_first_frame_and_clamps():
    assert budget_ray_count(1000, 0, 0, 10, 500, 300) == 300
    assert budget_ray_count(1000, 0, 0, 10, 200, 300) == 200
    assert budget_ray_count(1000, 10**6, 10, 50, 500, 300) == 50
    assert budget_ray_count(10**9, 10, 10, 50, 500, 300) == 500
