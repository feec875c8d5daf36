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


# ------------------------------------------------ in-frame rule (trace_ir with a segment budget)
from oracle.budget import frame_ray_count  # noqa: E402


def test_frame_rule_closed_box_gives_budget_over_k_plus_one():
    """Every ray of a closed box lives to the bounce limit: S0 = N0 (K + 1),
    and N0 + floor((B - S0) N0 / S0) = floor(B / (K + 1))."""
    c = R.tiny_config()
    K = 20
    segs, rays = _segments(c, c["sources"], c["listener"], 512, K, 1)
    assert segs == rays * (K + 1)
    for budget in (segs, segs + 1, 100_000, 123_457):
        assert frame_ray_count(budget, segs, rays, 10**9) == budget // (K + 1)


def test_frame_rule_open_box_fills_the_budget():
    """With escapes the first pass's segments per ray are below K + 1; the
    frame's rays [0, N') trace the budget within the sampling spread of the
    added rays' segment counts, and more rays than a closed box would take."""
    verts, tris, tm = R.merge(R.box_surfaces((0, 0, 0), (10, 7, 3), faces=("x0", "x1", "y0", "z0")), [0] * 4)
    sd = dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.full((1, 4), 0.1, np.float32),
              scattering=np.full((1, 4), 0.5, np.float32))
    src, lst, K, budget, n0 = np.array([[2.0, 2.0, 1.5]]), np.array([7.0, 5.0, 1.5]), 30, 60_000, 1024
    s0, _ = _segments(sd, src, lst, n0, K, 2)
    n1 = frame_ray_count(budget, s0, n0, 10**9)
    assert n1 > budget // (K + 1) and n1 > n0
    r = oracle.trace_ir(sd, src, lst, 0.5, n_rays_total=n1, max_bounces=K, sh_order=0, n_bins=4000,
                        bin_width_s=1e-3, seed=2, want_hash=False)
    segs = r["stats"][0]["n_segments"]
    # the first N0 rays are the same rays: only the n1 - n0 added ones are random
    assert abs(segs - budget) <= 5 * (K + 1) / 2 * math.sqrt(n1 - n0) + s0 / n0, (segs, budget)


def test_frame_rule_edges():
    assert frame_ray_count(1000, 1000, 100, 10**6) == 100  # budget met by the first pass
    assert frame_ray_count(500, 1000, 100, 10**6) == 100  # first pass over the budget: no more rays
    assert frame_ray_count(1000, 0, 100, 10**6) == 100  # no segments measured
    assert frame_ray_count(10**6, 1000, 100, 150) == 150  # clamped to max_rays
    assert frame_ray_count(1999, 1000, 100, 10**6) == 199  # floor, at the first pass's rate
