"""Segment budget per frame, FP64 / integer reference (Section 5: every frame
traces the same number of ray segments; rays that escape early leave budget
for more primary rays).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library,
with which it shares no code.

Reading: the serial rule (start rays in order until the budget is spent) is
a sequential prefix over per-ray segment counts that a parallel trace cannot
evaluate before tracing.  The frame instead traces N' rays, each with
1/N' of the source energy, where N' makes the previous frame's measured
segments per ray fill the budget:
    N' = clamp(floor(budget * prev_rays / prev_segments), min_rays, max_rays),
and the first frame (no previous measurement) traces max(min_rays,
min(nominal, max_rays)) rays.  Parity pins: tests/test_oracle_budget.py.
"""
from __future__ import annotations


def budget_ray_count(budget_segments: int, prev_segments: int, prev_rays: int, min_rays: int, max_rays: int,
                     nominal: int) -> int:
    if prev_segments <= 0 or prev_rays <= 0:
        n = nominal
    else:
        n = (budget_segments * prev_rays) // prev_segments
    return int(max(min_rays, min(n, max_rays)))


def frame_ray_count(budget_segments: int, first_segments: int, first_rays: int, max_rays: int) -> int:
    """Rays of a source within one frame (the in-call budget of trace_ir).

    Reading: the serial rule (start rays in order until the budget is spent)
    is evaluated in two passes.  The frame first traces N0 = first_rays
    rays; their segment count S0 measures this frame's segments per ray, and
    the frame then adds the rays that are expected to fill the rest of the
    budget at that rate:
        N' = clamp(N0 + floor((B - S0) * N0 / S0), N0, max_rays),
    with no further rays when S0 >= B.  Each of the N' rays carries 1/N' of
    the source energy.  Parity pins: tests/test_oracle_budget.py."""
    n0 = int(first_rays)
    if first_segments <= 0 or budget_segments <= first_segments:
        return n0
    dn = (int(budget_segments) - int(first_segments)) * n0 // int(first_segments)
    return int(min(n0 + dn, int(max_rays)))
