"""trace_ir with a segment budget (Section 5: the same number of ray path
segments every frame; rays that escape early leave budget for more primary
rays), through the C ABI, against the oracle.

The library traces N0 rays per source, derives each source's ray count N'
from their segment count S0 on the device, traces rays [N0, N') and weights
every ray by 1/N'.  The oracle applies the same rule (oracle.budget
.frame_ray_count) to its own count of the first N0 rays, and the GPU's result
must then equal the oracle's trace of rays [0, N') with 1/N' per ray: the
same N' (an integer, exactly), histograms within 1e-4 of each row, the same
statistics."""
import numpy as np
import pytest

import oracle
import paper_1803_00430_amd as P
import rpr_scenes as R
from oracle.budget import frame_ray_count
from parity import HIST_TOL, assert_hist_close, f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


def _gpu_budget(sc, srcs, lst, radius, *, n0, budget, max_rays, **kw):
    import torch
    hist, late, stats, rh = P.alloc_trace_outputs(len(srcs), kw["n_bins"], sc.n_bands, kw["sh_order"], max_rays,
                                                  want_hash=True)
    prm = P.trace_params(n_rays_total=n0, segment_budget=budget, max_rays=max_rays, **kw)
    P.trace_ir(sc, srcs, lst, radius, prm, hist, late, stats, rh)
    torch.cuda.synchronize()
    return hist.double().cpu().numpy(), late.double().cpu().numpy(), P.stats_host(stats), \
        rh.cpu().numpy().view(np.uint32)


def _check(sd, srcs, lst, radius, *, n0, budget, max_rays, **kw):
    srcs = np.atleast_2d(np.asarray(srcs, np.float32))
    sc = P.Scene.from_dict(sd)
    H, HL, st, rh = _gpu_budget(sc, srcs, lst, radius, n0=n0, budget=budget, max_rays=max_rays, **kw)
    okw = dict(kw, bin_width_s=f32(kw["bin_width_s"]))
    first = oracle.trace_ir(sd, srcs, lst, f32(radius), n_rays_total=n0, want_hash=False, **okw)
    out = []
    for s in range(len(srcs)):
        n1 = frame_ray_count(budget, int(first["stats"][s]["n_segments"]), n0, max_rays)
        assert int(st[s]["n_rays"]) == n1, (s, int(st[s]["n_rays"]), n1)
        o = oracle.trace_ir(sd, srcs[s:s + 1], lst, f32(radius), n_rays_total=n1, want_hash=True,
                            **dict(okw, pair_base=kw.get("pair_base", 0) + s))
        div = np.flatnonzero(rh[s, :n1] != o["ray_hash"][0])
        assert len(div) == 0, (s, div[:10])  # every path is the oracle's (FP64 ray state)
        assert_hist_close(H[s], o["hist"][0], what=f"hist[{s}]")
        assert_hist_close(HL[s], o["hist_late"][0], what=f"late[{s}]")
        os_ = o["stats"][0]
        for key in ("n_segments", "n_finite_segments", "n_escaped", "n_rays"):
            assert int(st[s][key]) == int(os_[key]), (s, key)
        assert abs(st[s]["e_emitted"] - 1.0) < 1e-6
        scale = np.abs(np.asarray(os_["e_class"])).max(axis=0)[:4] + 1e-30
        assert np.all(np.abs(np.asarray(st[s]["e_class"])[:, :4] - np.asarray(os_["e_class"])[:, :4])
                      <= HIST_TOL * scale)
        for k in ("e_escaped", "e_alive_at_stop", "e_absorbed"):
            assert np.allclose(np.asarray(st[s][k])[:4], np.asarray(os_[k])[:4], rtol=1e-4, atol=1e-12), k
        out.append((n1, int(st[s]["n_segments"])))
    sc.close()
    return out


def test_budget_closed_room(torch_cuda):
    """The tiny shoebox: every ray lives to the bounce limit, so N' =
    floor(B / (K + 1)) and the frame traces B segments up to one ray's worth."""
    c = R.tiny_config()
    K, B = 30, 60_000
    res = _check(c, c["sources"], c["listener"], c["radius"], n0=1024, budget=B, max_rays=8192, max_bounces=K,
                 sh_order=2, n_bins=2000, bin_width_s=1e-3, seed=4)
    (n1, segs), = res
    assert n1 == B // (K + 1) and B - (K + 1) < segs <= B


def test_budget_open_room_two_sources(torch_cuda):
    """An open box (four faces) with two sources: rays escape, each source's
    first pass measures its own segments per ray, and the escaped budget goes
    to more primary rays."""
    verts, tris, tm = R.merge(R.box_surfaces((0, 0, 0), (10, 7, 3), faces=("x0", "x1", "y0", "z0"), edge=1.0),
                              [0] * 4)
    sd = dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.array([[0.1, 0.2, 0.3, 0.4]], np.float32),
              scattering=np.array([[0.2, 0.4, 0.6, 0.8]], np.float32))
    srcs = np.array([[2.0, 2.0, 1.5], [8.5, 1.0, 2.5]], np.float32)
    K, B = 30, 40_000
    res = _check(sd, srcs, np.array([6.0, 4.0, 1.5], np.float32), 0.6, n0=1000, budget=B, max_rays=65536,
                 max_bounces=K, sh_order=3, n_bins=500, bin_width_s=1e-3, seed=9, pair_base=3)
    for n1, segs in res:
        assert n1 > B // (K + 1)  # escapes leave budget for more rays than a closed room takes
        assert abs(segs - B) < 0.05 * B


def test_budget_city_full_size(torch_cuda):
    """The city workload's scene, sources and listener (99,996 triangles,
    100 bounces, SH order 3, 3000 bins) under a budget of 6,000 segments per
    source from a first pass of 1,024 rays."""
    c = R.city_config()
    res = _check(c, c["sources"], c["listener"], c["radius"], n0=1024, budget=6000, max_rays=4096,
                 max_bounces=c["max_bounces"], sh_order=c["sh_order"], n_bins=c["n_bins"],
                 bin_width_s=c["bin_width_s"], seed=c["seed"])
    assert any(n1 > 1024 for n1, _ in res)  # open streets: rays escape, and the budget adds rays


def test_budget_met_by_first_pass_and_argument_checks(torch_cuda):
    """A budget the first pass already meets adds no rays (the result is the
    plain trace); invalid budget arguments are rejected before any launch."""
    c = R.tiny_config()
    sc = P.Scene.from_dict(c)
    kw = dict(max_bounces=10, sh_order=1, n_bins=300, bin_width_s=1e-3, seed=2)
    H, HL, st, rh = _gpu_budget(sc, c["sources"], c["listener"], c["radius"], n0=512, budget=1000, max_rays=4096,
                                **kw)
    assert int(st[0]["n_rays"]) == 512
    hist, late, stats, _ = P.alloc_trace_outputs(1, 300, 4, 1)
    P.trace_ir(sc, c["sources"], c["listener"], c["radius"], P.trace_params(n_rays_total=512, **kw), hist, late,
               stats)
    torch_cuda.cuda.synchronize()
    assert_hist_close(H[0], hist.double().cpu().numpy()[0], tol=1e-5)
    for bad in (dict(n_rays_total=512, ray_begin=1, segment_budget=100, max_rays=600),
                dict(n_rays_total=512, segment_budget=100, max_rays=100),
                dict(n_rays_total=512, segment_budget=-1, max_rays=600),
                dict(n_rays_total=512, segment_budget=2**62, max_rays=600)):
        prm = P.trace_params(**dict(kw, **bad))
        with pytest.raises(P.RprError):
            P.trace_ir(sc, c["sources"], c["listener"], c["radius"], prm, hist, late, stats)
    sc.close()
