"""GPU parity of the early-reflection paths against the oracle
(oracle/paths.py): the records of trace_ir_paths aggregated per path against
the oracle trace's (same rays; a ray whose discrete path differs between
FP32 and FP64 moves its mass to another key, so a small share of unmatched
mass is allowed), and the path cache and the prioritization on seeded
synthetic records given to both sides: every cached path after several
frames, the rendered paths in rank order, and the culled paths' moves into
the late histogram and class.  Edge cases: record overflow, cache overflow,
no records, n_er = 0."""
import math

import numpy as np
import pytest

import rpr_scenes as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NO_TRI = 0x7FFFFF


def _P():
    import paper_1803_00430_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P


def _key(s, o, t1, t2):
    return (int(s) << 48) | (int(o) << 46) | ((int(t1) & NO_TRI) << 23) | (int(t2) & NO_TRI if t2 >= 0 else NO_TRI)


def _pack_gpu(rc, nb, nc):
    n = len(rc["t"])
    a = np.zeros((n, 32), np.float32)
    u = a.view(np.uint32)
    for i in range(n):
        k = _key(rc["src"][i], rc["order"][i], rc["tri1"][i], rc["tri2"][i])
        u[i, 0], u[i, 1] = k & 0xFFFFFFFF, k >> 32
    a[:, 2:2 + nb] = rc["e"]
    a[:, 10] = rc["t"]
    a[:, 11:11 + nc] = rc["d"]
    return a


def _pack_oracle(rc, S, nb, nc):
    from oracle import paths as OP
    counts = np.bincount(rc["src"], minlength=S)
    rec = np.zeros((S, max(int(counts.max()), 1), 2, OP.REC_W))
    fill = np.zeros(S, int)
    for i in range(len(rc["t"])):
        s = int(rc["src"][i])
        x = rec[s, fill[s], 0]
        fill[s] += 1
        x[0], x[1], x[2], x[3] = 1, rc["order"][i], rc["tri1"][i], rc["tri2"][i]
        x[OP.REC_E:OP.REC_E + nb] = rc["e"][i]
        x[OP.REC_T] = rc["t"][i]
        x[OP.REC_D:OP.REC_D + nc] = rc["d"][i]
    return rec


def _gpu_paths(P, cache, n_max, **kw):
    out = torch.zeros((n_max, 128), dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    cache.select(0.0, n_max, out, n_out, **kw)
    torch.cuda.synchronize()
    n = int(n_out.item())
    return P.early_paths_host(out, n)


def _as_dict(paths, nb, nc):
    return {(int(p["source"]), int(p["order"]), int(p["tri"][0]), int(p["tri"][1])):
            dict(e=p["e"][:nb].astype(np.float64), t=float(p["t"]), d=p["d"][:nc].astype(np.float64)) for p in paths}


def _check_paths(g, o, what, rtol=2e-5):
    assert set(g) == set(o), (what, len(set(g) ^ set(o)))
    for k, v in o.items():
        gv = g[k]
        et = v["e"].sum()
        assert np.allclose(gv["e"], v["e"], rtol=rtol, atol=1e-7 * et), (what, k, gv["e"], v["e"])
        assert abs(gv["t"] - v["et"] / et) <= rtol * abs(v["et"] / et) + 1e-9, (what, k)
        assert np.allclose(gv["d"], v["d"], rtol=rtol, atol=rtol * et), (what, k)


def test_cache_frames_match_oracle():
    """Four frames of seeded records (alpha 0.3, min_energy cutting the
    faintest paths): after each frame every cached path equals the oracle's."""
    from oracle import paths as OP
    P = _P()
    S, nb, nc, a, emin = 8, 4, 4, 0.3, 2e-8
    cache = P.PathCache(max_paths=8192)
    oc = None
    for f in range(4):
        rc = R.path_records(100 + f, 6000, S, 1500 + 300 * f, nb, nc)
        g_rec = torch.from_numpy(_pack_gpu(rc, nb, nc)).cuda()
        n_rec = torch.tensor([len(rc["t"])], dtype=torch.int32, device="cuda")
        cache.update(g_rec, n_rec, a, f == 0, emin)
        fresh = OP.aggregate(_pack_oracle(rc, S, nb, nc), nb, nc)
        oc = OP.cache_update(oc, fresh, a, emin, first=(f == 0))
        info = cache.info()
        assert info["n_paths"] == len(oc) and info["overflow"] == 0, (f, info, len(oc))
        _check_paths(_as_dict(_gpu_paths(P, cache, 8192), nb, nc), oc, f"frame {f}")
    cache.close()


def test_select_matches_oracle():
    """Threshold and N_ER = 100 over 8 sources: the rendered paths in rank
    order, and the culled paths' intensity in the late histogram and moved
    from the early to the late class."""
    from oracle import paths as OP
    P = _P()
    S, nb, nc, T, dt = 8, 4, 9, 300, 1e-3
    rc = R.path_records(7, 8000, S, 2000, nb, nc, t_max=0.25)
    cache = P.PathCache(max_paths=4096)
    g_rec = torch.from_numpy(_pack_gpu(rc, nb, nc)).cuda()
    n_rec = torch.tensor([len(rc["t"])], dtype=torch.int32, device="cuda")
    cache.update(g_rec, n_rec, 1.0, True, 0.0)
    paths = OP.aggregate(_pack_oracle(rc, S, nb, nc), nb, nc)
    rng = np.random.default_rng(3)
    hl0 = rng.uniform(0, 1e-6, (S, T, nb)).astype(np.float32)
    st0 = np.zeros(S, P.IR_STATS_DTYPE)
    st0["e_class"][:, 1, :nb] = rng.uniform(1e-3, 2e-3, (S, nb))
    st0["e_class"][:, 2, :nb] = rng.uniform(1e-3, 2e-3, (S, nb))
    hl = torch.from_numpy(hl0.copy()).cuda()
    st = torch.from_numpy(st0.view(np.uint8).reshape(S, -1).copy()).cuda()
    out = torch.zeros((100, 128), dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    thr = 1e-6
    cache.select(thr, 100, out, n_out, hist_late=hl, stats=st, n_src=S, n_bins=T, n_bands=nb, bin_width_s=dt)
    torch.cuda.synchronize()
    hl_o = hl0.astype(np.float64)
    ec_o = np.array(st0["e_class"][:, :, :nb], np.float64)
    sel = OP.select(paths, thr, 100, hl_o, ec_o, dt)
    g = P.early_paths_host(out, int(n_out.item()))
    assert len(g) == len(sel) == 100
    gk = [(int(p["source"]), int(p["order"]), int(p["tri"][0]), int(p["tri"][1])) for p in g]
    ok = [k for k, _ in sel]
    for i, (a, b) in enumerate(zip(gk, ok)):
        if a != b:  # only a near tie may swap places
            ia, ib = paths[a]["e"].sum(), paths[b]["e"].sum()
            assert abs(ia - ib) <= 1e-5 * max(ia, ib), (i, a, b)
    assert set(gk) == set(ok)
    _check_paths(_as_dict(g, nb, nc), {k: v for k, v in sel}, "rendered")
    assert np.allclose(hl.cpu().numpy(), hl_o, rtol=1e-5, atol=1e-5 * np.abs(hl_o).max())
    ec = st.cpu().numpy().view(P.IR_STATS_DTYPE).reshape(-1)["e_class"][:, :, :nb]
    assert np.allclose(ec, ec_o, rtol=1e-6, atol=1e-12)
    assert not np.allclose(ec_o[:, 1], st0["e_class"][:, 1, :nb])  # something was moved
    cache.close()


def test_edge_cases():
    from oracle import paths as OP
    P = _P()
    S, nb, nc = 2, 4, 4
    rc = R.path_records(9, 3000, S, 800, nb, nc)
    g_rec = torch.from_numpy(_pack_gpu(rc, nb, nc)).cuda()
    # records past the count are not read
    n_rec = torch.tensor([1000], dtype=torch.int32, device="cuda")
    cache = P.PathCache(max_paths=4096)
    cache.update(g_rec, n_rec, 1.0, True, 0.0)
    part = {k: v[:1000] for k, v in rc.items()}
    _check_paths(_as_dict(_gpu_paths(P, cache, 4096), nb, nc),
                 OP.aggregate(_pack_oracle(part, S, nb, nc), nb, nc), "first 1000 records")
    # a count above the buffer reads the buffer only
    n_big = torch.tensor([10**6], dtype=torch.int32, device="cuda")
    cache.update(g_rec, n_big, 1.0, True, 0.0)
    _check_paths(_as_dict(_gpu_paths(P, cache, 4096), nb, nc),
                 OP.aggregate(_pack_oracle(rc, S, nb, nc), nb, nc), "count above the buffer")
    # no records: the cache decays by 1 - alpha
    before = _as_dict(_gpu_paths(P, cache, 4096), nb, nc)
    zero = torch.zeros(1, dtype=torch.int32, device="cuda")
    cache.update(g_rec, zero, 0.25, False, 0.0)
    after = _as_dict(_gpu_paths(P, cache, 4096), nb, nc)
    assert set(after) == set(before)
    for k in before:
        assert np.allclose(after[k]["e"], 0.75 * before[k]["e"], rtol=1e-6)
    # n_er = 0: everything above the threshold is culled
    out = torch.zeros((1, 128), dtype=torch.uint8, device="cuda")
    n_out = torch.ones(1, dtype=torch.int32, device="cuda")
    hl = torch.zeros((S, 50, nb), dtype=torch.float32, device="cuda")
    cache.select(0.0, 0, out, n_out, hist_late=hl, n_src=S, n_bins=50, n_bands=nb, bin_width_s=0.01)
    torch.cuda.synchronize()
    assert int(n_out.item()) == 0
    assert abs(hl.sum().item() - sum(v["e"].sum() for v in after.values())) < 1e-4 * hl.sum().item()
    cache.close()
    # capacity overflow is flagged and the cache stays within it
    small = P.PathCache(max_paths=100)
    small.update(g_rec, n_big, 1.0, True, 0.0)
    info = small.info()
    assert info["overflow"] == 1 and info["n_paths"] == 100
    assert len(_gpu_paths(P, small, 100)) == 100
    small.close()
    # bad arguments
    with pytest.raises(P.RprError):
        P.PathCache(max_paths=0)
    c2 = P.PathCache(max_paths=16)
    with pytest.raises(P.RprError):
        c2.update(g_rec, n_rec, 1.5, True)
    c2.close()


def _records_dict(P, rec, n, nb, nc):
    a = rec[:n].cpu().numpy()
    u = a.view(np.uint32)
    out = {}
    for i in range(n):
        k = int(u[i, 0]) | (int(u[i, 1]) << 32)
        s, o, t1, t2 = k >> 48, (k >> 46) & 3, (k >> 23) & NO_TRI, k & NO_TRI
        key = (s, o, t1, -1 if t2 == NO_TRI else t2)
        e = a[i, 2:2 + nb].astype(np.float64)
        p = out.setdefault(key, dict(e=np.zeros(nb), et=0.0, d=np.zeros(nc)))
        p["e"] += e
        p["et"] += e.sum() * float(a[i, 10])
        p["d"] += a[i, 11:11 + nc]
    return out


@pytest.mark.parametrize("scene_kind", ["tiny", "lroom"])
def test_trace_records_match_oracle(scene_kind):
    """The records of trace_ir_paths, aggregated per path, against the oracle
    trace's paths of the same rays (3 sources, scattering surfaces, K = 6):
    at most 1% of the early intensity on keys of one side only (rays whose
    discrete path differs), and the matched paths within FP32 rounding."""
    from oracle import paths as OP
    P = _P()
    c = R.tiny_config()
    if scene_kind == "tiny":
        sc = c
        srcs = np.array([[2, 2, 1.5], [8, 5, 2.0], [5, 1, 0.5]], np.float32)
        lp = c["listener"]
    else:
        verts, tris, tm = R.merge(R.lroom((12.0, 10.0, 3.0), (0.5, 0.5), edge=2.0), [0] * 8)
        sc = dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.array([[0.1, 0.2, 0.3, 0.4]], np.float32),
                  scattering=np.array([[0.2, 0.4, 0.6, 0.8]], np.float32))
        srcs = np.array([[11.0, 1.5, 1.5], [2.0, 2.0, 1.0], [9.0, 4.0, 2.0]], np.float32)
        lp = np.array([1.5, 9.0, 1.5], np.float32)
    nb, order, T, dt, N, K = 4, 1, 400, 1e-3, 16384, 6
    nc = (order + 1) ** 2
    scene = P.Scene.from_dict(sc, device="cuda")
    hist, late, stats, _ = P.alloc_trace_outputs(3, T, nb, order, device="cuda")
    rec = torch.zeros((200000, 32), dtype=torch.float32, device="cuda")
    n_rec = torch.zeros(1, dtype=torch.int32, device="cuda")
    prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=order, n_bins=T, bin_width_s=dt, seed=77)
    P.trace_ir_paths(scene, srcs, lp, 0.5, prm, hist, late, stats, rec, n_rec)
    torch.cuda.synchronize()
    n = int(n_rec.item())
    assert 0 < n <= rec.shape[0]
    g = _records_dict(P, rec, n, nb, nc)
    o = OP.trace_paths(sc, srcs.astype(np.float64), lp.astype(np.float64), 0.5, n_rays_total=N, max_bounces=K,
                       sh_order=order, n_bins=T, bin_width_s=dt, seed=77)
    op = OP.aggregate(o["records"], nb, nc)
    st = P.stats_host(stats)
    for s in range(3):
        ge = sum((v["e"] for k, v in g.items() if k[0] == s), np.zeros(nb))
        assert np.allclose(ge, st["e_class"][s][1][:nb], rtol=1e-4)  # the records are the early class
    tot = sum(v["e"].sum() for v in op.values())
    only = sum(v["e"].sum() for k, v in op.items() if k not in g) + sum(v["e"].sum() for k, v in g.items() if k not in op)
    assert only <= 1e-2 * tot, (only / tot)
    both = [k for k in op if k in g]
    assert len(both) > 0.9 * len(op)
    # matched paths: FP32 drift along a ray, largest for grazing chords through the sphere (their
    # time span is short), bounds each path; weighted by intensity the paths agree to 1e-4
    diff_e = diff_t = 0.0
    for k in both:
        ov, gv = op[k], g[k]
        et = ov["e"].sum()
        assert np.allclose(gv["e"], ov["e"], rtol=5e-3, atol=1e-6 * et), k
        assert np.allclose(gv["d"], ov["d"], rtol=2e-2, atol=5e-3 * et), k
        diff_e += np.abs(gv["e"] - ov["e"]).sum()
        diff_t += et * abs(gv["et"] / gv["e"].sum() - ov["et"] / et)
    mass = sum(op[k]["e"].sum() for k in both)
    assert diff_e <= 1e-4 * mass, diff_e / mass
    assert diff_t <= 1e-5 * mass, diff_t / mass  # seconds, intensity-weighted
    scene.close()


def test_trace_records_overflow_and_bad_arguments():
    P = _P()
    c = R.tiny_config()
    scene = P.Scene.from_dict(c, device="cuda")
    hist, late, stats, _ = P.alloc_trace_outputs(1, 200, 4, 1, device="cuda")
    rec = torch.full((64, 32), -7.0, dtype=torch.float32, device="cuda")
    big = torch.zeros((100000, 32), dtype=torch.float32, device="cuda")
    n_rec = torch.zeros(1, dtype=torch.int32, device="cuda")
    prm = P.trace_params(n_rays_total=8192, max_bounces=4, sh_order=1, n_bins=200, bin_width_s=1e-3, seed=5)
    P.trace_ir_paths(scene, c["sources"], c["listener"], c["radius"], prm, hist, late, stats, big, n_rec)
    torch.cuda.synchronize()
    n_all = int(n_rec.item())
    assert n_all > 64
    P.trace_ir_paths(scene, c["sources"], c["listener"], c["radius"], prm, hist, late, stats, rec, n_rec)
    torch.cuda.synchronize()
    assert int(n_rec.item()) == n_all  # every record counted, only 64 written
    assert not torch.any(rec == -7.0)
    with pytest.raises(P.RprError):
        bad = P.trace_params(n_rays_total=8192, max_bounces=4, sh_order=1, n_bins=200, bin_width_s=1e-3, seed=5,
                             flags=1)
        P.trace_ir_paths(scene, c["sources"], c["listener"], c["radius"], bad, hist, late, stats, rec, n_rec)
    scene.close()
