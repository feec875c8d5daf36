"""Seeded synthetic inputs: triangle scenes, materials, sources and listeners.

This module only builds geometry and draws the random scene parameters with
numpy's PCG64.  It holds none of the propagation or estimation arithmetic, so
both the HIP library's tests and the CPU oracle can take their inputs from it.

The paper's own scenes (City, Hospital, Space Station, Sub Bay, Tuscany;
Section 6, Table 1) are not available; the procedural scenes here stand in for
them, with the sizes and value ranges of the workloads that are measured.

Every scene is a dict with
  verts        float32 [V, 3]   metres
  tris         int32   [T, 3]   vertex indices
  tri_mat      int32   [T]      material index per triangle
  absorption   float32 [M, B]   per-band absorption coefficient in [0, 1]
  scattering   float32 [M, B]   per-band scattering coefficient in [0, 1]
plus generator-specific entries (sources, listener, radius, ...).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng", "rect", "box_surfaces", "merge", "shoebox", "tiny_config", "city_config",
    "lroom", "learn_room", "batch_config", "hospital_config", "random_rays",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def rect(p0, a, b, na: int = 1, nb: int = 1):
    """Planar rectangle p0 + s*a + t*b, s,t in [0,1], split into na x nb quads
    of two triangles each.  Returns (verts [V,3] f64, tris [T,3] i64)."""
    p0, a, b = (np.asarray(v, dtype=np.float64) for v in (p0, a, b))
    na, nb = max(1, int(na)), max(1, int(nb))
    s = np.arange(na + 1) / na
    t = np.arange(nb + 1) / nb
    S, Tt = np.meshgrid(s, t, indexing="ij")
    verts = p0 + S[..., None] * a + Tt[..., None] * b
    verts = verts.reshape(-1, 3)
    idx = np.arange((na + 1) * (nb + 1)).reshape(na + 1, nb + 1)
    v00 = idx[:-1, :-1].ravel()
    v10 = idx[1:, :-1].ravel()
    v01 = idx[:-1, 1:].ravel()
    v11 = idx[1:, 1:].ravel()
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    return verts, tris


def _n(length: float, edge: float | None) -> int:
    if edge is None or edge <= 0:
        return 1
    return max(1, int(math.ceil(length / edge - 1e-9)))


def box_surfaces(lo, hi, edge=None, faces=("x0", "x1", "y0", "y1", "z0", "z1")):
    """Axis-aligned box faces as tessellated rectangles.  Returns a list of
    (verts, tris) parts, one per face, in the order of `faces`."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = hi - lo
    ex, ey, ez = np.array([d[0], 0, 0]), np.array([0, d[1], 0]), np.array([0, 0, d[2]])
    out = []
    for f in faces:
        if f == "x0":
            out.append(rect(lo, ey, ez, _n(d[1], edge), _n(d[2], edge)))
        elif f == "x1":
            out.append(rect(lo + ex, ey, ez, _n(d[1], edge), _n(d[2], edge)))
        elif f == "y0":
            out.append(rect(lo, ex, ez, _n(d[0], edge), _n(d[2], edge)))
        elif f == "y1":
            out.append(rect(lo + ey, ex, ez, _n(d[0], edge), _n(d[2], edge)))
        elif f == "z0":
            out.append(rect(lo, ex, ey, _n(d[0], edge), _n(d[1], edge)))
        elif f == "z1":
            out.append(rect(lo + ez, ex, ey, _n(d[0], edge), _n(d[1], edge)))
        else:
            raise ValueError(f)
    return out


def merge(parts, mats):
    """Concatenate (verts, tris) parts; `mats` gives one material per part."""
    verts, tris, tri_mat = [], [], []
    off = 0
    for (v, t), m in zip(parts, mats):
        verts.append(v)
        tris.append(t + off)
        tri_mat.append(np.full(len(t), m, np.int32))
        off += len(v)
    return (np.concatenate(verts).astype(np.float32),
            np.concatenate(tris).astype(np.int32),
            np.concatenate(tri_mat).astype(np.int32))


def shoebox(dims, edge=None, material=0):
    parts = box_surfaces((0, 0, 0), dims, edge)
    return merge(parts, [material] * len(parts))


def tiny_config():
    """Shoebox 10 x 7 x 3 m as 12 triangles, one material with per-band
    absorption {0.1, 0.2, 0.3, 0.4} and scattering 0.5; source (2, 2, 1.5),
    listener sphere r = 0.5 m at (7, 5, 1.5); 4096 rays, 50 bounces, 2000 bins
    of 1 ms, SH order 2, Philox seed 0."""
    verts, tris, tri_mat = shoebox((10.0, 7.0, 3.0))
    return dict(
        name="tiny", verts=verts, tris=tris, tri_mat=tri_mat,
        absorption=np.array([[0.1, 0.2, 0.3, 0.4]], np.float32),
        scattering=np.full((1, 4), 0.5, np.float32),
        sources=np.array([[2.0, 2.0, 1.5]], np.float32),
        listener=np.array([7.0, 5.0, 1.5], np.float32), radius=0.5,
        n_rays=4096, max_bounces=50, n_bins=2000, bin_width_s=1e-3, sh_order=2, seed=0,
        volume=210.0, area=242.0,
    )


def _city_buildings(g, extent, cell):
    ncell = int(extent // cell)
    off = 0.5 * (extent - ncell * cell)
    b = []
    for gx in range(ncell):
        for gy in range(ncell):
            fx, fy = g.uniform(5.0, 30.0, 2)
            h = g.uniform(5.0, 60.0)
            x0 = off + gx * cell + 3.0 + g.uniform(0.0, max(0.0, cell - 6.0 - fx))
            y0 = off + gy * cell + 3.0 + g.uniform(0.0, max(0.0, cell - 6.0 - fy))
            b.append((x0, y0, fx, fy, h))
    return b


def _city_tri_count(buildings, extent, edge):
    n = 2 * _n(extent, edge) ** 2
    for (_, _, fx, fy, h) in buildings:
        n += 2 * 2 * (_n(fx, edge) + _n(fy, edge)) * _n(h, edge)
        n += 2 * _n(fx, edge) * _n(fy, edge)
    return n


def city_config(seed=1, target_tris=100_000, extent=500.0, cell=36.0, n_materials=8,
                n_bands=4, n_sources=8, radius=1.0, source_radius=80.0):
    """Procedural city: axis-aligned extruded boxes (footprint sides U[5,30] m,
    heights U[5,60] m) on a jittered street grid over a 500 x 500 m ground
    plane.  Facades, roofs and the ground are tessellated into square panels
    whose edge is chosen so that the triangle count is close to `target_tris`.
    8 materials with per-band absorption U[0.05,0.5] and scattering U[0.1,0.9];
    one material per face.  Listener (r = 1 m) at street level near the
    centre; sources at street level within `source_radius` of it, outside the
    buildings."""
    g = rng(seed)
    bld = _city_buildings(g, extent, cell)
    lo_e, hi_e = 0.5, 100.0
    for _ in range(60):
        mid = math.sqrt(lo_e * hi_e)
        if _city_tri_count(bld, extent, mid) > target_tris:
            lo_e = mid
        else:
            hi_e = mid
    cands = [lo_e, hi_e]
    edge = min(cands, key=lambda e: abs(_city_tri_count(bld, extent, e) - target_tris))
    parts, mats = [], []
    parts.append(rect((0, 0, 0), (extent, 0, 0), (0, extent, 0), _n(extent, edge), _n(extent, edge)))
    mats.append(int(g.integers(n_materials)))
    for (x0, y0, fx, fy, h) in bld:
        faces = box_surfaces((x0, y0, 0.0), (x0 + fx, y0 + fy, h), edge,
                             faces=("x0", "x1", "y0", "y1", "z1"))
        for f in faces:
            parts.append(f)
            mats.append(int(g.integers(n_materials)))
    verts, tris, tri_mat = merge(parts, mats)
    absorption = g.uniform(0.05, 0.5, (n_materials, n_bands)).astype(np.float32)
    scattering = g.uniform(0.1, 0.9, (n_materials, n_bands)).astype(np.float32)

    def free(p, clear):
        for (x0, y0, fx, fy, _) in bld:
            if x0 - clear <= p[0] <= x0 + fx + clear and y0 - clear <= p[1] <= y0 + fy + clear:
                return False
        return True

    while True:
        lp = np.array([g.uniform(0.4, 0.6) * extent, g.uniform(0.4, 0.6) * extent, 1.5])
        if free(lp, radius + 0.5):
            break
    srcs = []
    while len(srcs) < n_sources:
        ang = g.uniform(0, 2 * math.pi)
        rr = source_radius * math.sqrt(g.uniform(0.02, 1.0))
        p = lp + np.array([rr * math.cos(ang), rr * math.sin(ang), 0.0])
        if free(p, 0.5) and np.linalg.norm(p - lp) > radius + 1.0:
            srcs.append(p)
    return dict(
        name="city", verts=verts, tris=tris, tri_mat=tri_mat,
        absorption=absorption, scattering=scattering,
        sources=np.array(srcs, np.float32), listener=lp.astype(np.float32), radius=radius,
        n_rays=32768, max_bounces=100, n_bins=3000, bin_width_s=1e-3, sh_order=3, seed=1,
        panel_edge=edge, n_buildings=len(bld), buildings=bld,
    )


def city_source_walk(cfg, n_frames, step=3.0, seed=7, clear=0.5):
    """Street-level random walks of the city's sources: each frame a source
    moves `step` metres in its current heading, turning to a random heading
    whenever the move would enter a building (with `clear` metres margin) or
    leave the ground plane.  Returns [n_frames][n_sources][3] float32."""
    g = rng(seed)
    bld = cfg["buildings"]
    extent = float(cfg["verts"][:, 0].max())

    def free(p):
        if not (clear <= p[0] <= extent - clear and clear <= p[1] <= extent - clear):
            return False
        for (x0, y0, fx, fy, _) in bld:
            if x0 - clear <= p[0] <= x0 + fx + clear and y0 - clear <= p[1] <= y0 + fy + clear:
                return False
        return True

    pos = cfg["sources"].astype(np.float64).copy()
    head = g.uniform(0, 2 * math.pi, len(pos))
    out = []
    for _ in range(n_frames):
        out.append(pos.copy())
        for i in range(len(pos)):
            for _try in range(64):
                q = pos[i] + step * np.array([math.cos(head[i]), math.sin(head[i]), 0.0])
                if free(q):
                    pos[i] = q
                    break
                head[i] = g.uniform(0, 2 * math.pi)
    return np.array(out, np.float32)


def lroom(dims, notch, edge=None):
    """L-shaped room: the box [0,Lx]x[0,Ly]x[0,Lz] without the corner
    [nx*Lx, Lx] x [ny*Ly, Ly].  Returns a list of tessellated parts."""
    Lx, Ly, Lz = (float(v) for v in dims)
    nx, ny = notch
    ax, ay = nx * Lx, ny * Ly
    outline = [(0, 0), (Lx, 0), (Lx, ay), (ax, ay), (ax, Ly), (0, Ly)]
    parts = []
    for k in range(6):
        p = np.array([*outline[k], 0.0])
        q = np.array([*outline[(k + 1) % 6], 0.0])
        e = q - p
        parts.append(rect(p, e, (0, 0, Lz), _n(np.linalg.norm(e), edge), _n(Lz, edge)))
    for z in (0.0, Lz):
        parts.append(rect((0, 0, z), (Lx, 0, 0), (0, ay, 0), _n(Lx, edge), _n(ay, edge)))
        parts.append(rect((0, ay, z), (ax, 0, 0), (0, Ly - ay, 0), _n(ax, edge), _n(Ly - ay, edge)))
    return parts


def _inside_room(p, kind, dims, notch, clear):
    d = np.asarray(dims)
    if np.any(p < clear) or np.any(p > d - clear):
        return False
    if kind == "lroom":
        ax, ay = notch[0] * d[0], notch[1] * d[1]
        if p[0] > ax - clear and p[1] > ay - clear:
            return False
    return True


def _sample_pair(g, kind, dims, notch, blockers=(), clear=0.5, min_sep=1.0):
    d = np.asarray(dims, np.float64)

    def ok(p):
        if not _inside_room(p, kind, d, notch, clear):
            return False
        for (lo, hi) in blockers:
            if np.all(p > lo - clear) and np.all(p < hi + clear):
                return False
        return True

    for _ in range(100000):
        s = g.uniform(0, 1, 3) * d
        l = g.uniform(0, 1, 3) * d
        if ok(s) and ok(l) and np.linalg.norm(s - l) >= min_sep:
            return s, l
    raise RuntimeError("could not place a source/listener pair")


def learn_room(seed: int, n_bands=4):
    """One training / held-out room for the learned estimator: 50% shoebox and
    50% L-room, bounding dims U[3,40] m per axis, notch fractions U[0.3,0.7],
    per-band absorption U[0.02,0.6] and scattering U[0.1,0.9] (one material),
    source and listener uniform with 0.5 m wall clearance, >= 1 m apart,
    listener radius 0.5 m."""
    g = rng(seed)
    kind = "shoebox" if g.uniform() < 0.5 else "lroom"
    dims = g.uniform(3.0, 40.0, 3)
    notch = g.uniform(0.3, 0.7, 2)
    if kind == "shoebox":
        parts = box_surfaces((0, 0, 0), dims)
    else:
        parts = lroom(dims, notch)
    verts, tris, tri_mat = merge(parts, [0] * len(parts))
    absorption = g.uniform(0.02, 0.6, (1, n_bands)).astype(np.float32)
    scattering = g.uniform(0.1, 0.9, (1, n_bands)).astype(np.float32)
    s, l = _sample_pair(g, kind, dims, notch)
    return dict(name=f"learn{seed}", seed=seed, kind=kind, dims=dims, notch=notch, verts=verts, tris=tris,
                tri_mat=tri_mat, absorption=absorption, scattering=scattering,
                sources=s[None].astype(np.float32), listener=l.astype(np.float32), radius=0.5)


def _box_tri_count(d, edge):
    """Triangles of the six tessellated faces of a box with sides d."""
    nx, ny, nz = (_n(v, edge) for v in d)
    return 2 * 2 * (ny * nz + nx * nz + nx * ny)


def _room_tri_count(kind, dims, notch, edge, clutter):
    """Triangle count of the tessellated room (same rule as `rect`: two
    triangles per panel), without building the geometry."""
    Lx, Ly, Lz = (float(v) for v in dims)
    if kind == "lroom":
        ax, ay = notch[0] * Lx, notch[1] * Ly
        outline = [(0, 0), (Lx, 0), (Lx, ay), (ax, ay), (ax, Ly), (0, Ly)]
        n = 0
        for k in range(6):
            p, q = np.array(outline[k]), np.array(outline[(k + 1) % 6])
            n += 2 * _n(float(np.linalg.norm(q - p)), edge) * _n(Lz, edge)
        n += 2 * 2 * (_n(Lx, edge) * _n(ay, edge) + _n(ax, edge) * _n(Ly - ay, edge))
    else:
        n = _box_tri_count((Lx, Ly, Lz), edge)
    for (lo, hi) in clutter:
        n += _box_tri_count(np.asarray(hi) - np.asarray(lo), edge)
    return n


def batch_scene(seed: int, n_pairs=16, n_bands=4, tri_range=(1_000, 500_000)):
    """One scene of the batched workload: a shoebox, an L-room or a box-cluster
    interior (dims U[3,40] m), tessellated (plus clutter boxes for the cluster
    kind) to a log-uniform triangle count in `tri_range`; absorption
    U[0.02,0.6] and scattering U[0.1,0.9] per material and band; `n_pairs`
    source/listener pairs (r = 0.5 m) with log-uniform ray counts in
    [1024, 65536] and bounce limits U{50..200}."""
    g = rng(seed)
    kind = ("shoebox", "lroom", "cluster")[seed % 3]
    dims = g.uniform(3.0, 40.0, 3)
    dims[2] = min(dims[2], g.uniform(3.0, 12.0))
    notch = g.uniform(0.3, 0.7, 2)
    target = math.exp(g.uniform(math.log(tri_range[0]), math.log(tri_range[1])))
    clutter = []
    if kind == "cluster":
        for _ in range(int(g.integers(8, 40))):
            sz = g.uniform(0.05, 0.2, 3) * dims
            sz[2] = min(sz[2], 0.6 * dims[2])
            lo = g.uniform(0, 1, 3) * (dims - sz)
            lo[2] = 0.0
            clutter.append((lo, lo + sz))
    lo_e, hi_e = 1e-3, 100.0
    for _ in range(60):
        mid = math.sqrt(lo_e * hi_e)
        if _room_tri_count(kind, dims, notch, mid, clutter) > target:
            lo_e = mid
        else:
            hi_e = mid
    edge = min((lo_e, hi_e), key=lambda e: abs(_room_tri_count(kind, dims, notch, e, clutter) - target))
    parts = lroom(dims, notch, edge) if kind == "lroom" else box_surfaces((0, 0, 0), dims, edge)
    n_mat = 4
    mats = [int(g.integers(n_mat)) for _ in parts]
    for (lo, hi) in clutter:
        for f in box_surfaces(lo, hi, edge):
            parts.append(f)
            mats.append(int(g.integers(n_mat)))
    verts, tris, tri_mat = merge(parts, mats)
    absorption = g.uniform(0.02, 0.6, (n_mat, n_bands)).astype(np.float32)
    scattering = g.uniform(0.1, 0.9, (n_mat, n_bands)).astype(np.float32)
    pairs = []
    for _ in range(n_pairs):
        s, l = _sample_pair(g, "lroom" if kind == "lroom" else "shoebox", dims, notch, clutter)
        rays = int(round(math.exp(g.uniform(math.log(1024), math.log(65536)))))
        K = int(g.integers(50, 201))
        pairs.append(dict(source=s.astype(np.float32), listener=l.astype(np.float32), radius=0.5,
                          n_rays=rays, max_bounces=K))
    return dict(name=f"batch{seed}", kind=kind, dims=dims, verts=verts, tris=tris,
                tri_mat=tri_mat, absorption=absorption, scattering=scattering, pairs=pairs,
                panel_edge=edge)


def batch_config(n_scenes=16, pairs_per_scene=16, first_seed=100):
    """256 source-listener pairs over 16 scenes (seeds 100..115); pair p uses
    Philox seed 1000 + p; SH order 3, 4 bands, 2000 bins of 1 ms."""
    scenes = [batch_scene(first_seed + i, pairs_per_scene) for i in range(n_scenes)]
    return dict(name="batch", scenes=scenes, n_bins=2000, bin_width_s=1e-3, sh_order=3,
                seed_base=1000)


def hospital_config(seed=300, target_tris=1_000_000, nx=8, ny=6, n_sources=64):
    """Hospital-like interior: a grid of rooms (sides U[4,12] m, 3 m ceilings)
    joined by 2.5 m corridors with 1 x 2.1 m doorways, plus clutter boxes,
    tessellated to about `target_tris` triangles.  64 sources in the corridors
    and one listener (r = 0.5 m)."""
    g = rng(seed)
    H = 3.0
    corr = 2.5
    wx = g.uniform(4.0, 12.0, nx)
    wy = g.uniform(4.0, 12.0, ny)
    xs = np.concatenate([[0.0], np.cumsum(wx + corr)])
    ys = np.concatenate([[0.0], np.cumsum(wy + corr)])
    rooms = [(xs[i], ys[j], wx[i], wy[j]) for i in range(nx) for j in range(ny)]
    clutter = []
    for (x0, y0, w, d) in rooms:
        for _ in range(int(g.integers(2, 6))):
            sz = np.array([g.uniform(0.4, 2.0), g.uniform(0.4, 2.0), g.uniform(0.4, 1.8)])
            lo = np.array([x0 + g.uniform(0.3, max(0.31, w - sz[0] - 0.3)),
                           y0 + g.uniform(0.3, max(0.31, d - sz[1] - 0.3)), 0.0])
            clutter.append((lo, lo + sz))

    def build(edge):
        parts = []
        X, Y = xs[-1], ys[-1]
        parts += box_surfaces((-corr, -corr, 0.0), (X, Y, H), edge)
        for (x0, y0, w, d) in rooms:
            # four walls; the wall facing -y has a 1 m wide, 2.1 m high doorway
            door = x0 + 0.5 * w - 0.5
            for yy in (y0, y0 + d):
                if yy == y0:
                    parts.append(rect((x0, yy, 0), (door - x0, 0, 0), (0, 0, H), _n(door - x0, edge), _n(H, edge)))
                    parts.append(rect((door + 1.0, yy, 0), (x0 + w - door - 1.0, 0, 0), (0, 0, H),
                                      _n(x0 + w - door - 1.0, edge), _n(H, edge)))
                    parts.append(rect((door, yy, 2.1), (1.0, 0, 0), (0, 0, H - 2.1), _n(1.0, edge), _n(H - 2.1, edge)))
                else:
                    parts.append(rect((x0, yy, 0), (w, 0, 0), (0, 0, H), _n(w, edge), _n(H, edge)))
            for xx in (x0, x0 + w):
                parts.append(rect((xx, y0, 0), (0, d, 0), (0, 0, H), _n(d, edge), _n(H, edge)))
        for (lo, hi) in clutter:
            parts += box_surfaces(lo, hi, edge)
        return parts

    def count(edge):
        return sum(len(t) for _, t in build(edge))

    lo_e, hi_e = 0.05, 50.0
    for _ in range(40):
        mid = math.sqrt(lo_e * hi_e)
        if count(mid) > target_tris:
            lo_e = mid
        else:
            hi_e = mid
    edge = hi_e
    parts = build(edge)
    n_mat = 6
    mats = [int(g.integers(n_mat)) for _ in parts]
    verts, tris, tri_mat = merge(parts, mats)
    absorption = g.uniform(0.02, 0.5, (n_mat, 4)).astype(np.float32)
    scattering = g.uniform(0.1, 0.9, (n_mat, 4)).astype(np.float32)
    # corridor polylines: horizontal corridors at y = ys[j] - corr/2
    srcs = []
    for s in range(n_sources):
        j = int(g.integers(1, ny))
        y = ys[j] - 0.5 * corr
        x = g.uniform(0.5, xs[-1] - 0.5)
        srcs.append((x, y, 1.5))
    lp = np.array([0.5 * xs[-1] + 0.3, ys[ny // 2] - 0.5 * corr, 1.5])
    return dict(name="hosp", verts=verts, tris=tris, tri_mat=tri_mat, absorption=absorption,
                scattering=scattering, sources=np.array(srcs, np.float32),
                listener=lp.astype(np.float32), radius=0.5, n_rays=131072, max_bounces=200,
                n_bins=3000, bin_width_s=1e-3, sh_order=3, seed=300, panel_edge=edge)


def random_rays(seed: int, n: int, lo, hi):
    """Random ray origins uniform in the box [lo, hi] and directions uniform
    on the sphere (for closest-hit cross-checks)."""
    g = rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    o = lo + g.uniform(0, 1, (n, 3)) * (hi - lo)
    d = g.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def reverb_inputs(seed: int, n_ir: int, n_bands: int, sh_order: int, n_bins: int = 80, bin_width_s: float = 0.01,
                  mfp_range=(2.0, 40.0)):
    """Seeded inputs of the SH reverberator, shaped like the estimates of
    rooms and outdoor scenes: RT60 U(0.2, 3) s per band, g_reverb U(0.01,
    0.5), mean free path U(mfp_range) m, a predelay (first late bin) 2..12
    bins after t = 0 and a first arrival one to two bins earlier, an
    all-orders histogram [n_ir][n_bins][n_bands][(n+1)^2] whose energy decays
    from the first arrival while its dominant direction turns from bin to
    bin, a directional distribution per band (coefficient 0 = 1/sqrt(4 pi),
    the others uniform in +-0.3 of it), the standard normals of the comb
    delays and the rotation angles in [pi/2, 3pi/2].  Plain random numbers and
    shapes only: returns a dict of numpy arrays."""
    g = rng(seed)
    nc = (sh_order + 1) ** 2
    B, T = n_bands, n_bins
    fa = g.integers(0, 10, size=n_ir)
    pre = fa + g.integers(1, 3, size=n_ir)
    hist = np.zeros((n_ir, T, B, nc), np.float32)
    for i in range(n_ir):
        tau = g.uniform(3.0, 25.0)
        env = np.zeros(T)
        env[fa[i]:] = np.exp(-np.arange(T - fa[i]) / tau)
        a0 = g.normal(size=3)
        a1 = g.normal(size=3)
        for t in range(fa[i], T):
            s = (t - fa[i]) / max(T - fa[i] - 1, 1)
            u = (1 - s) * a0 + s * a1
            u = u / (np.linalg.norm(u) + 1e-30)
            for b in range(B):
                e = env[t] * g.uniform(0.5, 1.0) / (b + 1)
                hist[i, t, b, 0] = e * 0.28209479177387814
                if nc >= 4:
                    k = 0.4886025119029199 * e * g.uniform(0.3, 0.9)
                    hist[i, t, b, 1:4] = (-k * u[1], k * u[2], -k * u[0])
                if nc > 4:
                    hist[i, t, b, 4:] = e * g.uniform(-0.05, 0.05, size=nc - 4)
    xbar = np.zeros((n_ir, 8, 16), np.float32)
    xbar[:, :B, 0] = 1 / math.sqrt(4 * math.pi)
    xbar[:, :B, 1:nc] = g.uniform(-0.3, 0.3, size=(n_ir, B, nc - 1)) / math.sqrt(4 * math.pi)
    rt = np.zeros((n_ir, 8), np.float32)
    rt[:, :B] = g.uniform(0.2, 3.0, size=(n_ir, B))
    gr = np.zeros((n_ir, 8), np.float32)
    gr[:, :B] = g.uniform(0.01, 0.5, size=(n_ir, B))
    return dict(
        rt60=rt, g_reverb=gr, dir_loudness=xbar,
        mean_free_path_m=g.uniform(*mfp_range, size=n_ir).astype(np.float32),
        predelay_s=(pre * bin_width_s).astype(np.float32), first_arrival_s=(fa * bin_width_s).astype(np.float32),
        hist=hist, bin_width_s=bin_width_s,
        z=g.normal(size=(n_ir, 8)).astype(np.float32),
        angles=g.uniform(math.pi / 2, 1.5 * math.pi, size=(n_ir, 8, 3)).astype(np.float32))


def band_audio(seed: int, n_src: int, n_bands: int, n: int, scale: float = 0.1):
    """Seeded band audio [n_src][n_bands][n] f32: white noise, scale rms."""
    return (rng(seed).normal(size=(n_src, n_bands, n)) * scale).astype(np.float32)


def path_records(seed: int, n: int, n_src: int, n_keys: int, n_bands: int = 4, n_coeffs: int = 4,
                 n_tris: int = 5000, t_max: float = 0.2):
    """Seeded early-path records: n records over about n_keys distinct paths
    (source, order 1 or 2, one or two triangles), band intensities
    log-uniform over five decades, arrival times uniform in [0, t_max) and
    directivities uniform in +-1 of the intensity.  Plain random numbers:
    returns dict(src, order, tri1, tri2 (-1 for none), e [n][n_bands],
    t [n], d [n][n_coeffs])."""
    g = rng(seed)
    ks = g.integers(0, n_src, size=n_keys)
    ko = g.integers(1, 3, size=n_keys)
    k1 = g.integers(0, n_tris, size=n_keys)
    k2 = np.where(ko == 2, g.integers(0, n_tris, size=n_keys), -1)
    pick = g.integers(0, n_keys, size=n)
    e = (10.0 ** g.uniform(-9, -4, size=(n, 1)) * g.uniform(0.2, 1.0, size=(n, n_bands))).astype(np.float32)
    t = g.uniform(0, t_max, size=n).astype(np.float32)
    d = (e.sum(axis=1, keepdims=True) * g.uniform(-1, 1, size=(n, n_coeffs))).astype(np.float32)
    return dict(src=ks[pick], order=ko[pick], tri1=k1[pick], tri2=k2[pick], e=e, t=t, d=d)
