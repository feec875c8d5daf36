"""Pins of the oracle's listener-origin trace (next-event estimation toward
each source ball, Section 5) against facts fixed outside it: the moments of
the cone sampler, the closed-form direct sound of a ball, the image-source
answer of a specular shoebox, the stationary late field of a closed room
without absorption, the energy budget, and the forward trace of the same
room with the roles of the two points swapped (one estimator scored two
ways, so their expectations are equal).  All CPU-only."""
import math

import numpy as np
import pytest

import rpr_scenes as R
from test_oracle_pins import _direct_bins, _direct_energy, _images_order_1_2, _mean_se


def _batched_listener(orc, scene, listener, sources, radius, nb_total, n_batches, **kw):
    per = nb_total // n_batches
    return [orc.trace_listener(scene, sources, listener, radius, n_rays_total=nb_total, ray_begin=i * per,
                               ray_end=(i + 1) * per, **kw) for i in range(n_batches)]


def test_cone_sampling_moments(orc):
    """Uniform in the cone of half-angle g: cos to the axis is uniform on
    [cos g, 1], so E[cos] = (1 + cos g) / 2 and E[cos^2] = (1 + cg + cg^2) / 3;
    the azimuth is uniform, so the perpendicular part averages to zero."""
    a = np.array([0.3, -0.5, 0.8])
    a /= np.linalg.norm(a)
    for cg in (0.2, 0.9, 0.9995):
        d = orc.cone_batch(5, 3, 2, 7, a, cg, 400000)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
        ct = d @ a
        assert ct.min() >= cg - 1e-12 and ct.max() <= 1.0 + 1e-12
        n = len(d)
        se1 = (1 - cg) / math.sqrt(12 * n)
        assert abs(ct.mean() - (1 + cg) / 2) < 5 * se1
        assert abs((ct**2).mean() - (1 + cg + cg * cg) / 3) < 5 * 2 * se1
        perp = d - ct[:, None] * a
        s_perp = math.sqrt(max(1 - cg * cg, 1e-30))
        assert np.all(np.abs(perp.mean(0)) < 5 * s_perp / math.sqrt(n))


def test_listener_direct_sound_closed_form(orc):
    """K = 0: only the next-event query from the listener contributes.  Its
    expectation is the direct energy of a ball, (1/(4 pi c)) <1/rho^2>_ball,
    per band and per bin (shell areas), and its arrival direction points at
    the source."""
    c = R.tiny_config()
    src, lp, r = c["sources"][0].astype(np.float64), c["listener"].astype(np.float64), c["radius"]
    d = float(np.linalg.norm(src - lp))
    T, dt = 40, 1e-3
    runs = _batched_listener(orc, c, lp, src[None], r, 65536, 16, max_bounces=0, sh_order=1, n_bins=T,
                             bin_width_s=dt, seed=21)
    e, se = _mean_se([x["stats"][0]["e_class"][0][0] for x in runs])
    ref = _direct_energy(d, r)
    assert abs(e - ref) < 5 * se and se < 2e-3 * ref, (e, ref, se)
    I = [math.sqrt(4 * math.pi) * x["hist"][0, :, 0, 0] for x in runs]
    Im, Ise = _mean_se(I)
    ref_bins = _direct_bins(d, r, T, dt)
    nz = ref_bins > 0
    assert np.array_equal(Im > 0, nz)
    assert np.all(np.abs(Im - ref_bins)[nz] < 5 * Ise[nz] + 1e-15)
    H = sum(x["hist"][0] for x in runs)
    for b in range(4):
        assert np.allclose(H[:, b], H[:, 0], rtol=1e-12, atol=0)
    # first-order SH: (-Y_11, -Y_1-1, Y_10) / sqrt(3 / 4 pi) is the direction
    v = np.array([-H[:, 0, 3].sum(), -H[:, 0, 1].sum(), H[:, 0, 2].sum()]) / math.sqrt(3 / (4 * math.pi))
    v /= H[:, 0, 0].sum() / math.sqrt(1 / (4 * math.pi))
    u = (src - lp) / d
    assert np.linalg.norm(v - u * np.dot(v, u)) < 1e-3
    assert 1 - (r / d) ** 2 < np.dot(v, u) < 1.0
    assert all(x["stats"][0]["n_next_event"] == 4096 for x in runs)


@pytest.mark.slow
def test_listener_specular_shoebox_matches_image_sources(orc):
    """Scattering 0: the next-event queries at reflections carry nothing
    (their diffuse share is zero), and the segments after the mirror
    reflections reach the source ball as from the image sources."""
    c = R.tiny_config()
    sc = dict(c, scattering=np.zeros((1, 4), np.float32))
    dims = np.array([10.0, 7.0, 3.0])
    src, lp = c["sources"][0].astype(np.float64), c["listener"].astype(np.float64)
    imgs = _images_order_1_2(src, dims)
    runs = _batched_listener(orc, sc, lp, src[None], c["radius"], 2**22, 32, max_bounces=2, sh_order=0,
                             n_bins=200, bin_width_s=1e-3, seed=22)
    alpha = c["absorption"][0].astype(np.float64)
    for b in range(4):
        e, se = _mean_se([x["stats"][0]["e_class"][1][b] for x in runs])
        ref = sum((1 - alpha[b]) ** o * _direct_energy(float(np.linalg.norm(p - lp)), c["radius"])
                  for p, o in imgs)
        assert abs(e - ref) < 5 * se, (b, e, ref, se)
    e0, se0 = _mean_se([x["stats"][0]["e_class"][0][0] for x in runs])
    assert abs(e0 - _direct_energy(float(np.linalg.norm(src - lp)), c["radius"])) < 5 * se0


@pytest.mark.parametrize("scat", [[0.5, 0.5, 0.5, 0.5], [0.05, 0.35, 0.65, 0.95]])
def test_listener_zero_absorption_late_field(orc, scat):
    """Closed room, no absorption: the late field is uniform and stationary,
    dt / V per bin per unit source energy, in every band, whatever the
    scattering.  Next-event weights that miss a factor (1/pi, the cosine, the
    solid angle), a diffuse continuation that is also scored, or a band that
    takes another band's scattering all move this level."""
    c = R.tiny_config()
    sc = dict(c, absorption=np.zeros((1, 4), np.float32), scattering=np.array([scat], np.float32))
    r = orc.trace_listener(sc, c["sources"], c["listener"], c["radius"], n_rays_total=32768, max_bounces=100000,
                           sh_order=0, n_bins=2000, bin_width_s=1e-3, seed=23)
    st = r["stats"][0]
    assert st["n_escaped"] == 0 and np.all(st["e_absorbed"] == 0)
    I = math.sqrt(4 * math.pi) * r["hist"][0][:, :, 0]
    late = I[300:].mean(axis=0)
    assert np.all(np.abs(late / (1e-3 / 210.0) - 1) < 0.02), late


def test_listener_energy_budget_and_subsets(orc):
    """Open box: absorbed + escaped + alive = emitted in every band (equal
    scattering across bands); disjoint ray ranges add up to the whole and
    keep their per-ray hashes; the path statistics are repeated per source."""
    verts, tris, tm = R.merge(R.box_surfaces((0, 0, 0), (10, 7, 3), faces=("x0", "x1", "y0", "y1", "z0")), [0] * 5)
    sc = dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.array([[0.05, 0.2, 0.5, 0.9]], np.float32),
              scattering=np.full((1, 4), 0.3, np.float32))
    srcs = np.array([[2, 2, 1.5], [8, 5, 2.0]])
    kw = dict(n_rays_total=4096, max_bounces=30, sh_order=1, n_bins=300, bin_width_s=1e-3, seed=24)
    full = orc.trace_listener(sc, srcs, np.array([7, 5, 1.5]), 0.5, want_hash=True, **kw)
    st = full["stats"]
    tot = st[0]["e_absorbed"] + st[0]["e_escaped"] + st[0]["e_alive_at_stop"]
    assert np.allclose(tot, 1.0, atol=1e-12) and st[0]["n_escaped"] > 0
    for k in ("n_segments", "n_escaped", "n_next_event", "seg_len_sum"):
        assert st[0][k] == st[1][k]
    assert not np.allclose(st[0]["e_class"], st[1]["e_class"])
    a = orc.trace_listener(sc, srcs, np.array([7, 5, 1.5]), 0.5, ray_end=1500, want_hash=True, **kw)
    b = orc.trace_listener(sc, srcs, np.array([7, 5, 1.5]), 0.5, ray_begin=1500, want_hash=True, **kw)
    assert np.allclose(a["hist"] + b["hist"], full["hist"], rtol=1e-12, atol=1e-12 * np.abs(full["hist"]).max())
    assert np.array_equal(np.concatenate([a["ray_hash"], b["ray_hash"]]), full["ray_hash"])


def _lroom_scene():
    verts, tris, tm = R.merge(R.lroom((12.0, 10.0, 3.0), (0.5, 0.5)), [0] * 8)
    return dict(verts=verts, tris=tris, tri_mat=tm, absorption=np.array([[0.1, 0.2, 0.3, 0.4]], np.float32),
                scattering=np.array([[0.2, 0.4, 0.6, 0.8]], np.float32))


@pytest.mark.slow
def test_listener_equals_forward_with_roles_swapped(orc):
    """The listener-origin estimate for a source ball at B heard at point A
    scores the paths of a trace from A at the ball around B, so its
    expectation equals the forward trace from a source at A to a listener
    sphere at B: per class, band and 10 ms block of channel 0.  The L-room
    hides B from A, so the occlusion of the next-event queries is exercised
    (no direct sound on either side)."""
    sc = _lroom_scene()
    A, B, r = np.array([11.0, 1.5, 1.5]), np.array([1.5, 9.0, 1.5]), 0.5
    kw = dict(max_bounces=30, sh_order=0, n_bins=200, bin_width_s=1e-3)
    bw = _batched_listener(orc, sc, A, B[None], r, 2**17, 16, seed=25, **kw)
    fw = [orc.trace_ir(sc, A[None], B, r, n_rays_total=2**20, ray_begin=i * 2**16, ray_end=(i + 1) * 2**16,
                       seed=26, **kw) for i in range(16)]
    eb, seb = _mean_se([x["stats"][0]["e_class"] for x in bw])
    ef, sef = _mean_se([x["stats"][0]["e_class"] for x in fw])
    assert np.all(eb[0] == 0) and np.all(ef[0] == 0)
    z = np.abs(eb - ef)[1:] / np.sqrt(seb**2 + sef**2)[1:]
    assert np.all(z < 5), z
    # per ray, the next-event estimate is the less noisy one where reflections are mostly diffuse
    assert np.all(seb[1:, 3] * math.sqrt(2**17) < 0.6 * sef[1:, 3] * math.sqrt(2**20))
    Ib, sIb = _mean_se([x["hist"][0, :, :, 0].reshape(20, 10, 4).sum(1) for x in bw])
    If, sIf = _mean_se([x["hist"][0, :, :, 0].reshape(20, 10, 4).sum(1) for x in fw])
    ok = (Ib > 0) | (If > 0)
    zb = np.abs(Ib - If)[ok] / np.sqrt(sIb**2 + sIf**2)[ok]
    assert np.all(zb < 5), zb.max()
