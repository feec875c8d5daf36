"""Pins of the oracle's SH reverberator (Sections 4.1, 4.2, 5) against facts
fixed outside it: the quadrature's exactness and the orthonormality of the
SH basis, the defining property and the group law of SH rotation matrices
with the closed form of turns about z, the directional-loudness matrix of a
distribution whose amplitude gain is a polynomial (the z-multiplication
recurrence of the SH), the comb-delay rule, and the closed-form impulse
responses of a feedback comb and of Schroeder all-passes, with the decay
rate that Eq. 7 fixes.  CPU-only."""
import math

import numpy as np
import pytest

import oracle
from oracle import reverb as RV


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def test_quadrature_is_exact_and_basis_orthonormal():
    d, w = RV.quadrature()
    assert abs(w.sum() - 4 * math.pi) < 1e-12
    assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-14)
    # integral of z^2k over the sphere is 4 pi / (2k + 1), exact up to degree 15
    for k in range(8):
        assert abs((w * d[:, 2] ** (2 * k)).sum() - 4 * math.pi / (2 * k + 1)) < 1e-12
        assert abs((w * d[:, 0] ** (2 * k)).sum() - 4 * math.pi / (2 * k + 1)) < 1e-12
    Y = oracle.sh_eval(3, d)
    assert np.allclose((Y * w[:, None]).T @ Y, np.eye(16), atol=1e-12)


def test_sh_rotation_defining_property_and_group_law():
    rng = np.random.default_rng(1)
    for order in (1, 2, 3):
        R1 = RV.rotation(rng.uniform(math.pi / 2, 1.5 * math.pi, 3))
        R2 = RV.rotation(rng.uniform(0, 2 * math.pi, 3))
        J1, J2 = RV.sh_rotation(R1, order), RV.sh_rotation(R2, order)
        assert np.allclose(J1 @ J1.T, np.eye(len(J1)), atol=1e-12)
        # a function turned by R: its coefficients J c, so Y(R v) = J Y(v)
        v = rng.normal(size=(20, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        assert np.allclose(oracle.sh_eval(order, v @ R1.T), oracle.sh_eval(order, v) @ J1.T, atol=1e-12)
        assert np.allclose(RV.sh_rotation(R1 @ R2, order), J1 @ J2, atol=1e-12)
        # no mixing between degrees
        for l in range(order + 1):
            blk = slice(l * l, (l + 1) ** 2)
            off = np.ones(len(J1), bool)
            off[blk] = False
            assert np.allclose(J1[blk][:, off], 0, atol=1e-12)
    # first order: Y_1 = sqrt(3 / 4 pi) (-y, z, -x), so J_1 = P R P^T
    P = np.array([[0, -1, 0], [0, 0, 1], [-1, 0, 0]], np.float64)
    R = RV.rotation((2.0, 2.5, 1.8))
    assert np.allclose(RV.sh_rotation(R, 1)[1:, 1:], P @ R @ P.T, atol=1e-12)


def test_sh_rotation_about_z_closed_form():
    """A turn by phi about z turns the (l, m), (l, -m) pair by m phi: the
    cos(m phi) diagonal and +-sin(m phi) off-diagonal, for every degree."""
    phi = 2.2
    J = RV.sh_rotation(RV.rotation((0, 0, phi)), 3)
    for l in range(4):
        for m in range(0, l + 1):
            kp, kn = l * l + l + m, l * l + l - m
            assert abs(J[kp, kp] - math.cos(m * phi)) < 1e-12
            assert abs(J[kn, kn] - math.cos(m * phi)) < 1e-12
            if m > 0:
                assert abs(abs(J[kp, kn]) - abs(math.sin(m * phi))) < 1e-12
                assert abs(J[kp, kn] + J[kn, kp]) < 1e-12


def _a_lm(l, m):
    return math.sqrt(((l + 1) ** 2 - m * m) / ((2 * l + 1) * (2 * l + 3)))


def test_loudness_matrix_closed_forms():
    """Isotropic (or empty) distribution: D = I.  For f = 3 (1 + z)^2 / (16 pi)
    (integral 1) the gain is g = sqrt(4 pi f) = (sqrt 3 / 2)(1 + z), a
    polynomial, so D = (sqrt 3 / 2)(I + Z) with Z the matrix of z in the SH
    basis: z Y_lm = a_lm Y_l+1,m + a_l-1,m Y_l-1,m."""
    for order in (0, 1, 2, 3):
        nc = (order + 1) ** 2
        iso = np.zeros(nc)
        iso[0] = 1 / math.sqrt(4 * math.pi)
        assert np.allclose(RV.loudness_matrix(iso, order), np.eye(nc), atol=1e-12)
        assert np.array_equal(RV.loudness_matrix(np.zeros(nc), order), np.eye(nc))
    order = 2
    rng = np.random.default_rng(2)
    v = rng.normal(size=(200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = 3 * (1 + v[:, 2]) ** 2 / (16 * math.pi)
    xbar = np.linalg.lstsq(oracle.sh_eval(order, v), f, rcond=None)[0]  # f lies in the span: exact
    assert abs(xbar[0] - 1 / math.sqrt(4 * math.pi)) < 1e-12
    Z = np.zeros((9, 9))
    for l in range(order):
        for m in range(-l, l + 1):
            Z[l * l + l + m, (l + 1) ** 2 + (l + 1) + m] = Z[(l + 1) ** 2 + (l + 1) + m, l * l + l + m] = _a_lm(l, m)
    assert np.allclose(RV.loudness_matrix(xbar, order), math.sqrt(3) / 2 * (np.eye(9) + Z), atol=1e-12)


def test_comb_delay_rule():
    c, tmax = 343.0, 0.3
    z = np.array([0.0, 1.0, -1.0, 2.5, -2.5, 3.5, -5.0, 0.3])
    t, mfp = RV.comb_delays(10.0, c, z, tmax)
    m = 10.0 / c
    assert mfp == 10.0
    assert np.allclose(t[:5], m * (1 + z[:5] / 3), rtol=1e-15)
    assert abs(t[5] - 2 * m) < 1e-15 and abs(t[6] - 0.1 * m) < 1e-15
    # within 2 sigma of the last draw's mean (sigma = m / 3): kept
    for mfp2 in (12.0, 14.0, 6.7, -1.0, 0.0):
        t2, d2 = RV.comb_delays(mfp2, c, z + 1, tmax, prev=(t, mfp))
        assert np.array_equal(t2, t) and d2 == 10.0
    # beyond: drawn again (and the new draw is the reference after that)
    for mfp2 in (17.0, 3.2):
        t2, d2 = RV.comb_delays(mfp2, c, z * 0, tmax, prev=(t, mfp))
        assert np.allclose(t2, mfp2 / c) and d2 == mfp2
    # floor of 1 ms, cap at the capacity, no mean free path yet
    assert np.allclose(RV.comb_delays(0.1, c, z, tmax)[0], 1e-3)
    assert np.allclose(RV.comb_delays(0.0, c, z, tmax)[0], 1e-3) and RV.comb_delays(0.0, c, z, tmax)[1] == 0.0
    assert RV.comb_delays(100.0, c, z, tmax)[0].max() == tmax
    # the Gaussian of Section 4.2: mean m, sigma m / 3 (the clamp moves neither visibly)
    zz = np.random.default_rng(3).normal(size=200000)
    tt = RV.comb_delays(20.0, c, zz, 1.0)[0]
    m = 20.0 / c
    assert abs(tt.mean() / m - 1) < 3e-3 and abs(tt.std() / (m / 3) - 1) < 1e-2


def test_input_directions_interpolate_first_order():
    """Bins j0, j0 + 1 hold energy e1, e2 from directions u1, u2 (first-order
    coefficients e Y_1(u)); at t_first + t = (j0 + 1/4) dt the direction is
    that of 3/4 e1 u1 + 1/4 e2 u2, since (-X_11, -X_1-1, X_10) = sqrt(3/4pi) u."""
    T, B, dt, j0 = 40, 3, 0.01, 7
    u1, u2 = _unit([1, 2, -0.5]), _unit([-2, 0.3, 1])
    H = np.zeros((T, B, 4))
    for b, share in enumerate((0.5, 0.3, 0.2)):
        H[j0, b] = 2.0 * share * oracle.sh_eval(1, u1[None])[0]
        H[j0 + 1, b] = 5.0 * share * oracle.sh_eval(1, u2[None])[0]
    t = np.array([0.25 * dt, 0.0, dt, 0.5 * dt, (T - j0 + 3) * dt, (T - j0 - 1.5) * dt, 0.75 * dt, 0.1 * dt])
    d = RV.input_directions(H, dt, j0 * dt, t)
    assert np.allclose(d[0], _unit(0.75 * 2 * u1 + 0.25 * 5 * u2), atol=1e-12)
    assert np.allclose(d[1], u1, atol=1e-12) and np.allclose(d[2], u2, atol=1e-12)
    assert np.allclose(d[3], _unit(u1 + 2.5 * u2), atol=1e-12)
    assert np.all(d[4] == 0) and np.all(d[5] == 0)  # past the end, or on empty bins: no direction
    assert np.all(RV.input_directions(H[:, :, :1], dt, j0 * dt, t) == 0)
    # t_first: the predelay, else the first arrival, else 0
    assert RV.input_time(dict(predelay_s=0.05, first_arrival_s=0.01)) == 0.05
    assert RV.input_time(dict(predelay_s=-1.0, first_arrival_s=0.01)) == 0.01
    assert RV.input_time(dict(predelay_s=-1.0, first_arrival_s=-1.0)) == 0.0


def _ap_ir(M, g, N):
    """Impulse response of one Schroeder all-pass (-g + z^-M)/(1 - g z^-M):
    -g at 0, (1 - g^2) g^(k-1) at k M."""
    h = np.zeros(N)
    h[0] = -g
    k = np.arange(1, (N - 1) // M + 1)
    h[k * M] = (1 - g * g) * g ** (k - 1)
    return h


def _manual_setup(order, B, M, g, a, J, D=None, g_reverb=None, fs=8000.0):
    nc = (order + 1) ** 2
    return dict(m_comb=np.asarray(M), g_comb=np.asarray(g, np.float64).reshape(B, RV.N_COMB), a=np.asarray(a),
                J=np.asarray(J), D=np.stack([np.eye(nc)] * B) if D is None else D,
                g_reverb=np.ones(B) if g_reverb is None else np.asarray(g_reverb),
                ap_delays=np.array([RV.samples(t, fs) for t in RV.AP_DELAYS_S]))


def test_render_single_comb_closed_form():
    """One scalar comb (others silent): its impulse response is a g^(k-1) at
    k M; the output is that convolved with the four all-pass responses, times
    g_reverb.  The all-pass chain alone has a flat magnitude response."""
    N, M, g, a0 = 3000, 37, 0.93, 0.125
    a = np.zeros((8, 1))
    a[0, 0] = a0
    gc = np.zeros((1, 8))
    gc[0, 0] = g
    st = _manual_setup(0, 1, [M] + [50] * 7, gc, a, np.ones((8, 1, 1)), g_reverb=[1.7])
    x = np.zeros((1, N))
    x[0, 0] = 1.0
    out = RV.render(x, st, 0)[0]
    comb = np.zeros(N)
    k = np.arange(1, (N - 1) // M + 1)
    comb[k * M] = a0 * g ** (k - 1)
    exp = comb
    chain = np.zeros(N)
    chain[0] = 1.0
    for Mj in st["ap_delays"]:
        exp = np.convolve(exp, _ap_ir(int(Mj), RV.AP_GAIN, N))[:N]
        chain = np.convolve(chain, _ap_ir(int(Mj), RV.AP_GAIN, 1 << 16))[: 1 << 16]
    assert np.allclose(out, 1.7 * exp, rtol=0, atol=1e-13)
    assert np.allclose(np.abs(np.fft.rfft(chain)), 1.0, atol=1e-6)


def test_render_rotation_in_feedback_closed_form():
    """First order, one comb fed from direction u with a half-turn about z in
    its feedback: echo k arrives from Rz(pi)^(k-1) u, so its SH coefficients
    are g^(k-1) Y(Rz(pi)^(k-1) u) / 8 (before the per-channel all-passes)."""
    N, M, g = 1500, 29, 0.9
    u = _unit([0.3, -0.8, 0.5])
    R = RV.rotation((0.0, 0.0, math.pi))
    J = np.stack([RV.sh_rotation(R, 1)] * 8)
    a = np.zeros((8, 4))
    a[0] = oracle.sh_eval(1, u[None])[0] / 8
    gc = np.zeros((1, 8))
    gc[0, 0] = g
    st = _manual_setup(1, 1, [M] * 8, gc, a, J)
    x = np.zeros((1, N))
    x[0, 0] = 1.0
    out = RV.render(x, st, 1)
    y = np.zeros((4, N))
    v = u.copy()
    for k in range(1, (N - 1) // M + 1):
        y[:, k * M] = g ** (k - 1) * oracle.sh_eval(1, v[None])[0] / 8
        v = R @ v
    for c in range(4):
        e = y[c]
        for Mj in st["ap_delays"]:
            e = np.convolve(e, _ap_ir(int(Mj), RV.AP_GAIN, N))[:N]
        assert np.allclose(out[c], e, rtol=0, atol=1e-13)


def _params(rt60, mfp, order, B, xbar=None, g_reverb=None, predelay=0.0):
    nc = (order + 1) ** 2
    if xbar is None:
        xbar = np.zeros((B, nc))
        xbar[:, 0] = 1 / math.sqrt(4 * math.pi)
    return dict(rt60=np.asarray(rt60, np.float64), g_reverb=np.ones(B) if g_reverb is None else g_reverb,
                dir_loudness=xbar, predelay_s=predelay, first_arrival_s=predelay, mean_free_path_m=mfp)


@pytest.mark.parametrize("rt60", [0.4, 1.2])
def test_render_decays_60_db_per_rt60(rt60):
    """Eq. 7 sets every comb's loop gain so that it loses 60 dB in RT60
    seconds; the rotations are orthogonal and the all-passes lossless, so the
    output energy of the whole reverberator (8 combs, random rotations,
    order 1) decays at that rate: a least-squares line through the
    backward-integrated energy between -5 and -35 dB gives RT60 within a few
    percent (the echoes of 8 combs are a few ms apart, so single crossings
    are coarser)."""
    fs, order = 8000.0, 1
    rng = np.random.default_rng(4)
    st = RV.setup(_params([rt60], 8.0, order, 1), np.zeros((10, 1, 4)), 0.01, rng.normal(size=8),
                  rng.uniform(math.pi / 2, 1.5 * math.pi, (8, 3)), order=order, n_bands=1, fs=fs, c=343.0, t_max=0.3)
    N = int(1.3 * rt60 * fs)
    x = np.zeros((1, N))
    x[0, :16] = rng.normal(size=16)
    e = (RV.render(x, st, order) ** 2).sum(axis=0)
    sch = np.cumsum(e[::-1])[::-1]
    db = 10 * np.log10(sch / sch[0])
    sel = (db <= -5) & (db >= -35)
    slope = np.polyfit(np.flatnonzero(sel) / fs, db[sel], 1)[0]
    assert abs(-60 / slope / rt60 - 1) < 0.04, -60 / slope


def test_setup_fields_and_kept_delays():
    rng = np.random.default_rng(5)
    order, B, fs = 1, 4, 44100.0
    T, dt = 60, 0.005
    H = np.zeros((T, B, 4))
    u = _unit([1.0, 1.0, 0.0])
    H[10:, :, :] = oracle.sh_eval(1, u[None])[0] * np.exp(-0.1 * np.arange(T - 10))[:, None, None]
    xbar = H.sum(0) / (math.sqrt(4 * math.pi) * H[:, :, 0].sum(0))[:, None]
    p = _params([0.5, 0.8, 1.1, 0.0], 6.0, order, B, xbar=xbar, g_reverb=np.array([0.3, 0.2, 0.1, 0.0]),
                predelay=10 * dt)
    z, ang = rng.normal(size=8), rng.uniform(math.pi / 2, 1.5 * math.pi, (8, 3))
    st = RV.setup(p, H, dt, z, ang, order=order, n_bands=B, fs=fs, c=343.0, t_max=0.3)
    assert np.all(st["m_comb"] == np.floor(st["t_comb"] * fs + 0.5)) and st["mfp_drawn"] == 6.0
    assert st["predelay_samples"] == round(10 * dt * fs)
    assert np.allclose(st["dir"], u, atol=1e-12)  # every comb reads the same direction
    assert np.allclose(st["a"], oracle.sh_eval(1, u[None])[0] / 8, atol=1e-14)
    assert np.all(st["g_comb"][3] == 0) and np.all((st["g_comb"][:3] > 0) & (st["g_comb"][:3] < 1))
    assert list(st["ap_delays"]) == [216, 181, 150, 128]
    for i in range(8):
        assert np.allclose(st["J"][i], RV.sh_rotation(RV.rotation(ang[i]), order), atol=0)
    p2 = dict(p, mean_free_path_m=7.0)
    st2 = RV.setup(p2, H, dt, z + 0.5, ang, order=order, n_bands=B, fs=fs, c=343.0, t_max=0.3, prev=st)
    assert np.array_equal(st2["t_comb"], st["t_comb"]) and st2["mfp_drawn"] == 6.0
