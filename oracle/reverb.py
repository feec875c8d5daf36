"""SH-domain Schroeder reverberator: its parameters from the estimated reverb
parameters and the IR, and its audio-rate rendering, FP64 numpy with plain
per-sample loops (Section 4.1 "Sound Rendering": input spatialization, SH
rotations in the comb feedback, directional loudness; Section 4.2: Eq. 7 comb
gains, comb delays drawn around the mean free path, the predelay; Section 5
"Auralization": 8 combs in parallel, 4 all-passes in series).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the bench's CPU baseline,
never by the product library, with which it shares no code.

Readings (the paper leaves these open):
  * comb delays: t_i = m (1 + clamp(z_i, -2.7, 3) / 3) with m = r_free / c
    (mean m, standard deviation m / 3, Section 4.2) and the caller's standard
    normals z_i, then clamped to [1 ms, t_max] (t_max the delay capacity);
    M_i = floor(t_i fs + 1/2) samples.  They are drawn on the first call and
    again only when m differs from the m of the last draw by more than twice
    that draw's sigma; a mean free path <= 0 (no finite segment) keeps the
    last draw;
  * all-passes: delays 4.9, 4.1, 3.4, 2.9 ms (M = floor(t fs + 1/2)), gain 0.7;
  * comb i is Schroeder's, z^-M / (1 - G z^-M) with the SH feedback matrix
    G = g_b,i J_i:  y_i[n] = a_i x[n - M_i] + G y_i[n - M_i], so its first
    output leaves t_comb,i after the input tap;
  * the input tap is the predelay (the first late arrival; the first arrival
    when there is none; 0 when the IR is empty), which the caller's delay line
    applies; the input direction of comb i is read from the all-orders
    histogram at t_first + t_comb,i with t_first that same time: the
    band-summed first-order coefficients, linear between bin starts (zero
    past the last bin), direction (-X_11, -X_1-1, X_10) normalised (Section
    4.1); a zero vector gives an omnidirectional input, a_i = Y_00 e_0 / 8,
    else a_i = Y(dir_i) / 8;
  * rotation of comb i: R_i = Rz(c) Ry(b) Rx(a) from the caller's three angles
    (drawn in [pi/2, 3pi/2]); J(R) maps the SH coefficients of a field to
    those of the field turned by R: J_kk' = integral of Y_k(R v) Y_k'(v) over
    the sphere, exact by the product quadrature below since the integrand is a
    polynomial of degree <= 2n (the paper builds J by the Ivanic recurrence,
    which gives the same matrix);
  * directional loudness: D_b = sum_q w_q g_b(v_q) Y(v_q) Y(v_q)^T with the
    amplitude gain g_b(v) = sqrt(max(0, 4 pi sum_k Xbar_b,k Y_k(v))) (Eq. 1's
    energy distribution, which integrates to 1, rescaled to mean 1 and taken
    to amplitude), over the product quadrature of 8 Gauss-Legendre nodes in
    cos(theta) times 16 equally spaced azimuths (the paper samples a
    spherical t-design); a band with Xbar_00 <= 0 (no energy) gets D = I;
  * rendering, per band b, from zero state: the 8 comb outputs are summed,
    each SH channel passes the 4 all-passes v[n] = -g u[n] + u[n-M] + g v[n-M]
    in series, and the band adds g_reverb,b D_b v[n] to the output.

Parity pins: tests/test_oracle_reverb.py.
"""
from __future__ import annotations

import math

import numpy as np

from . import sh_eval

N_COMB = 8
N_AP = 4
AP_DELAYS_S = (4.9e-3, 4.1e-3, 3.4e-3, 2.9e-3)
AP_GAIN = 0.7
MIN_COMB_S = 1e-3


def samples(t, fs) -> int:
    return int(math.floor(t * fs + 0.5))


def quadrature():
    """Product quadrature: 8 Gauss-Legendre nodes in z times 16 azimuths.
    Returns (dirs [128, 3], weights [128]) with weights summing to 4 pi."""
    z, wz = np.polynomial.legendre.leggauss(8)
    phi = 2 * np.pi * (np.arange(16) + 0.5) / 16
    d, w = [], []
    for zi, wi in zip(z, wz):
        r = math.sqrt(max(0.0, 1 - zi * zi))
        for p in phi:
            d.append((r * math.cos(p), r * math.sin(p), zi))
            w.append(wi * 2 * np.pi / 16)
    return np.array(d), np.array(w)


def rotation(angles):
    """R = Rz(c) Ry(b) Rx(a) for angles (a, b, c) in radians."""
    a, b, c = (float(v) for v in angles)
    Rx = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Rz = np.array([[math.cos(c), -math.sin(c), 0], [math.sin(c), math.cos(c), 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def sh_rotation(R, order):
    """J with J_kk' = integral Y_k(R v) Y_k'(v) dv."""
    d, w = quadrature()
    Y = sh_eval(order, d)
    YR = sh_eval(order, d @ np.asarray(R, np.float64).T)
    return (YR * w[:, None]).T @ Y


def loudness_matrix(xbar, order):
    """D = sum_q w_q g(v_q) Y(v_q) Y(v_q)^T, g = sqrt(max(0, 4 pi xbar . Y));
    the identity when xbar_00 <= 0."""
    nc = (order + 1) ** 2
    xbar = np.asarray(xbar, np.float64)[:nc]
    if not xbar[0] > 0:
        return np.eye(nc)
    d, w = quadrature()
    Y = sh_eval(order, d)
    g = np.sqrt(np.maximum(4 * np.pi * (Y @ xbar), 0.0))
    return (Y * (w * g)[:, None]).T @ Y


def comb_delays(mfp, c, z, t_max, prev=None):
    """Returns (t [8] seconds, mfp of the draw).  prev = (t, mfp_drawn) of the
    last draw, or None."""
    if prev is not None and prev[1] > 0:
        if mfp <= 0:
            return np.array(prev[0], np.float64), prev[1]
        m_prev = prev[1] / c
        if abs(mfp / c - m_prev) <= 2 * (m_prev / 3):
            return np.array(prev[0], np.float64), prev[1]
    m = max(float(mfp), 0.0) / c
    zc = np.clip(np.asarray(z, np.float64), -2.7, 3.0)
    t = np.clip(m * (1 + zc / 3), MIN_COMB_S, t_max)
    return t, (float(mfp) if mfp > 0 else 0.0)


def comb_gains(t, rt60):
    """Eq. 7: g = 10^(-3 t / RT60); 0 where RT60 <= 0.  [bands][combs]."""
    rt = np.asarray(rt60, np.float64)
    g = np.zeros((len(rt), len(t)))
    ok = rt > 0
    g[ok] = 10.0 ** (-3.0 * np.asarray(t, np.float64)[None, :] / rt[ok, None])
    return g


def input_time(params) -> float:
    """t_first: the predelay, else the first arrival, else 0."""
    if params["predelay_s"] >= 0:
        return float(params["predelay_s"])
    if params["first_arrival_s"] >= 0:
        return float(params["first_arrival_s"])
    return 0.0


def input_directions(hist, dt, t_first, t_comb):
    """Dominant direction of comb i from the band-summed first-order
    coefficients at t_first + t_comb,i.  hist [T][B][NC]; returns [8][3]
    (zero rows: no direction)."""
    H = np.asarray(hist, np.float64)
    out = np.zeros((len(t_comb), 3))
    if H.shape[2] < 4:
        return out
    H1 = H[:, :, 1:4].sum(axis=1)  # [T][3]: X_1-1, X_10, X_11
    T = H1.shape[0]

    def at(j):
        return H1[j] if 0 <= j < T else np.zeros(3)

    for i, ti in enumerate(t_comb):
        p = (float(t_first) + float(ti)) / float(dt)
        m = int(math.floor(p))
        f = p - m
        a = at(m) * (1 - f) + at(m + 1) * f
        v = np.array([-a[2], -a[0], a[1]])
        nv = np.linalg.norm(v)
        if nv > 0:
            out[i] = v / nv
    return out


def setup(params, hist, dt, z, angles, *, order, n_bands, fs, c, t_max, prev=None):
    """All reverberator parameters of one IR.  params: the reverb estimate
    (dict with rt60, g_reverb, dir_loudness, predelay_s, first_arrival_s,
    mean_free_path_m); hist [T][B][NC]; z [8]; angles [8][3]; prev: the last
    setup (its t_comb and mfp_drawn are kept while the mean free path stays
    within 2 sigma), or None."""
    nc = (order + 1) ** 2
    B = n_bands
    pv = None if prev is None else (prev["t_comb"], prev["mfp_drawn"])
    t, mfp_drawn = comb_delays(float(params["mean_free_path_m"]), c, z, t_max, pv)
    M = np.array([max(1, samples(ti, fs)) for ti in t])
    t_first = input_time(params)
    dirs = input_directions(hist, dt, t_first, t)
    a = np.zeros((N_COMB, nc))
    y00 = sh_eval(0, np.array([[0.0, 0.0, 1.0]]))[0, 0]
    for i in range(N_COMB):
        if np.linalg.norm(dirs[i]) > 0:
            a[i] = sh_eval(order, dirs[i][None])[0] / N_COMB
        else:
            a[i, 0] = y00 / N_COMB
    J = np.stack([sh_rotation(rotation(angles[i]), order) for i in range(N_COMB)])
    D = np.stack([loudness_matrix(np.asarray(params["dir_loudness"][b]), order) for b in range(B)])
    return dict(t_comb=t, m_comb=M, mfp_drawn=mfp_drawn, predelay_samples=samples(t_first, fs), dir=dirs, a=a,
                J=J, D=D, g_comb=comb_gains(t, np.asarray(params["rt60"][:B])),
                g_reverb=np.asarray(params["g_reverb"][:B], np.float64),
                ap_delays=np.array([samples(td, fs) for td in AP_DELAYS_S]))


def render(x, st, order):
    """x [B][N] band inputs at the predelay tap; st from setup(); returns
    out [(n+1)^2][N] from zero state."""
    nc = (order + 1) ** 2
    x = np.asarray(x, np.float64)
    B, N = x.shape
    out = np.zeros((nc, N))
    M = [int(m) for m in st["m_comb"]]
    for b in range(B):
        u = np.zeros((N, nc))
        for i in range(N_COMB):
            y = np.zeros((N, nc))
            G = st["g_comb"][b, i] * np.asarray(st["J"][i], np.float64)
            a = st["a"][i]
            for n in range(M[i], N):
                y[n] = a * x[b, n - M[i]] + G @ y[n - M[i]]
            u += y
        for Mj in st["ap_delays"]:
            Mj = int(Mj)
            v = np.zeros_like(u)
            for n in range(N):
                v[n] = -AP_GAIN * u[n]
                if n >= Mj:
                    v[n] += u[n - Mj] + AP_GAIN * v[n - Mj]
            u = v
        out += st["g_reverb"][b] * (np.asarray(st["D"][b], np.float64) @ u.T)
    return out
