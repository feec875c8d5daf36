"""FP64 oracle of the learned reverb-parameter estimator.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: imported by tests/, the
smoke check and the benchmark's CPU leg, never by the product library, and it
shares no code with the HIP path.

The paper has no learned component.  Its low-ray-count denoiser is temporal
smoothing of the estimated parameters (Section 4.2, Eq. 4); the learned
estimator replaces that step: a 4-layer MLP maps the SH x band histogram of a
cheap trace (1k rays, 200 bins of 10 ms) to the parameters that the plain
estimator (Section 4.2) returns on a converged trace, with a per-output
variance.  Everything here is the plain definition, in float64:

  featurize   trace -> input vector: the histogram in its bin-major order
              (per band the Schroeder decay curve in the l = 0 channel, the
              signed log of the energy-normalised directional coefficients)
              followed by 64 features of the trace's statistics
  targets     ReverbParams of a converged trace -> the 4B regression targets
              and their validity mask
  forward     z_l = h_l W_l^T + b_l, h_{l+1} = relu(z_l), last layer linear
  nll         Gaussian negative log-likelihood, mean over the batch
  backward    gradients of nll w.r.t. every W_l and b_l (chain rule)
  adam_step   Adam (Kingma and Ba, 2015) with bias correction and decoupled
              weight decay on the matrices (Loshchilov and Hutter, 2019)
  decode      network output -> per-band RT60, energies, sigma, gate

Pins: tests/test_oracle_mlp.py (a hand-built ReLU network, finite
differences, the Gaussian NLL's closed-form stationary points, hand-computed
Adam steps, bf16 rounding against torch's conversion, featurize invariances).
"""
from __future__ import annotations

import math

import numpy as np

FEAT_GAIN = 1.0e6       # u -> log1p(FEAT_GAIN |u|): -60 dB of u still maps to a value of order 1
FEAT_SCALE = 0.125      # brings the features to order one
DECAY_FLOOR_DB = -60.0  # the decay-curve channel is clipped at -60 dB and scaled to [-1, 0]
STAT_FEATURES = 64      # trace statistics appended to the histogram features (4 per band for up to 8 bands + 5)
ENERGY_FLOOR = 1.0e-4   # log(E / e_in + floor): absent classes (an occluded direct path) stay finite
ST_INVALID_FIT = 1 | 2 | 4   # NO_ENERGY | BAD_FIT | NO_RANGE


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), through
    float32 (exact for values that are already float32)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = r.astype(np.uint32)
    nan = np.isnan(f)
    r[nan] = 0x7FC00000
    return r.view(np.float32).astype(np.float64)


def input_energy(hist):
    """e_in: the mean over bands of the time-integrated intensity,
    (1/B) sum_{m,b} sqrt(4 pi) H[m][b][0] (intensity from the l=0 coefficient,
    as in the estimator of Section 4.2)."""
    H = np.asarray(hist, np.float64)
    return math.sqrt(4.0 * math.pi) * H[:, :, 0].sum() / H.shape[1]


def featurize(hist, stats=None):
    """One trace -> features [T*B*NC + STAT_FEATURES].

    Histogram part (hist [T][B][NC], in the histogram's own order): channel
    k = 0 carries each band's Schroeder decay curve, the backward integral
    S_b[m] = sum_{j>=m} I_b[j] of the intensity I_b = sqrt(4 pi) H_b,0 (summed
    from the last bin down): bin 0 holds ln(S_b[0] / e_in), bins m >= 1 hold
    10 log10(S_b[m] / S_b[0]) / 60 clipped below at -1 (-60 dB).  Channels
    k >= 1 (the directional coefficients) hold sign(u) log1p(FEAT_GAIN |u|)
    FEAT_SCALE with u = H / e_in.  All zero when the trace carries no energy;
    a band without energy has a zero channel 0.

    Statistics part (the same trace's IrStats as a dict, or None for zeros),
    with r(x) = ln(max(x / e_emitted, floor)):
      [4b + 0]  ln(max(-r(e_alive_at_stop[b]), 1e-3)) / 5, floor 1e-300: the
                log of the ray population's decay exponent over the window
                (all rays, not only sphere crossings; a diffuse decay gives
                log RT60 = ln(6 ln 10 x window) - 5 x this)
      [4b + 1]  r(e_absorbed[b]) / 10, floor 1e-30
      [4b + 2]  r(e_escaped[b]) / 10, floor 1e-12
      [4b + 3]  r(e_alive_at_bounce_cap[b]) / 60, floor 1e-30
      [32] ln(mean free path / 1 m) / 3, [33] ln(segments per ray) / 5,
      [34] escaped rays / rays, [35] first arrival bin / T, [36] first late
      bin / T (1 when none); the rest zero.  All zero without rays.
    Returns (features, e_in)."""
    H = np.asarray(hist, np.float64)
    T, B, NC = H.shape
    fs = np.zeros(STAT_FEATURES)
    if stats is not None and stats["n_rays"] > 0 and stats["e_emitted"] > 0:
        em = float(stats["e_emitted"])
        for b in range(B):
            for j, (key, fl, sc) in enumerate((("e_alive_at_stop", 1e-300, 5.0), ("e_absorbed", 1e-30, 10.0),
                                                ("e_escaped", 1e-12, 10.0), ("e_alive_at_bounce_cap", 1e-30, 60.0))):
                r = math.log(max(float(stats[key][b]) / em, fl))
                fs[4 * b + j] = (math.log(max(-r, 1e-3)) if j == 0 else r) / sc
        nf = stats["n_finite_segments"]
        fs[32] = math.log(stats["seg_len_sum"] / nf) / 3.0 if nf > 0 and stats["seg_len_sum"] > 0 else 0.0
        fs[33] = math.log(stats["n_segments"] / stats["n_rays"]) / 5.0
        fs[34] = stats["n_escaped"] / stats["n_rays"]
        fa, fl_ = stats["first_arrival_bin"], stats["first_late_bin"]
        fs[35] = min(fa, T) / T
        fs[36] = min(fl_, T) / T
    e = input_energy(H)
    if not e > 0.0:
        return np.concatenate([np.zeros(H.size), fs]), 0.0
    u = H / e
    f = np.sign(u) * np.log1p(FEAT_GAIN * np.abs(u)) * FEAT_SCALE
    I = math.sqrt(4.0 * math.pi) * H[:, :, 0]
    for b in range(B):
        S = np.cumsum(I[::-1, b])[::-1]
        f[:, b, 0] = 0.0
        if S[0] > 0.0:
            f[0, b, 0] = math.log(S[0] / e)
            with np.errstate(divide="ignore"):
                db = 10.0 * np.log10(S[1:] / S[0])
            f[1:, b, 0] = np.maximum(db, DECAY_FLOOR_DB) / -DECAY_FLOOR_DB
    return np.concatenate([f.reshape(-1), fs]), e


def targets(params, e_in, n_bands):
    """Regression targets of one IR from the estimator output of a converged
    trace (a dict as returned by oracle.estimate_reverb) and the cheap trace's
    e_in: [log RT60_b | log(E_direct_b/e_in + floor) | same for early | late],
    with mask 1 where the target is defined (RT60: a fit without the
    NO_ENERGY, BAD_FIT or NO_RANGE flags and RT60 > 0; energies: e_in > 0)."""
    B = n_bands
    t = np.zeros(4 * B)
    w = np.zeros(4 * B)
    for b in range(B):
        rt = float(params["rt60"][b])
        if rt > 0.0 and not (int(params["status"][b]) & ST_INVALID_FIT):
            t[b] = math.log(rt)
            w[b] = 1.0
        if e_in > 0.0:
            for c, key in enumerate(("e_direct", "e_early", "e_late")):
                t[(c + 1) * B + b] = math.log(float(params[key][b]) / e_in + ENERGY_FLOOR)
                w[(c + 1) * B + b] = 1.0
    return t, w


def _identity(x):
    return x


def forward(params, X, rnd=None):
    """params: list of (W [d_out][d_in], b [d_out]); X [M][d_0].
    Returns (pre-activations z_l, activations h_l with h_0 = X); the network
    output is z[-1].  `rnd`, if given, rounds every activation where it
    enters a product (e.g. bf16_round, to take the ReLU decisions of the next
    layers in the precision of a BF16 implementation); default: exact."""
    r = rnd or _identity
    h = [np.asarray(X, np.float64)]
    z = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        zl = r(h[-1]) @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        z.append(zl)
        if l < L - 1:
            h.append(np.maximum(zl, 0.0))
    return z, h


def nll(out, T, Wm):
    """Mean over the batch of sum_j 1/2 w_j ((mu_j - t_j)^2 exp(-s_j) + s_j),
    out = [mu | s] with s = log sigma^2.  Returns (loss, d loss / d out)."""
    out = np.asarray(out, np.float64)
    M, n2 = out.shape
    n = n2 // 2
    mu, s = out[:, :n], out[:, n:]
    r = mu - T
    e = np.exp(-s)
    loss = 0.5 * np.sum(Wm * (r * r * e + s)) / M
    g = np.empty_like(out)
    g[:, :n] = Wm * r * e / M
    g[:, n:] = 0.5 * Wm * (1.0 - r * r * e) / M
    return loss, g


def backward(params, X, T, Wm, rnd=None):
    """Loss and its gradients [(dW_l, db_l)] by the chain rule.  `rnd` as in
    forward, applied also to the gradient where it enters a product (the
    bias gradient sums the unrounded gradient)."""
    r = rnd or _identity
    z, h = forward(params, X, rnd)
    loss, g = nll(z[-1], T, Wm)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W = np.asarray(params[l][0], np.float64)
        grads[l] = (r(g).T @ r(h[l]), g.sum(axis=0))
        if l > 0:
            g = (r(g) @ W) * (z[l - 1] > 0.0)
    return loss, grads


def tower_structure(params, n_hist, tower_width):
    """Layer 0 as a two-tower layer: rows r < tower_width keep their weights
    on the first n_hist inputs (the histogram) and get zeros on the S
    statistics inputs; row tower_width + j (j < S) passes statistic j through
    with weight +1, row tower_width + S + j with weight -1; those rows' biases
    are 0.  Returns the parameter list with layer 0 rewritten (FP64)."""
    W, b = (np.array(p, np.float64) for p in params[0])
    d1, d0 = W.shape
    S = d0 - n_hist
    assert d1 == tower_width + 2 * S
    W[:tower_width, n_hist:] = 0.0
    W[tower_width:, :] = 0.0
    for j in range(S):
        W[tower_width + j, n_hist + j] = 1.0
        W[tower_width + S + j, n_hist + j] = -1.0
    b[tower_width:] = 0.0
    return [(W, b)] + list(params[1:])


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One Adam step in place.  state: dict(t, m, v) with m, v lists shaped
    like params (created on the first call).  Decoupled weight decay scales
    the matrices only: W -= lr * weight_decay * W."""
    if "m" not in state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W, dtype=np.float64), np.zeros_like(b, dtype=np.float64)) for W, b in params]
        state["v"] = [(np.zeros_like(W, dtype=np.float64), np.zeros_like(b, dtype=np.float64)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    new = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for i, (p, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][l][i]
            v = state["v"][l][i]
            m *= beta1
            m += (1.0 - beta1) * g
            v *= beta2
            v += (1.0 - beta2) * g * g
            step = (m / c1) / (np.sqrt(v / c2) + eps)
            p = np.asarray(p, np.float64)
            if i == 0 and weight_decay:
                p = p - lr * weight_decay * p
            out.append(p - lr * step)
        new.append((out[0], out[1]))
    return new


def decode(out, e_in, n_bands, kappa):
    """Network output [mu | s] of one IR -> dict(rt60, sigma (per RT60 output,
    sigma = exp(s/2), the standard deviation of log RT60), e_direct, e_early,
    e_late, uncertain).  The IR is uncertain when it carried no energy or when
    any band's sigma exceeds kappa; the caller then re-traces it."""
    out = np.asarray(out, np.float64)
    B = n_bands
    n = 4 * B
    mu, s = out[:n], out[n:]
    res = dict(rt60=np.exp(mu[:B]), sigma=np.exp(0.5 * s[:B]))
    for c, key in enumerate(("e_direct", "e_early", "e_late")):
        res[key] = np.maximum(np.exp(mu[(c + 1) * B:(c + 2) * B]) - ENERGY_FLOOR, 0.0) * e_in
    res["uncertain"] = bool(not e_in > 0.0 or np.any(res["sigma"] > kappa))
    return res
