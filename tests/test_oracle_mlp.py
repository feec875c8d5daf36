"""Pins of the learned estimator's FP64 oracle (oracle/mlp.py) against values
fixed by construction or computed by hand, not by the oracle's own formulas."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _rand_params(dims, seed):
    g = np.random.default_rng(seed)
    return [(g.normal(0, 1.0 / math.sqrt(a), (b, a)), g.normal(0, 0.1, b)) for a, b in zip(dims[:-1], dims[1:])]


def test_bf16_round_known_values_and_torch():
    one = 1.0
    ulp = 2.0 ** -7  # bf16 spacing at 1
    x = np.array([one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + 2 ** -20, -2.5, 0.0, 3.0e38, 1e-40])
    want = np.array([one, one, one + 2 * ulp, one + ulp, -2.5, 0.0, None, None], dtype=object)
    r = M.bf16_round(x)
    for got, w in zip(r[:6], want[:6]):
        assert got == w
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(0)
    v = np.concatenate([g.normal(0, 1, 20000), g.normal(0, 1e-30, 100), g.uniform(-1e30, 1e30, 100)]).astype(np.float32)
    t = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(v), t)


def test_forward_hand_built_relu_network():
    """A network that computes |x0 - x1| + |x2| and a constant 7 (weights set by
    hand, non-square layers so a transposed operand cannot pass)."""
    W0 = np.array([[1, -1, 0], [-1, 1, 0], [0, 0, 1], [0, 0, -1]], float)  # 3 -> 4
    b0 = np.zeros(4)
    W1 = np.array([[1, 1, 0, 0], [0, 0, 1, 1]], float)  # 4 -> 2: |x0-x1|, |x2|
    b1 = np.zeros(2)
    W2 = np.array([[1, 1], [0, 0], [0, 0]], float)  # 2 -> 3
    b2 = np.array([0.0, 2.0, -5.0])
    W3 = np.array([[1, 0, 0], [0, 3.5, 0]], float)  # 3 -> 2
    b3 = np.array([0.0, 0.0])
    P = [(W0, b0), (W1, b1), (W2, b2), (W3, b3)]
    X = np.array([[1.0, 4.0, -2.0], [-3.0, -3.0, 0.5], [0.0, 2.0, 0.0]])
    z, h = M.forward(P, X)
    assert np.array_equal(z[-1], np.array([[5.0, 7.0], [0.5, 7.0], [2.0, 7.0]]))
    assert len(h) == 4 and np.array_equal(h[0], X)


def test_nll_closed_forms():
    mu = np.array([[0.3, -1.0]])
    s = np.array([[0.0, math.log(4.0)]])
    T = np.array([[0.3, 1.0]])
    W = np.ones((1, 2))
    loss, g = M.nll(np.hstack([mu, s]), T, W)
    # target 0: residual 0, s = 0 -> 0; target 1: residual -2, sigma^2 = 4 -> 1/2 (4/4 + ln 4)
    assert loss == pytest.approx(0.5 * (1.0 + math.log(4.0)), rel=1e-15)
    # d/dmu = r e^{-s}: 0 and -2/4; d/ds = (1 - r^2 e^{-s})/2: 1/2 and 0 (s is at its optimum log r^2)
    assert g[0, 0] == 0.0 and g[0, 1] == pytest.approx(-0.5, rel=1e-15)
    assert g[0, 2] == pytest.approx(0.5, rel=1e-15) and abs(g[0, 3]) < 1e-15
    # a masked target contributes nothing
    loss2, g2 = M.nll(np.hstack([mu, s]), T, np.array([[1.0, 0.0]]))
    assert loss2 == 0.0 and np.all(g2[:, [1, 3]] == 0.0)
    # the mean over the batch: two copies give the same loss and half the gradient each
    loss3, g3 = M.nll(np.vstack([np.hstack([mu, s])] * 2), np.vstack([T, T]), np.ones((2, 2)))
    assert loss3 == pytest.approx(loss, rel=1e-15) and np.allclose(g3[0], g[0] / 2, rtol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    dims = [20, 16, 12, 10, 8]
    P = _rand_params(dims, seed)
    g = np.random.default_rng(100 + seed)
    X = g.normal(0, 1, (7, dims[0]))
    T = g.normal(0, 1, (7, 4))
    W = (g.uniform(0, 1, (7, 4)) > 0.2).astype(float)
    loss, grads = M.backward(P, X, T, W)
    h = 1e-6
    for l in range(len(P)):
        for which in (0, 1):
            arr = P[l][which]
            for _ in range(6):
                idx = tuple(int(g.integers(0, n)) for n in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = M.nll(M.forward(P, X)[0][-1], T, W)[0]
                arr[idx] = old - h
                lm = M.nll(M.forward(P, X)[0][-1], T, W)[0]
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[l][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)), (l, which, idx, fd, an)


def test_adam_hand_computed_steps():
    lr = 0.01
    P = [(np.array([[1.0]]), np.array([0.0]))]
    st = {}
    # constant gradient: every bias-corrected step is lr * g / (|g| + eps)
    for k in range(1, 4):
        P = M.adam_step(P, [(np.array([[2.0]]), np.array([-0.5]))], st, lr, eps=0.0)
        assert P[0][0][0, 0] == pytest.approx(1.0 - k * lr, rel=1e-14)
        assert P[0][1][0] == pytest.approx(k * lr, rel=1e-14)
    # sign flip: g1 = +1, g2 = -1 (by hand: m2 = -0.01, v2 = 0.001999,
    # m2_hat = -0.01 / 0.19, v2_hat = 0.001999 / 0.001999 = 1)
    P = [(np.array([[0.0]]), np.array([0.0]))]
    st = {}
    P = M.adam_step(P, [(np.array([[1.0]]), np.array([1.0]))], st, lr, eps=0.0)
    assert P[0][0][0, 0] == pytest.approx(-lr, rel=1e-14)
    P = M.adam_step(P, [(np.array([[-1.0]]), np.array([-1.0]))], st, lr, eps=0.0)
    assert P[0][0][0, 0] == pytest.approx(-lr + lr * 0.01 / 0.19, rel=1e-12)
    # decoupled weight decay scales the matrix, not the bias
    P = [(np.array([[2.0]]), np.array([2.0]))]
    P = M.adam_step(P, [(np.array([[0.0]]), np.array([0.0]))], {}, 0.1, weight_decay=0.5)
    assert P[0][0][0, 0] == pytest.approx(2.0 - 0.1 * 0.5 * 2.0, rel=1e-15) and P[0][1][0] == 2.0


def test_featurize_invariances_and_values():
    g = np.random.default_rng(3)
    H = g.normal(0, 1e-6, (200, 4, 16))
    H[:, :, 0] = np.abs(H[:, :, 0])
    f, e = M.featurize(H)
    assert f.shape == (200 * 4 * 16 + M.STAT_FEATURES,) and e > 0 and not f[-M.STAT_FEATURES:].any()
    # scale invariance (the level is carried by e_in, not by the features)
    f2, e2 = M.featurize(H * 37.0)
    assert np.allclose(f2, f, rtol=1e-12, atol=1e-14) and e2 == pytest.approx(37.0 * e, rel=1e-14)
    # odd in the signed coefficients, zero at zero, bin-major order
    H2 = H.copy()
    H2[5, 2, 7] = -H[5, 2, 7]
    H2[9, 1, 3] = 0.0
    f3, _ = M.featurize(H2)
    assert f3[(5 * 4 + 2) * 16 + 7] == -f[(5 * 4 + 2) * 16 + 7] and f3[(9 * 4 + 1) * 16 + 3] == 0.0
    # a directional value with FEAT_GAIN |u| = e - 1 maps to exactly FEAT_SCALE
    H3 = np.zeros((2, 1, 2))
    H3[0, 0, 0] = 1.0
    e3 = math.sqrt(4 * math.pi)  # e_in of H3
    H3[1, 0, 1] = (math.e - 1.0) / M.FEAT_GAIN * e3
    f4, _ = M.featurize(H3)
    assert f4[3] == pytest.approx(M.FEAT_SCALE, rel=1e-12)
    # no energy: zero features, e_in = 0
    f5, e5 = M.featurize(np.zeros((3, 2, 4)))
    assert e5 == 0.0 and not f5.any()


def test_featurize_decay_channel_closed_form():
    """Channel 0 of a pure exponential decay I[m] = r^m over T bins: the
    backward integral is S[m] = (r^m - r^T) / (1 - r), so the curve is
    10 log10((r^m - r^T) / (1 - r^T)) / 60, clipped at -1; bin 0 holds
    ln(S_b[0] / e_in), 0 when all bands are equal and ln 2 - ln 1.5 for a
    band twice as loud as the other."""
    T, r = 120, 0.9
    m = np.arange(T)
    I = r ** m
    H = np.zeros((T, 2, 4))
    H[:, 0, 0] = I / math.sqrt(4 * math.pi)
    H[:, 1, 0] = 2 * I / math.sqrt(4 * math.pi)
    f, e = M.featurize(H)
    f = f[:-M.STAT_FEATURES].reshape(T, 2, 4)
    want = np.maximum(10 * np.log10((r ** m[1:] - r ** T) / (1 - r ** T)), -60.0) / 60.0
    assert np.allclose(f[1:, 0, 0], want, rtol=1e-12, atol=1e-14)
    assert np.allclose(f[1:, 1, 0], want, rtol=1e-12, atol=1e-14)
    assert np.any(want == -1.0) and np.any(want > -1.0)
    assert f[0, 0, 0] == pytest.approx(math.log(1 / 1.5), rel=1e-12)
    assert f[0, 1, 0] == pytest.approx(math.log(2 / 1.5), rel=1e-12)
    # a band without energy has a zero decay channel
    H[:, 1, 0] = 0.0
    f, _ = M.featurize(H)
    assert not f[:-M.STAT_FEATURES].reshape(T, 2, 4)[:, 1, 0].any()


def test_featurize_statistics_by_hand():
    st = dict(n_rays=1000, e_emitted=0.5, n_segments=50000, n_finite_segments=49000, seg_len_sum=49000 * 7.0,
              n_escaped=10, first_arrival_bin=12, first_late_bin=2**31 - 1,
              e_alive_at_stop=np.array([0.5 * math.exp(-30.0), 0.0]), e_absorbed=np.array([0.25, 0.5]),
              e_escaped=np.array([0.0, 0.05]), e_alive_at_bounce_cap=np.array([0.0, 0.5 * math.exp(-6.0)]))
    H = np.zeros((40, 2, 4))
    H[5, :, 0] = 1.0
    f, e = M.featurize(H, st)
    s = f[-M.STAT_FEATURES:]
    assert s[0] == pytest.approx(math.log(30.0) / 5, rel=1e-12)          # alive, band 0: ln of the decay exponent
    assert s[4] == pytest.approx(math.log(-math.log(1e-300)) / 5, rel=1e-12)  # alive, band 1: floored
    assert s[1] == pytest.approx(math.log(0.5) / 10, rel=1e-12) and s[5] == 0.0  # absorbed
    assert s[2] == pytest.approx(math.log(1e-12) / 10, rel=1e-12)        # escaped, band 0: floored
    assert s[6] == pytest.approx(math.log(0.1) / 10, rel=1e-12)
    assert s[7] == pytest.approx(-6.0 / 60, rel=1e-12)                   # alive at the bounce cap, band 1
    assert s[32] == pytest.approx(math.log(7.0) / 3, rel=1e-12)          # mean free path
    assert s[33] == pytest.approx(math.log(50.0) / 5, rel=1e-12)         # segments per ray
    assert s[34] == pytest.approx(0.01, rel=1e-12)
    assert s[35] == pytest.approx(12 / 40, rel=1e-12) and s[36] == 1.0
    assert not s[8:32].any() and not s[37:].any()
    # no decay at all (alive = emitted): the exponent is floored at 1e-3
    f1, _ = M.featurize(H, dict(st, e_alive_at_stop=np.array([0.5, 0.5])))
    assert f1[-M.STAT_FEATURES] == pytest.approx(math.log(1e-3) / 5, rel=1e-12)
    # the statistics do not depend on the histogram, nor the histogram part on them
    f0, _ = M.featurize(H)
    assert np.array_equal(f[:-M.STAT_FEATURES], f0[:-M.STAT_FEATURES])


def test_targets_and_decode_by_hand():
    prm = dict(rt60=np.array([1.0, 2.0]), status=np.array([0, 2]), e_direct=np.array([0.5, 0.0]),
               e_early=np.array([1.0, 1.0]), e_late=np.array([2.0, 4.0]))
    t, w = M.targets(prm, 2.0, 2)
    assert np.array_equal(w, [1, 0, 1, 1, 1, 1, 1, 1])
    assert t[0] == 0.0
    assert t[2] == pytest.approx(math.log(0.25 + M.ENERGY_FLOOR), rel=1e-15)
    assert t[3] == pytest.approx(math.log(M.ENERGY_FLOOR), rel=1e-15)
    assert t[7] == pytest.approx(math.log(2.0 + M.ENERGY_FLOOR), rel=1e-15)
    out = np.concatenate([t, [0.0, 2 * math.log(0.2), 0, 0, 0, 0, 0, 0]])
    d = M.decode(out, 2.0, 2, kappa=0.5)
    assert d["rt60"][0] == pytest.approx(1.0) and d["sigma"][1] == pytest.approx(0.2)
    assert d["e_direct"][0] == pytest.approx(0.5, rel=1e-12) and d["e_late"][1] == pytest.approx(4.0, rel=1e-12)
    assert d["uncertain"]  # sigma of band 0 is 1 > 0.5
    assert not M.decode(out, 2.0, 2, kappa=1.5)["uncertain"]
    assert M.decode(out, 0.0, 2, kappa=1e9)["uncertain"]


def test_tower_structure_is_the_two_tower_network():
    """A layer 0 rewritten by tower_structure computes, written out by hand:
    the histogram inputs through the tower's own rows (ReLU), then each
    statistic as max(s, 0) and max(-s, 0); the rest of the network as given."""
    g = np.random.default_rng(3)
    n_hist, S, tw = 40, 6, 8
    dims = (n_hist + S, tw + 2 * S, 16, 4)
    params = [(g.normal(0, 0.5, (b, a)), g.normal(0, 0.1, b)) for a, b in zip(dims[:-1], dims[1:])]
    st = M.tower_structure(params, n_hist, tw)
    X = g.normal(0, 1, (9, dims[0]))
    z, _ = M.forward(st, X)
    W0, b0 = params[0]
    tower = np.maximum(X[:, :n_hist] @ W0[:tw, :n_hist].T + b0[:tw], 0.0)
    s = X[:, n_hist:]
    h1 = np.concatenate([tower, np.maximum(s, 0.0), np.maximum(-s, 0.0)], axis=1)
    h2 = np.maximum(h1 @ params[1][0].T + params[1][1], 0.0)
    out = h2 @ params[2][0].T + params[2][1]
    assert np.allclose(z[-1], out, rtol=1e-12, atol=1e-12)
    # the other layers and the tower's own weights are untouched
    assert np.array_equal(st[0][0][:tw, :n_hist], W0[:tw, :n_hist]) and np.array_equal(st[0][1][:tw], b0[:tw])
    assert all(np.array_equal(a[0], b[0]) for a, b in zip(st[1:], params[1:]))
