"""Learned estimator on the GPU against the FP64 oracle (oracle/mlp.py):
featurisation, targets and decoding element by element; the BF16 MLP's
forward pass, gradients and Adam step per tensor, on BF16-rounded weights and
inputs (the oracle then computes in float64 without intermediate rounding)."""
import math

import numpy as np
import pytest

import paper_1803_00430_amd as P
from oracle import mlp as M

pytestmark = pytest.mark.gpu

# Per-tensor bounds on ||gpu - oracle|| / ||oracle||.  The parity bar is
# against the oracle with its product operands rounded to BF16 where the
# kernels round them (activations and gradients entering a product), so that
# both sides take the ReLU decisions in the same precision.  What remains is
# FP32 accumulation in another order than FP64's, which moves values across
# BF16 rounding boundaries and near-zero pre-activations across the ReLU
# threshold.  That residue was measured on the CPU by running the same
# rounded-operand computation with FP32 accumulation: 3e-8 at the small shape,
# 3.6e-3 for the first layer's weight gradient at the full shape; each
# case's bound (rel_emu) is about three times its measured residue, with a
# floor of 1e-3.  The BF16 roundings themselves move the result away from
# the exact FP64 oracle by an amount the oracle measures on its own (exact vs
# rounded operands, up to ~6% at full size); against the exact oracle the test
# asks for that gap plus rel_emu, and a cosine above COS_EXACT.
COS_EXACT = 0.995


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


def bf16_bits_to_f64(bits):
    b = np.asarray(bits).view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def f64_to_bf16_bits(x):
    f = M.bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def split_params(vec, dims):
    out, o = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = vec[o:o + a * b].reshape(b, a)
        o += a * b
        out.append((W, vec[o:o + b]))
        o += b
    return out


def rel_cos(g, o):
    g = np.asarray(g, np.float64).ravel()
    o = np.asarray(o, np.float64).ravel()
    rel = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-300)
    cos = float(g @ o / max(np.linalg.norm(g) * np.linalg.norm(o), 1e-300))
    return rel, cos


def random_hist(g, n, T, B, NC):
    H = g.normal(0, 1e-6, (n, T, B, NC)) * np.exp(-np.arange(T) / (0.2 * T))[None, :, None, None]
    H[..., 0] = np.abs(H[..., 0])
    H[:, : T // 10] = 0.0  # nothing before the first arrival
    H[-1] = 0.0            # an IR without energy
    return H.astype(np.float32)


def random_stats(g, n, B, T):
    st = np.zeros(n, P.IR_STATS_DTYPE)
    st["n_rays"] = g.integers(100, 2000, n)
    st["e_emitted"] = st["n_rays"] / 2048.0
    st["n_segments"] = st["n_rays"] * g.integers(5, 300, n)
    st["n_finite_segments"] = st["n_segments"] - g.integers(0, 50, n)
    st["seg_len_sum"] = st["n_finite_segments"] * g.uniform(1, 20, n)
    st["n_escaped"] = g.integers(0, 50, n)
    st["first_arrival_bin"] = g.integers(0, T, n)
    st["first_late_bin"] = np.where(g.uniform(0, 1, n) < 0.3, P.INT32_MAX, g.integers(0, T, n))
    for k, lo, hi in (("e_alive_at_stop", -80, 0), ("e_absorbed", -5, 0), ("e_escaped", -40, -1),
                      ("e_alive_at_bounce_cap", -90, -1)):
        st[k][:, :B] = st["e_emitted"][:, None] * np.exp(g.uniform(lo, hi, (n, B)))
    st["e_escaped"][0, :B] = 0.0
    st[-1]["n_rays"] = 0  # a trace without rays: zero statistics block
    return st


def stats_dict(row):
    return {k: row[k] for k in row.dtype.names}


@pytest.mark.parametrize("T,B,NC", [(200, 4, 16), (37, 3, 9)])
def test_featurize_matches_oracle(torch, T, B, NC):
    g = np.random.default_rng(T)
    H = random_hist(g, 5, T, B, NC)
    st = random_stats(g, 5, B, T)
    f, e = P.featurize(torch.as_tensor(H, device="cuda"), T, B, NC,
                       stats=torch.as_tensor(st.view(np.uint8).reshape(5, -1), device="cuda"))
    torch.cuda.synchronize()
    fg = bf16_bits_to_f64(f.cpu().numpy())
    eg = e.cpu().numpy()
    assert fg.shape == (5, T * B * NC + P.STAT_FEATURES)
    for i in range(H.shape[0]):
        fo, eo = M.featurize(H[i].astype(np.float64), stats_dict(st[i]))
        assert eg[i] == pytest.approx(eo, rel=1e-6, abs=0)
        # the GPU computes u and log1p in FP32 (the decay curve and the
        # statistics in FP64) and rounds once to BF16: within one BF16 unit in
        # the last place of the oracle's value, plus an absolute floor for
        # values that are zero up to the rounding of e_in's sum
        tol = np.abs(fo) * 2.0 ** -7 + 1e-12
        assert np.all(np.abs(fg[i] - fo) <= tol), (i, np.argmax(np.abs(fg[i] - fo) - tol))
    assert not fg[-1].any() and eg[-1] == 0.0


def test_feature_stats_and_normalize(torch):
    """Input normalisation: per-feature mean and population std (FP64), the
    histogram group's gain sqrt(n_stats / n_hist), and the in-place affine map,
    against numpy on the same BF16 values."""
    g = np.random.default_rng(4)
    n, F, F_hist = 333, 200, 136
    X = g.normal(0, 1, (n, F)) * g.uniform(0.01, 3.0, F) + g.normal(0, 2, F)
    X[:, 5] = 0.25  # a constant feature: std floored at 1e-3
    Xb = f64_to_bf16_bits(X)
    xd = torch.as_tensor(Xb, device="cuda")
    mean, scale = P.feature_stats(xd, F_hist)
    P.normalize(xd, mean, scale)
    torch.cuda.synchronize()
    Xf = bf16_bits_to_f64(Xb)
    mu = Xf.mean(axis=0)
    gain = np.where(np.arange(F) < F_hist, math.sqrt((F - F_hist) / F_hist), 1.0)
    sc = gain / np.maximum(Xf.std(axis=0), 1e-3)
    assert np.allclose(mean.cpu().numpy(), mu, rtol=1e-6, atol=1e-7)
    assert np.allclose(scale.cpu().numpy(), sc, rtol=1e-6)
    want = (Xf - mean.cpu().numpy().astype(np.float64)) * scale.cpu().numpy().astype(np.float64)
    got = bf16_bits_to_f64(xd.cpu().numpy())
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -7 + 1e-6)


def test_ood_gate_flags_rows_outside_the_training_support(torch):
    g = np.random.default_rng(8)
    n, F, c0 = 50, 128, 96
    X = g.normal(0, 1, (n, F))
    X[:, c0:] = np.clip(X[:, c0:], -5.9, 5.9)
    X[7, c0 + 3] = 6.5     # beyond +6 in the gated columns
    X[11, c0 + 30] = -8.0
    X[13, 10] = 50.0       # outside the gated columns: ignored
    xd = torch.as_tensor(f64_to_bf16_bits(X), device="cuda")
    prm = P.alloc_params(n)
    prm.zero_()
    unc = torch.zeros(n, dtype=torch.int32, device="cuda")
    P.ood_gate(xd, c0, F, 6.0, 4, params=prm, uncertain=unc)
    torch.cuda.synchronize()
    u = unc.cpu().numpy()
    assert set(np.nonzero(u)[0]) == {7, 11}
    st = P.params_host(prm)["status"]
    assert np.all(st[[7, 11], :4] == P.ST_UNCERTAIN) and not st[np.setdiff1d(np.arange(n), [7, 11])].any()


def test_targets_and_decode_match_oracle(torch):
    g = np.random.default_rng(1)
    n, B = 64, 4
    prm = np.zeros(n, P.REVERB_PARAMS_DTYPE)
    prm["rt60"][:, :B] = g.uniform(0.05, 20.0, (n, B))
    prm["status"][:, :B] = g.choice([0, 0, 0, P.ST_BAD_FIT, P.ST_TAIL_COMPENSATED, P.ST_NO_RANGE], (n, B))
    prm["rt60"][prm["status"] & (P.ST_BAD_FIT | P.ST_NO_RANGE) > 0] = 0.0
    for k in ("e_direct", "e_early", "e_late"):
        prm[k][:, :B] = g.uniform(0, 1e-3, (n, B)) * (g.uniform(0, 1, (n, B)) > 0.1)
    e_in = g.uniform(1e-4, 2e-3, n).astype(np.float32)
    e_in[3] = 0.0
    ref = torch.as_tensor(prm.view(np.uint8).reshape(n, -1), device="cuda")
    t, w = P.targets(ref, torch.as_tensor(e_in, device="cuda"), B)
    torch.cuda.synchronize()
    t, w = t.cpu().numpy(), w.cpu().numpy()
    for i in range(n):
        d = {k: prm[k][i] for k in ("rt60", "status", "e_direct", "e_early", "e_late")}
        to, wo = M.targets(d, float(e_in[i]), B)
        assert np.array_equal(w[i], wo), i
        assert np.allclose(t[i][wo > 0], to[wo > 0], rtol=1e-6, atol=1e-6), i
    out = np.concatenate([g.normal(0, 1, (n, 4 * B)), g.normal(-3, 1.5, (n, 4 * B))], axis=1).astype(np.float32)
    kappa = 0.3
    pg, sg, ug = P.decode(torch.as_tensor(out, device="cuda"), torch.as_tensor(e_in, device="cuda"), B, kappa)
    torch.cuda.synchronize()
    pg = P.params_host(pg)
    sg, ug = sg.cpu().numpy(), ug.cpu().numpy()
    for i in range(n):
        d = M.decode(out[i].astype(np.float64), float(e_in[i]), B, kappa)
        assert bool(ug[i]) == d["uncertain"], i
        assert np.allclose(pg["rt60"][i][:B], d["rt60"], rtol=1e-6)
        assert np.allclose(sg[i], d["sigma"], rtol=1e-6)
        for k in ("e_direct", "e_early", "e_late"):
            assert np.allclose(pg[k][i][:B], d[k], rtol=1e-5, atol=1e-12), (i, k)
        assert np.all(pg["status"][i][:B] == (P.ST_LEARNED | (P.ST_UNCERTAIN if d["uncertain"] else 0)))


CASES = [
    # (dims, batch rows, rel_emu): ragged batch and layer widths that are not
    # multiples of the 64-wide tile; the full shape of the learned estimator
    ((160, 96, 64, 96, 32), 45, 1e-3),
    (P.LEARN_DIMS, 64, 1e-2),
]


def _setup(torch, dims, m, seed):
    g = np.random.default_rng(seed)
    model = P.Model(dims, max_batch=max(m, 64), seed=seed)
    n_params = model.n_params
    vec = np.concatenate([np.concatenate([g.uniform(-1, 1, b * a) * math.sqrt(6.0 / a) * (0.3 if l == len(dims) - 2
                                                                                            else 1.0),
                                          g.normal(0, 0.05, b)])
                          for l, (a, b) in enumerate(zip(dims[:-1], dims[1:]))]).astype(np.float32)
    assert vec.size == n_params
    model.load(torch.as_tensor(vec, device="cuda"))
    n_rows = m + 7
    X = g.normal(0, 0.5, (n_rows, dims[0]))
    Xb = f64_to_bf16_bits(X)
    nt = dims[-1] // 2
    T = g.normal(0, 1, (n_rows, nt)).astype(np.float32)
    W = (g.uniform(0, 1, (n_rows, nt)) > 0.15).astype(np.float32)
    return model, vec, Xb, T, W


@pytest.mark.parametrize("dims,m,rel_emu", CASES)
def test_forward_matches_oracle(torch, dims, m, rel_emu):
    model, vec, Xb, T, W = _setup(torch, dims, m, 11)
    out = model.forward(torch.as_tensor(Xb[:m], device="cuda"))
    torch.cuda.synchronize()
    # the GPU multiplies the BF16 copies of the FP32 weights
    params = [(M.bf16_round(Wl), bl.astype(np.float64)) for Wl, bl in split_params(vec.astype(np.float64), dims)]
    z, _ = M.forward(params, bf16_bits_to_f64(Xb[:m]))
    ze, _ = M.forward(params, bf16_bits_to_f64(Xb[:m]), rnd=M.bf16_round)
    rel, cos = rel_cos(out.cpu().numpy(), ze[-1])
    assert rel <= rel_emu, rel
    gap, _ = rel_cos(ze[-1], z[-1])
    rel, cos = rel_cos(out.cpu().numpy(), z[-1])
    assert rel <= gap + rel_emu and cos >= COS_EXACT, (rel, gap, cos)
    # more rows than max_batch: chunked
    big = np.concatenate([Xb] * ((3 * model.max_batch) // Xb.shape[0] + 1))[: 2 * model.max_batch + 3]
    outb = model.forward(torch.as_tensor(big, device="cuda"))
    out1 = model.forward(torch.as_tensor(big[-5:], device="cuda"))
    torch.cuda.synchronize()
    assert torch.allclose(outb[-5:], out1, rtol=1e-5, atol=1e-6)
    model.close()


@pytest.mark.parametrize("dims,m,rel_emu", CASES)
def test_gradients_and_adam_match_oracle(torch, dims, m, rel_emu):
    model, vec, Xb, T, W = _setup(torch, dims, m, 12)
    g = np.random.default_rng(99)
    n_rows = Xb.shape[0]
    rows = g.permutation(n_rows)[:m].astype(np.int32)
    rows[3] = n_rows + 5  # out of range: a zero row with zero weight
    dev = dict(X=torch.as_tensor(Xb, device="cuda"), T=torch.as_tensor(T, device="cuda"),
               W=torch.as_tensor(W, device="cuda"), rows=torch.as_tensor(rows, device="cuda"))
    loss = model.backward(dev["X"], dev["T"], dev["W"], rows=dev["rows"])
    gr = model.grads()
    torch.cuda.synchronize()
    params = [(M.bf16_round(Wl), bl.astype(np.float64)) for Wl, bl in split_params(vec.astype(np.float64), dims)]
    Xo = np.zeros((m, dims[0]))
    To = np.zeros((m, dims[-1] // 2))
    Wo = np.zeros_like(To)
    for i, r in enumerate(rows):
        if r < n_rows:
            Xo[i], To[i], Wo[i] = bf16_bits_to_f64(Xb[r]), T[r], W[r]
    lo, go = M.backward(params, Xo, To, Wo)
    le, ge = M.backward(params, Xo, To, Wo, rnd=M.bf16_round)
    assert float(loss.cpu()[0]) == pytest.approx(le, rel=rel_emu)
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=abs(le - lo) / abs(lo) + rel_emu)
    gg = split_params(gr.cpu().numpy().astype(np.float64), dims)
    for l, ((gW, gb), (oW, ob), (eW, eb)) in enumerate(zip(gg, go, ge)):
        for name, a, b, c in (("W", gW, oW, eW), ("b", gb, ob, eb)):
            rel, cos = rel_cos(a, c)
            assert rel <= rel_emu, (l, name, "bf16 operands", rel, cos)
            gap, _ = rel_cos(c, b)
            rel, cos = rel_cos(a, b)
            assert rel <= gap + rel_emu and cos >= COS_EXACT, (l, name, "exact", rel, gap, cos)
    # one Adam step from the GPU's own gradients: elementwise FP32 vs FP64
    model.adam(1e-3, weight_decay=0.01)
    new = model.save()
    torch.cuda.synchronize()
    want = M.adam_step(split_params(vec.astype(np.float64), dims), gg, {}, 1e-3, weight_decay=0.01)
    got = split_params(new.cpu().numpy().astype(np.float64), dims)
    for (a, b), (c, d) in zip(got, want):
        assert np.allclose(a, c, rtol=1e-5, atol=1e-7) and np.allclose(b, d, rtol=1e-5, atol=1e-7)
    assert model.info()["step"] == 1
    model.close()


def test_training_fits_a_smooth_function(torch):
    """A few hundred train steps on a synthetic regression (targets a smooth
    function of the inputs, noise of known variance): the loss falls and the
    predicted log-variance approaches the noise's."""
    dims = (128, 128, 128, 128, 32)
    g = np.random.default_rng(5)
    n = 4096
    X = g.normal(0, 1, (n, dims[0]))
    A = g.normal(0, 1 / math.sqrt(dims[0]), (dims[0], 16))
    noise = 0.1
    T = (np.tanh(X @ A) + noise * g.normal(0, 1, (n, 16))).astype(np.float32)
    W = np.ones_like(T)
    model = P.Model(dims, max_batch=256, seed=3)
    Xd = torch.as_tensor(f64_to_bf16_bits(X), device="cuda")
    Td, Wd = torch.as_tensor(T, device="cuda"), torch.as_tensor(W, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    first = None
    gen = torch.Generator(device="cpu").manual_seed(0)
    for step in range(600):
        rows = torch.randperm(n, generator=gen)[:256].to(device="cuda", dtype=torch.int32)
        model.train_step(Xd, Td, Wd, rows, loss, lr=2e-3)
        if step == 0:
            torch.cuda.synchronize()
            first = float(loss.cpu()[0])
    out = model.forward(Xd[:1024])
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    mse = np.mean((o[:, :16] - T[:1024]) ** 2)
    assert mse < 0.25 * np.var(T), (mse, np.var(T))
    assert float(loss.cpu()[0]) < first - 1.0, (first, float(loss.cpu()[0]))
    assert np.median(o[:, 16:]) < math.log(0.5 * np.var(T)), np.median(o[:, 16:])
    model.close()


@pytest.mark.parametrize("dims,n_hist,tw,m", [((160, 96, 64, 96, 32), 128, 32, 45),
                                              (P.LEARN_DIMS_TOWER, 12800, P.LEARN_TOWER, 64)])
def test_two_tower_layer_matches_oracle(torch, dims, n_hist, tw, m):
    """reverb_model_set_tower: the forward pass is the oracle's over the
    structured parameters (oracle.mlp.tower_structure), and one backward +
    Adam step equals the oracle's Adam step followed by the structure, whose
    fixed entries come out exact."""
    model, vec, Xb, T, W = _setup(torch, dims, m, 21)
    model.set_tower(n_hist, tw)
    rel_emu = 1e-3 if dims[0] < 1000 else 1e-2
    st = M.tower_structure(split_params(vec.astype(np.float64), dims), n_hist, tw)
    params = [(M.bf16_round(Wl), bl) for Wl, bl in st]
    out = model.forward(torch.as_tensor(Xb[:m], device="cuda"))
    torch.cuda.synchronize()
    ze, _ = M.forward(params, bf16_bits_to_f64(Xb[:m]), rnd=M.bf16_round)
    rel, cos = rel_cos(out.cpu().numpy(), ze[-1])
    assert rel <= rel_emu and cos >= COS_EXACT, (rel, cos)
    rows = np.arange(m, dtype=np.int32)
    dev = dict(X=torch.as_tensor(Xb, device="cuda"), T=torch.as_tensor(T, device="cuda"),
               W=torch.as_tensor(W, device="cuda"), rows=torch.as_tensor(rows, device="cuda"))
    model.backward(dev["X"], dev["T"], dev["W"], rows=dev["rows"])
    gr = model.grads()
    s0 = model.save()
    torch.cuda.synchronize()
    gg = split_params(gr.cpu().numpy().astype(np.float64), dims)
    # the structure was written into the model's own parameters
    have = split_params(s0.cpu().numpy().astype(np.float64), dims)
    assert np.array_equal(have[0][0], st[0][0].astype(np.float32).astype(np.float64))
    model.adam(1e-3, weight_decay=0.01)
    new = model.save()
    torch.cuda.synchronize()
    want = M.tower_structure(M.adam_step(st, gg, {}, 1e-3, weight_decay=0.01), n_hist, tw)
    got = split_params(new.cpu().numpy().astype(np.float64), dims)
    for (a, b), (c, d) in zip(got, want):
        assert np.allclose(a, c, rtol=1e-5, atol=1e-7) and np.allclose(b, d, rtol=1e-5, atol=1e-7)
    S = dims[0] - n_hist
    W0 = got[0][0]
    assert np.all(W0[:tw, n_hist:] == 0.0) and np.all(W0[tw:tw + S, n_hist:] == np.eye(S))
    assert np.all(W0[tw + S:, n_hist:] == -np.eye(S)) and np.all(W0[tw:, :n_hist] == 0.0)
    assert np.all(got[0][1][tw:] == 0.0)
    model.close()
