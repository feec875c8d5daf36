"""GPU parity of the SH reverberator (reverb_setup, reverb_render) against the
oracle (oracle/reverb.py) on seeded inputs: every setup field, and the
rendered output over several consecutive calls of ragged lengths (delay lines
carried across calls), for SH orders 0-3 and 1, 4 and 8 bands, plus the
full-size workload on sampled sources and the edge cases (empty calls, the
delay capacity, the keep rule of the comb delays, bad arguments)."""
import math

import numpy as np
import pytest

import rpr_scenes as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_1803_00430_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P


def _gpu_params(P, inp):
    n = inp["z"].shape[0]
    a = np.zeros(n, P.REVERB_PARAMS_DTYPE)
    for k in ("rt60", "g_reverb", "dir_loudness", "mean_free_path_m", "predelay_s", "first_arrival_s"):
        a[k] = inp[k]
    return torch.from_numpy(a.view(np.uint8).reshape(n, -1).copy()).cuda()


def _orc_params(inp, i, B, nc):
    return dict(rt60=inp["rt60"][i, :B].astype(np.float64), g_reverb=inp["g_reverb"][i, :B].astype(np.float64),
                dir_loudness=inp["dir_loudness"][i, :B, :nc].astype(np.float64),
                predelay_s=float(inp["predelay_s"][i]), first_arrival_s=float(inp["first_arrival_s"][i]),
                mean_free_path_m=float(inp["mean_free_path_m"][i]))


def _orc_setup(inp, i, desc, prev=None, z=None):
    from oracle import reverb as RV
    B, order = desc.n_bands, desc.sh_order
    nc = (order + 1) ** 2
    return RV.setup(_orc_params(inp, i, B, nc), inp["hist"][i].astype(np.float64), float(np.float32(inp["bin_width_s"])),
                    (inp["z"] if z is None else z)[i].astype(np.float64), inp["angles"][i].astype(np.float64),
                    order=order, n_bands=B, fs=float(np.float32(desc.sample_rate)), c=float(np.float32(desc.speed_of_sound)),
                    t_max=float(np.float32(desc.max_comb_delay_s)), prev=prev)


def _gpu_setup(P, inp, desc, setup=None, first=True, z=None):
    return P.reverb_setup(_gpu_params(P, inp), torch.from_numpy(inp["hist"]).cuda(), inp["bin_width_s"],
                          torch.from_numpy(inp["z"] if z is None else z).cuda(), torch.from_numpy(inp["angles"]).cuda(),
                          desc, setup=setup, first=first)


def _check_setup(g, o, desc, what):
    B, nc = desc.n_bands, (desc.sh_order + 1) ** 2
    assert np.allclose(g["t_comb"], o["t_comb"], rtol=1e-6, atol=0), (what, g["t_comb"], o["t_comb"])
    assert np.array_equal(g["m_comb"], o["m_comb"]), (what, g["m_comb"], o["m_comb"])
    assert abs(g["mfp_drawn"] - o["mfp_drawn"]) <= 1e-6 * abs(o["mfp_drawn"]), what
    assert g["predelay_samples"] == o["predelay_samples"], what
    assert g["n_bands"] == B and g["sh_order"] == desc.sh_order
    assert np.allclose(g["g_comb"][:B], o["g_comb"], rtol=2e-6, atol=1e-30), what
    assert np.all(g["g_comb"][B:] == 0)
    assert np.array_equal(g["g_reverb"][:B], o["g_reverb"].astype(np.float32)), what
    dir_ok = np.linalg.norm(o["dir"], axis=1) > 0
    assert np.array_equal(g["dir"][:, 3] > 0, dir_ok), what
    assert np.allclose(g["dir"][:, :3], o["dir"], atol=2e-5), (what, g["dir"], o["dir"])
    assert np.allclose(g["a"][:, :nc], o["a"], atol=2e-6), what
    assert np.all(g["a"][:, nc:] == 0)
    assert np.allclose(g["J"][:, :nc, :nc], o["J"], atol=3e-6), (what, np.abs(g["J"][:, :nc, :nc] - o["J"]).max())
    assert np.allclose(g["D"][:B, :nc, :nc], o["D"], atol=1e-5 * max(1.0, np.abs(o["D"]).max())), what


def _render_gpu(P, setup, x, desc, chunks):
    st = P.reverb_state(x.shape[0], desc)
    xs = torch.from_numpy(x).cuda()
    outs, n0 = [], 0
    for c in chunks:
        outs.append(P.reverb_render(setup, xs[:, :, n0:n0 + c].contiguous(), st, desc))
        n0 += c
    assert n0 == x.shape[2]
    torch.cuda.synchronize()
    return torch.cat(outs, dim=2).cpu().numpy()


def _check_render(g, o, what):
    scale = max(np.abs(o).max(), 1e-30)
    err = np.abs(g - o).max() / scale
    assert err < 3e-5, (what, err)


CASES = [  # (n_bands, sh_order, sample_rate, seed)
    (4, 1, 44100.0, 11),
    (1, 0, 44100.0, 12),
    (8, 2, 48000.0, 13),
    (4, 3, 16000.0, 14),
]


@pytest.mark.parametrize("nb,order,fs,seed", CASES)
def test_setup_matches_oracle(nb, order, fs, seed):
    P = _P()
    desc = P.reverb_desc(nb, order, fs, 343.0, 0.3)
    inp = R.reverb_inputs(seed, 6, nb, order)
    # edge cases: no late arrival; empty IR; no mean free path; a band without energy or decay; delay cap
    inp["predelay_s"][1] = -1.0
    inp["predelay_s"][2] = inp["first_arrival_s"][2] = -1.0
    inp["mean_free_path_m"][3] = 0.0
    inp["rt60"][4, 0] = 0.0
    inp["dir_loudness"][4, 0] = 0.0
    inp["mean_free_path_m"][5] = 400.0
    g = P.reverb_setup_host(_gpu_setup(P, inp, desc))
    for i in range(6):
        _check_setup(g[i], _orc_setup(inp, i, desc), desc, f"ir {i} {nb}b o{order} {fs}")
    assert (g[5]["m_comb"] == math.floor(float(np.float32(0.3)) * fs + 0.5)).sum() >= 6
    assert np.all(g[3]["t_comb"] == np.float32(1e-3)) and g[3]["mfp_drawn"] == 0


def test_setup_keep_rule_across_frames():
    P = _P()
    desc = P.reverb_desc(4, 1)
    inp = R.reverb_inputs(21, 4, 4, 1)
    inp["mean_free_path_m"][:] = 10.0
    st = _gpu_setup(P, inp, desc)
    prev = [_orc_setup(inp, i, desc) for i in range(4)]
    z2 = (inp["z"] + 0.7).astype(np.float32)
    inp2 = dict(inp, mean_free_path_m=np.array([12.0, 17.0, 0.0, 6.5], np.float32))
    g = P.reverb_setup_host(_gpu_setup(P, inp2, desc, setup=st, first=False, z=z2))
    for i in range(4):
        o = _orc_setup(inp2, i, desc, prev=prev[i], z=z2)
        _check_setup(g[i], o, desc, f"frame 2 ir {i}")
    g0 = P.reverb_setup_host(st)  # the same buffer: updated in place
    assert np.array_equal(g0["t_comb"][0], P.reverb_setup_host(_gpu_setup(P, inp, desc))["t_comb"][0])
    assert g[0]["mfp_drawn"] == 10.0 and g[1]["mfp_drawn"] == 17.0 and g[2]["mfp_drawn"] == 10.0


# plus order 1 with 8 bands, and order 1 with comb delays of a few ms (sub-steps shorter
# than a wave's 64 samples)
RENDER_CASES = [c + ((2.0, 8.0),) for c in CASES] + [(8, 1, 44100.0, 15, (2.0, 8.0)), (4, 1, 44100.0, 16, (0.5, 1.0))]


@pytest.mark.parametrize("nb,order,fs,seed,mfp", RENDER_CASES)
def test_render_matches_oracle(nb, order, fs, seed, mfp):
    """Four consecutive calls of ragged lengths against one oracle run."""
    from oracle import reverb as RV
    P = _P()
    desc = P.reverb_desc(nb, order, fs, 343.0, 0.3)
    n_src = 3
    inp = R.reverb_inputs(seed, n_src, nb, order, mfp_range=mfp)
    setup = _gpu_setup(P, inp, desc)
    N = 2600 if nb < 8 else 1400
    x = R.band_audio(seed + 100, n_src, nb, N)
    chunks = [1000, 1, 511, N - 1512]
    g = _render_gpu(P, setup, x, desc, chunks)
    for s in range(n_src):
        o = RV.render(x[s].astype(np.float64), _orc_setup(inp, s, desc), order)
        _check_render(g[s], o, f"src {s} {nb}b o{order}")


def test_render_delay_capacity_and_impulse():
    """Delays at the capacity (the longest lines) and an impulse input."""
    from oracle import reverb as RV
    P = _P()
    desc = P.reverb_desc(2, 1, 16000.0, 343.0, 0.05)
    inp = R.reverb_inputs(31, 2, 2, 1)
    inp["mean_free_path_m"][:] = 60.0  # t >= 0.0175 s, many combs at the 0.05 s cap
    setup = _gpu_setup(P, inp, desc)
    gs = P.reverb_setup_host(setup)
    assert (gs["m_comb"] == 800).sum() >= 2
    N = 4000
    x = np.zeros((2, 2, N), np.float32)
    x[:, :, 0] = 1.0
    x[1, 1, 37] = -0.5
    g = _render_gpu(P, setup, x, desc, [1234, 2766])
    for s in range(2):
        _check_render(g[s], RV.render(x[s].astype(np.float64), _orc_setup(inp, s, desc), 1), f"src {s}")


def test_render_empty_zero_and_bad_arguments():
    P = _P()
    desc = P.reverb_desc(4, 1)
    inp = R.reverb_inputs(41, 2, 4, 1)
    setup = _gpu_setup(P, inp, desc)
    st = P.reverb_state(2, desc)
    z = torch.zeros((2, 4, 700), dtype=torch.float32, device="cuda")
    out = P.reverb_render(setup, z, st, desc)
    assert torch.all(out == 0)
    e = P.reverb_render(setup, torch.zeros((2, 4, 0), dtype=torch.float32, device="cuda"), st, desc)
    assert e.shape == (2, 4, 0)
    torch.cuda.synchronize()
    assert torch.all(st[:, 64:] == 0)  # the phases move; the lines stay zero
    bad = [P.reverb_desc(0, 1), P.reverb_desc(4, 4), P.reverb_desc(4, 1, 1000.0), P.reverb_desc(4, 1, 44100.0, 0.0),
           P.reverb_desc(4, 1, 44100.0, 343.0, 3.0)]
    for d in bad:
        with pytest.raises(P.RprError):
            P.reverb_state_bytes(d)
    # a misaligned state is refused on the host, before any launch
    with pytest.raises(P.RprError):
        P._check(P.lib().reverb_render(P._ptr(setup), 2, P._ptr(z), 700, P.C.c_void_p(st.data_ptr() + 4), P._ptr(out),
                                       P.C.byref(desc), P._stream(None)))
    with pytest.raises(P.RprError):
        P._check(P.lib().reverb_state_reset(P.C.c_void_p(st.data_ptr() + 4), 1, P.C.byref(desc), P._stream(None)))
    P._check(P.lib().reverb_render(None, 0, None, 0, None, None, P.C.byref(desc), P._stream(None)))


def test_render_delay_change_between_calls_stays_finite():
    """A redraw changes the comb delays of a running reverberator: the lines
    keep their contents (no oracle for the transition); the output stays
    finite and bounded, and a fresh state with the new delays renders as the
    oracle does."""
    from oracle import reverb as RV
    P = _P()
    desc = P.reverb_desc(4, 1, 44100.0)
    inp = R.reverb_inputs(51, 2, 4, 1, mfp_range=(15.0, 20.0))
    setup = _gpu_setup(P, inp, desc)
    st = P.reverb_state(2, desc)
    x = torch.from_numpy(R.band_audio(52, 2, 4, 8000)).cuda()
    P.reverb_render(setup, x[:, :, :4000].contiguous(), st, desc)
    inp2 = dict(inp, mean_free_path_m=np.array([3.0, 40.0], np.float32))
    _gpu_setup(P, inp2, desc, setup=setup, first=False)
    o2 = P.reverb_render(setup, x[:, :, 4000:].contiguous(), st, desc)
    assert torch.isfinite(o2).all() and o2.abs().max() < 100
    g = _render_gpu(P, setup, R.band_audio(53, 2, 4, 3000), desc, [3000])
    for s in range(2):
        o = RV.render(R.band_audio(53, 2, 4, 3000)[s].astype(np.float64), _orc_setup(inp2, s, desc), 1)
        _check_render(g[s], o, f"src {s} after the redraw")


def test_render_full_size_sampled_sources():
    """The bench's workload (2048 sources, 4 bands, order 1, 44.1 kHz, two
    1024-sample blocks) in its launch configuration; sampled sources against
    the oracle."""
    from oracle import reverb as RV
    P = _P()
    n_src, nb, order, n = 2048, 4, 1, 1024
    desc = P.reverb_desc(nb, order, 44100.0, 343.0, 0.3)
    inp = R.reverb_inputs(61, n_src, nb, order, n_bins=40)
    setup = _gpu_setup(P, inp, desc)
    x = R.band_audio(62, n_src, nb, 2 * n)
    g = _render_gpu(P, setup, x, desc, [n, n])
    assert np.isfinite(g).all()
    for s in (0, 777, n_src - 1):
        _check_render(g[s], RV.render(x[s].astype(np.float64), _orc_setup(inp, s, desc), order), f"src {s}")
