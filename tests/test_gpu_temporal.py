"""GPU parity of the temporal smoothing entry points (IR cache, Eq. 4
parameter smoothing) against the FP64 oracle, through the C ABI.  Both are
elementwise FP32: a few FP32 roundings per frame, held to 2e-6 relative over
a dozen frames; the first frame copies exactly."""
import math

import numpy as np
import pytest

import paper_1803_00430_amd as P
from oracle import temporal as TC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


def test_ir_cache_matches_oracle(torch_cuda):
    torch = torch_cuda
    g = np.random.default_rng(3)
    n = 3000 * 4 * 16 * 3 + 7  # several histograms and a ragged tail
    a = P.temporal_alpha(0.1, 3.0)
    assert math.isclose(a, TC.smoothing_alpha(0.1, 3.0), rel_tol=1e-6)
    cache = torch.empty(n, dtype=torch.float32, device="cuda")
    ref = None
    for f in range(12):
        x = g.exponential(size=n).astype(np.float32) * (g.uniform(size=n) < 0.7)
        P.ir_cache_update(cache, torch.as_tensor(x, device="cuda"), a, first=(f == 0))
        ref = TC.ema(ref, x.astype(np.float64), a, first=(f == 0))
        got = cache.cpu().numpy().astype(np.float64)
        if f == 0:
            assert np.array_equal(got, x.astype(np.float64))
        assert np.all(np.abs(got - ref) <= 2e-6 * np.abs(ref) + 1e-30), f


def _random_params(g, n, B):
    p = np.zeros(n, P.REVERB_PARAMS_DTYPE)
    p["rt60"][:, :B] = g.uniform(0.2, 3.0, (n, B))
    st = np.where(g.uniform(size=(n, B)) < 0.2, g.choice([1, 2, 4], size=(n, B)), 0)
    st |= np.where(g.uniform(size=(n, B)) < 0.3, 16, 0)  # a flag that does not invalidate the fit
    p["status"][:, :B] = st
    p["rt60"][:, :B] = np.where((st & 7) != 0, 0.0, p["rt60"][:, :B])
    p["rt60_range"][:, :B] = g.integers(0, 4, (n, B))
    for k in ("e_direct", "e_early", "e_late"):
        p[k][:, :B] = g.exponential(1e-3, (n, B))
    p["predelay_s"] = g.uniform(0, 0.05, n)
    return p


def _as_dict(row, B):
    return {k: (row[k][:B].astype(np.float64) if k in ("rt60", "e_direct", "e_early", "e_late", "g_reverb")
                else row[k][:B].copy() if k in ("status", "rt60_range") else row[k]) for k in row.dtype.names}


def test_params_smooth_matches_oracle(torch_cuda):
    torch = torch_cuda
    g = np.random.default_rng(4)
    n, B = 333, 4
    aE, aL = P.temporal_alpha(0.1, 1.0), P.temporal_alpha(0.1, 3.0)
    cache = P.alloc_params(n)
    ref = [None] * n
    for f in range(10):
        fresh = _random_params(g, n, B)
        P.reverb_params_smooth(cache, torch.as_tensor(fresh.view(np.uint8).reshape(n, -1), device="cuda"), B, aE,
                               aL, first=(f == 0))
        got = P.params_host(cache)
        for i in range(n):
            ref[i] = TC.smooth_params(ref[i], _as_dict(fresh[i], B), aE, aL, B)
            r = ref[i]
            assert np.allclose(got["rt60"][i][:B], r["rt60"], rtol=2e-6, atol=0), (f, i)
            assert np.array_equal(got["status"][i][:B], r["status"]), (f, i)
            assert np.array_equal(got["rt60_range"][i][:B], r["rt60_range"]), (f, i)
            for k in ("e_direct", "e_early", "e_late"):
                assert np.allclose(got[k][i][:B], r[k], rtol=2e-6, atol=0), (f, i, k)
            if f > 0:
                assert np.allclose(got["g_reverb"][i][:B], r["g_reverb"], rtol=4e-6, atol=0), (f, i)
            assert got["predelay_s"][i] == np.float32(fresh["predelay_s"][i])


def test_temporal_rejects_bad_arguments(torch_cuda):
    torch = torch_cuda
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(P.RprError):
        P.ir_cache_update(buf[1:17], buf[20:36], 0.5, first=False)  # 4-byte offset: misaligned
    with pytest.raises(P.RprError):
        P.ir_cache_update(buf[:16], buf[16:32], 1.5, first=False)
