"""Dataset, training and evaluation loop of the learned reverb-parameter
estimator, over the C ABI (every step runs in the library's kernels; this
module only orders the calls and moves indices).

  trace_rooms     trace one source-listener pair per room with the batched
                  persistent launch, in chunks, keeping the reverb parameters
                  and, if asked, the BF16 features of the histograms
  make_dataset    features of a cheap trace + targets from a converged trace
  train           minibatch Adam on the GPU (Gaussian NLL)
  predict         features -> network output -> reverb parameters + gate
  rt60_error      per-band relative RT60 error against reference parameters

A room is a scene dict (verts, tris, tri_mat, absorption, scattering) with one
source and one listener (as `rpr_scenes.learn_room` builds them).  Seeds: the
pair of room r traced with `seed_offset` uses the Philox key r + seed_offset,
so the cheap input, the training target and the evaluation reference of one
room are independent streams.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import (Batch, Model, Scene, decode, feature_stats, featurize, normalize, ood_gate, params_host, targets,
               LEARN_DIMS, STAT_FEATURES, ST_BAD_FIT, ST_NO_ENERGY, ST_NO_RANGE)

SH_ORDER = 3
MAX_BOUNCES = 1000
INPUT = dict(n_bins=200, bin_width_s=0.01)       # 1k-ray input histogram: 200 bins of 10 ms
CONVERGED = dict(n_bins=2000, bin_width_s=0.001)  # targets and references: 2000 bins of 1 ms
SEED_INPUT = 1 << 32
SEED_TARGET = 1 << 33
SEED_REFERENCE = 1 << 34
SEED_SWEEP = 1 << 35  # + n_rays: the plain method's own traces in the ray-count sweep
INVALID_FIT = ST_NO_ENERGY | ST_BAD_FIT | ST_NO_RANGE
OOD_ZMAX = 6.0  # statistics features further than this many training std devs: outside the training support


def room_pairs(rooms, n_rays, seed_offset, max_bounces=MAX_BOUNCES):
    return [dict(scene=i, source=r["sources"][0], listener=r["listener"], radius=r["radius"], n_rays=int(n_rays),
                 max_bounces=int(max_bounces), seed=int(r["seed"]) + int(seed_offset), pair_id=0)
            for i, r in enumerate(rooms)]


def trace_rooms(scenes, rooms, *, n_rays, n_bins, bin_width_s, seed_offset, want_features=False, chunk=512,
                device="cuda", log=None, method="source", order=0):
    """Trace every room once (one pair each) in chunks of `chunk` pairs, from
    the source (method "source") or from the listener with next-event
    queries toward the source ("listener").  Returns dict(params uint8
    [n][752] on the device, features int16 [n][F] (BF16 bits) and e_in [n]
    if want_features, segments, seconds)."""
    import torch
    n = len(rooms)
    out = dict(params=torch.empty((n, 752), dtype=torch.uint8, device=device), segments=0, seconds=0.0)
    nc = (SH_ORDER + 1) ** 2
    nb = scenes[0].n_bands
    if want_features:
        out["features"] = torch.empty((n, n_bins * nb * nc + STAT_FEATURES), dtype=torch.int16, device=device)
        out["e_in"] = torch.empty(n, dtype=torch.float32, device=device)
    pairs = room_pairs(rooms, n_rays, seed_offset)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        sub = [dict(p, scene=p["scene"] - c0, pair_id=k) for k, p in enumerate(pairs[c0:c1])]
        t0 = time.perf_counter()
        b = Batch(scenes[c0:c1], sub, n_bins=n_bins, sh_order=SH_ORDER, bin_width_s=bin_width_s, autotune=False,
                  use_graph=False, late=False, device=device, method=method, order=order)
        b.run()
        if want_features:
            f, e = featurize(b.hist, n_bins, nb, nc, stats=b.stats)
            out["features"][c0:c1] = f
            out["e_in"][c0:c1] = e
        out["params"][c0:c1] = b.params
        torch.cuda.synchronize()
        out["seconds"] += time.perf_counter() - t0
        from . import stats_host
        out["segments"] += int(stats_host(b.stats)["n_segments"].sum())
        b.close()
        if log:
            log(f"  traced rooms {c0}..{c1 - 1} at {n_rays} rays ({out['seconds']:.1f} s)")
    return out


def make_scenes(rooms, device="cuda"):
    return [Scene.from_dict(r, device=device) for r in rooms]


def make_dataset(scenes, rooms, *, n_input=1024, n_target=262144, inputs_per_room=1, chunk=512, log=None):
    """Features of n_input-ray traces (200 x 10 ms bins) and the targets from
    the reverb parameters of an independent n_target-ray trace (2000 x 1 ms
    bins).  With inputs_per_room = k > 1 every room is traced k times at
    n_input rays with independent keys (SEED_INPUT + j 2^36), giving k rows
    that share one converged target: the network then sees several noisy
    views of each room.  Returns dict(features, e_in, t, w, target_params)
    with rows ordered room-major."""
    import torch
    nb = scenes[0].n_bands
    conv = trace_rooms(scenes, rooms, n_rays=n_target, seed_offset=SEED_TARGET, chunk=chunk, log=log, **CONVERGED)
    feats, e_ins, ts, ws = [], [], [], []
    secs, segs = conv["seconds"], conv["segments"]
    for j in range(inputs_per_room):
        cheap = trace_rooms(scenes, rooms, n_rays=n_input, seed_offset=SEED_INPUT + (j << 36), want_features=True,
                            chunk=chunk, log=log, **INPUT)
        t, w = targets(conv["params"], cheap["e_in"], nb)
        feats.append(cheap["features"])
        e_ins.append(cheap["e_in"])
        ts.append(t)
        ws.append(w)
        secs += cheap["seconds"]
        segs += cheap["segments"]
    k = inputs_per_room

    def interleave(xs):
        return torch.stack(xs, dim=1).reshape((-1,) + tuple(xs[0].shape[1:])) if k > 1 else xs[0]

    return dict(features=interleave(feats), e_in=interleave(e_ins), t=interleave(ts), w=interleave(ws),
                target_params=conv["params"], trace_seconds=secs, segments=segs)


def train(model: Model, data, *, epochs=30, batch=256, lr=1e-3, weight_decay=1e-4, seed=0, log=None):
    """Fit the input normalisation on the dataset's features (per-feature
    mean and scale, the histogram group balanced against the statistics; kept
    as model.input_norm), then minibatch Adam over the normalised rows (a
    fresh permutation per epoch), learning rate decayed by a cosine to 5% of
    `lr`.  Returns the mean loss of each epoch."""
    import torch
    X, t, w = data["features"], data["t"], data["w"]
    n, F = X.shape
    if getattr(model, "input_norm", None) is None:
        model.input_norm = feature_stats(X, F - STAT_FEATURES)
    Xn = normalize(X.clone(), *model.input_norm)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    step = 0
    loss = torch.zeros(steps_per_epoch, dtype=torch.float64, device=X.device)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(device=X.device, dtype=torch.int32)
        for i in range(steps_per_epoch):
            frac = step / max(1, total - 1)
            lr_i = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * frac)))
            model.train_step(Xn, t, w, perm[i * batch:(i + 1) * batch], loss[i:i + 1], lr=lr_i,
                             weight_decay=weight_decay)
            step += 1
        losses.append(float(loss.mean().cpu()))
        if log:
            log(f"  epoch {ep}: loss {losses[-1]:.4f}")
    return losses


def predict(model: Model, features, e_in, n_bands, kappa, in_place=False, zmax=OOD_ZMAX):
    """(params uint8 [n][752], sigma [n][B], uncertain [n]) on the device;
    the features are normalised with model.input_norm first (a copy unless
    in_place).  Rows are uncertain when any band's sigma exceeds kappa or,
    with a fitted normalisation, when a statistics feature lies beyond zmax
    training standard deviations (outside the inputs the network has seen)."""
    f = features if in_place else features.clone()
    norm = getattr(model, "input_norm", None)
    if norm is not None:
        normalize(f, *norm)
    out = model.forward(f)
    params, sigma, unc = decode(out, e_in, n_bands, kappa)
    if norm is not None and zmax is not None:
        F = f.shape[1]
        ood_gate(f, F - STAT_FEATURES, F, zmax, n_bands, params=params, uncertain=unc)
    return params, sigma, unc


def rt60_error(params, ref_params, n_bands):
    """|RT60 - RT60_ref| / RT60_ref per (room, band) on the host, for the
    rooms and bands whose reference fit is valid; an invalid estimate counts
    as an error of 1.  Returns (errors [n][B] with NaN where the reference is
    invalid)."""
    p = params_host(params)
    r = params_host(ref_params)
    B = n_bands
    rt, st = p["rt60"][:, :B].astype(np.float64), p["status"][:, :B]
    rr, sr = r["rt60"][:, :B].astype(np.float64), r["status"][:, :B]
    ref_ok = (rr > 0) & ((sr & INVALID_FIT) == 0)
    est_ok = (rt > 0) & ((st & INVALID_FIT) == 0)
    err = np.where(est_ok, np.abs(rt - rr) / np.where(ref_ok, rr, 1.0), 1.0)
    return np.where(ref_ok, err, np.nan)


def rt60_error_summary(err):
    e = err[np.isfinite(err)]
    return dict(mean=float(e.mean()) if e.size else float("nan"),
                p90=float(np.percentile(e, 90)) if e.size else float("nan"), n=int(e.size))


def choose_kappa(sigma_max, err_learned, err_fallback, target=0.05):
    """Largest threshold kappa on the per-room maximum sigma such that the
    mean error, with rooms above kappa taking the fallback's error, stays at
    or below `target` (errors [rooms][bands], NaN where undefined).  Returns
    (kappa, fallback fraction, mean error); kappa = 0 sends every room to
    the fallback."""
    order = np.argsort(sigma_max)
    el = np.nan_to_num(err_learned, nan=0.0)
    ef = np.nan_to_num(err_fallback, nan=0.0)
    cnt = np.isfinite(err_learned).sum(axis=1)
    n = len(order)
    best = (0.0, 1.0, float(ef.sum() / max(1, cnt.sum())))
    # rooms sorted by sigma: the first j use the network, the rest fall back
    cum_l = np.concatenate([[0.0], np.cumsum(el[order].sum(axis=1))])
    cum_f = np.concatenate([[0.0], np.cumsum(ef[order].sum(axis=1))])
    total = max(1, cnt.sum())
    for j in range(1, n + 1):
        mean = (cum_l[j] + (cum_f[n] - cum_f[j])) / total
        if mean <= target:
            best = (float(sigma_max[order[j - 1]]), 1.0 - j / n, float(mean))
    return best


def timed_plain(scenes, rooms, n_rays, *, steps=3, device="cuda", method="source", order=0):
    """IRs per second of the plain method at n_rays per pair: one graph-
    captured batch (reset, trace, estimate) over all rooms, replayed `steps`
    times after one warm-up.  Returns (IRs/s, params of the last replay)."""
    import torch
    b = Batch(scenes, [dict(p, pair_id=k) for k, p in enumerate(room_pairs(rooms, n_rays, SEED_SWEEP + n_rays))],
              n_bins=CONVERGED["n_bins"], sh_order=SH_ORDER, bin_width_s=CONVERGED["bin_width_s"], autotune=False,
              use_graph=True, late=False, device=device, method=method, order=order)
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    params = b.params.clone()
    b.close()
    return len(rooms) / dt, params


def learned_estimate(model, scenes, rooms, kappa, n_fallback, *, cheap=None, device="cuda", fallback="source"):
    """The learned path for a set of rooms: a 1k-ray trace (one graph replay
    of `cheap`, a planned Batch over the rooms at INPUT bins, built here when
    None), features, network, decoding; rooms whose uncertainty exceeds kappa
    are traced again at n_fallback rays by the plain method (`fallback`:
    "source", or "listener" with next-event queries) and their parameters
    replace the network's.  Returns (params, uncertain mask, cheap batch)."""
    import torch
    nb = scenes[0].n_bands
    nc = (SH_ORDER + 1) ** 2
    if cheap is None:
        cheap = Batch(scenes, [dict(p, pair_id=k) for k, p in enumerate(room_pairs(rooms, 1024, SEED_INPUT))],
                      n_bins=INPUT["n_bins"], sh_order=SH_ORDER, bin_width_s=INPUT["bin_width_s"], autotune=False,
                      use_graph=True, late=False, device=device)
    cheap.run()
    f, e = featurize(cheap.hist, INPUT["n_bins"], nb, nc, stats=cheap.stats)
    params, sigma, unc = predict(model, f, e, nb, kappa, in_place=True)
    idx = torch.nonzero(unc).flatten().to(torch.int32)
    n_fb = int(idx.numel())  # synchronises
    if n_fb:
        sel = idx.cpu().numpy()
        sub_scenes = [scenes[i] for i in sel]
        pairs = [dict(p, scene=k, pair_id=k) for k, p in
                 enumerate(room_pairs([rooms[i] for i in sel], n_fallback, SEED_SWEEP + n_fallback))]
        fb = Batch(sub_scenes, pairs, n_bins=CONVERGED["n_bins"], sh_order=SH_ORDER,
                   bin_width_s=CONVERGED["bin_width_s"], autotune=False, use_graph=False, late=False, device=device,
                   method=fallback, order=2 if fallback == "listener" else 0)
        fb.run()
        from . import params_scatter
        params_scatter(fb.params, idx, params)
        torch.cuda.synchronize()
        fb.close()
    return params, unc, cheap
