"""Benchmark: ray-bounces/s of the full propagation path on one MI355X.

Workload (the procedural city): 99,996 triangles, 8 sources x 32,768 rays,
up to 100 bounces, 4 bands, SH order 3, 3000 bins of 1 ms, FP32.  One step is
one pass of the hot path over that input: the scene's linear BVH is rebuilt
(scene_create), every source is traced (trace_ir) and the reverb parameters
of the 8 IRs are estimated (estimate_reverb).  `value` is ray-bounces
(closest-hit queries) per second of the whole step.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per k_trace launch on the city workload, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes scaled by a copy kernel of known size
# (profiles/k_trace_city_hbm_counters.md).  Valid only for the trace and build
# sources it was measured on (the build makes the tree the trace reads):
# reported as null once they change.
TRACE_TRAFFIC = {"bytes": 38906512.0,
                 "sources_sha256": "1635a69901fda02eca29bd98a72760f7ec608ea1b60201ea0551edbbe836f110"}
TRACE_SOURCES = ("paper_1803_00430_amd/csrc/trace.hip", "paper_1803_00430_amd/csrc/rpr_device.hpp",
                 "paper_1803_00430_amd/csrc/rpr_internal.hpp", "paper_1803_00430_amd/csrc/trace_acc.hpp",
                 "paper_1803_00430_amd/csrc/lbvh.hip")


# HBM bytes per k_reverb_render launch on the default reverb workload (4096 sources x
# 1024 samples, 4 bands, order 1), from FETCH_SIZE / WRITE_SIZE passes scaled by the same
# copy kernel (profiles/k_reverb_render_hbm_counters.md); null once the sources change.
REVERB_TRAFFIC = {"bytes": 4863029675.0,
                  "sources_sha256": "4908398ff6a22659b2d5684116d9d6e7fa7b304c881150bc1ae06c0a8121f8e2"}
REVERB_SOURCES = ("paper_1803_00430_amd/csrc/reverb.hip", "paper_1803_00430_amd/csrc/rpr_device.hpp",
                  "paper_1803_00430_amd/csrc/rpr_internal.hpp")


def trace_sources_sha256(sources=TRACE_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 60 for the city workload, 20 for the others)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="city: run the steps one after another on one stream (default: pipelined streams)")
    ap.add_argument("--streams", type=int, default=3, help="city: streams the consecutive steps rotate over")
    ap.add_argument("--waves-per-cu", type=int, default=0,
                    help="city: resident trace waves per CU (0: as many as fit); fewer waves refill their lanes")
    ap.add_argument("--cpu-rays", type=int, default=8192, help="rays per source in the oracle sample")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workload", choices=("city", "batch", "learn", "hospital", "rooms", "reverb", "paths", "probe"),
                    default="city",
                    help="city: the single-scene frame (default, the headline line); batch: 256 pairs over "
                         "16 scenes in one persistent graph-captured launch; learn: IRs/s at <= 5%% RT60 error, "
                         "learned estimator vs plain ray trace (builds its dataset and trains first); rooms: "
                         "IRs/s at <= 5%% RT60 error of the plain trace from the sources vs from the listener "
                         "with next-event estimation; reverb: audio-rate rendering of the SH reverberator for "
                         "many sources; paths: early-reflection paths per frame (records, path cache, "
                         "prioritization) on the city")
    ap.add_argument("--learn-train", type=int, default=100000, help="training rooms of the learn workload")
    ap.add_argument("--learn-eval", type=int, default=2048, help="calibration and held-out rooms (each)")
    ap.add_argument("--learn-epochs", type=int, default=16)
    ap.add_argument("--learn-arch", choices=("dense", "tower"), default="tower",
                    help="learn: one dense 12,864 -> 512 first layer, or the histogram through a 64-unit tower "
                         "beside the statistics (reverb_model_set_tower)")
    ap.add_argument("--learn-views", type=int, default=4, help="1k-ray input traces per training room")
    ap.add_argument("--learn-target-rays", type=int, default=65536, help="rays of each training target trace")
    ap.add_argument("--learn-fallback", choices=("source", "listener"), default="listener",
                    help="learn: plain method that traces the uncertain rooms again (at its own N*)")
    ap.add_argument("--learn-target-err", type=float, default=0.048,
                    help="mean RT60 error the gate is tuned to on the calibration rooms (margin below 5%%)")
    ap.add_argument("--rooms-rays", type=int, default=0,
                    help="rooms: skip the references and sweeps, and time only --method at this ray count "
                         "(for profiling)")
    ap.add_argument("--segment-budget", type=int, default=0,
                    help="city: run frames with the sources walking through the streets, tracing each frame with "
                         "a fixed ray count and then under this segment budget per frame (rays chosen from the "
                         "previous frame's segments per ray)")
    ap.add_argument("--frames", type=int, default=8, help="frames of the hospital workload (city: 40 with "
                                                          "--segment-budget)")
    ap.add_argument("--method", choices=("source", "listener"), default="source",
                    help="hospital: trace from every source to the listener sphere (source), or from the "
                         "listener with next-event estimation toward every source ball (listener)")
    ap.add_argument("--rays", type=int, default=0,
                    help="hospital: rays per source (source method) or of the listener (listener method); "
                         "0 = the workload's 131,072")
    ap.add_argument("--temporal", action="store_true",
                    help="hospital: smooth across frames (IR caches with tau 1 s / 3 s and Eq. 4 on the RT60) "
                         "and report the frame-to-frame RT60 jitter")
    ap.add_argument("--convergence", action="store_true",
                    help="hospital: also trace frame 0 with two more independent seeds and report their mean "
                         "RT60 disagreement")
    ap.add_argument("--reference", action="store_true",
                    help="hospital: RT60 of the plain methods against a listener-origin reference traced twice "
                         "with independent seeds (--ref-rays)")
    ap.add_argument("--ref-rays", type=int, default=262144, help="hospital --reference: rays of each reference trace")
    ap.add_argument("--learned", action="store_true",
                    help="hospital: also run the learned estimator inline (trains it first on --learn-train "
                         "rooms), with a ray-trace fallback for uncertain sources")
    ap.add_argument("--reverb-sources", type=int, default=4096, help="reverb: sources rendered per step")
    ap.add_argument("--reverb-block", type=int, default=1024, help="reverb: samples per source per step")
    ap.add_argument("--reverb-order", type=int, default=1, help="reverb: SH order of the rendered channels")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device three times "
                         "(a known-size reference for the HBM byte counters)")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = 60 if a.workload == "city" else 20
    return a


def probe_rate(P, torch, nbytes, pattern, *, grid, block, iters, reps=5):
    """Median rate of `reps` memory-probe launches over a working set of
    `nbytes` (include/rpr.h memory_probe), timed with events on the current
    stream: (GB/s, ms per launch, bytes per launch)."""
    nbytes = max(128, (int(nbytes) + 127) // 128 * 128)
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    sink = torch.empty(grid * block, dtype=torch.float32, device="cuda")
    P.memory_probe(buf, pattern, iters, grid, block, sink)  # first touch: the data enters the caches
    ms = []
    nb = 0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb = P.memory_probe(buf, pattern, iters, grid, block, sink)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    m = float(np.median(ms))
    del buf, sink
    return nb / (m * 1e-3) / 1e9, m, nb


def trace_roof(P, torch, work_bytes, cus):
    """The measured roof of the traversal at its working set: 128-byte lines
    gathered at scattered addresses by the trace's launch shape (one-wave
    workgroups, 16 per compute unit)."""
    grid = cus * 16
    gbs, ms, nb = probe_rate(P, torch, work_bytes, 1, grid=grid, block=64, iters=256)
    return {"gather_gbs": gbs, "working_set_bytes": int(work_bytes), "probe_ms": ms, "probe_bytes": nb,
            "launch": f"{grid} x 64 threads, 256 lines of 128 B per thread"}


def run_probe(a):
    """The bandwidth-vs-working-set curve of the memory hierarchy for the
    traversal's read patterns (memory_probe): streaming reads, independent
    128-byte line gathers (throughput) and dependent line chases (latency),
    from 1 MiB to 8 GiB."""
    import torch

    import paper_1803_00430_amd as P
    cus = P.device_cus()
    sizes = [1 << k for k in range(20, 34)]  # 1 MiB .. 8 GiB
    rows = []
    for ws in sizes:
        it_stream = max(1, (4 << 30) // ws)
        s_gbs, s_ms, _ = probe_rate(P, torch, ws, 0, grid=cus * 8, block=256, iters=it_stream, reps=3)
        g_gbs, g_ms, _ = probe_rate(P, torch, ws, 1, grid=cus * 16, block=64, iters=256, reps=3)
        c_gbs, c_ms, _ = probe_rate(P, torch, ws, 2, grid=cus * 16, block=64, iters=64, reps=3)
        c1_gbs, c1_ms, _ = probe_rate(P, torch, ws, 2, grid=cus, block=64, iters=64, reps=3)
        row = {"working_set_bytes": ws, "stream_gbs": s_gbs, "gather_gbs": g_gbs,
               "chase_ns_loaded": c_ms * 1e6 / 64, "chase_ns_one_wave_per_cu": c1_ms * 1e6 / 64}
        rows.append(row)
        log(f"{ws / 2**20:8.0f} MiB: stream {s_gbs:9.0f} GB/s, gather {g_gbs:9.0f} GB/s, "
            f"chase {row['chase_ns_loaded']:7.0f} ns loaded / {row['chase_ns_one_wave_per_cu']:6.0f} ns alone",
            a.quiet)
    out = {"metric": "memory bandwidth vs working set", "value": max(r["gather_gbs"] for r in rows), "unit": "GB/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "memory_probe over 1 MiB .. 8 GiB: streaming reads (grid CUs x 8 x 256), "
                                  "128-byte line gathers and chases (grid CUs x 16 x 64, the trace's shape)"},
           "curve": rows}
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or '' where there is none."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def run_batch(a):
    """256 source-listener pairs over 16 procedural scenes (shoeboxes, L-rooms,
    cluttered interiors; 1.5k-254k triangles), rays log-uniform in
    [1024, 65536] per pair, 50-200 bounces, SH order 3, 2000 bins of 1 ms.  The
    batch is planned once (pair table upload, launch-shape autotuning, graph
    capture); one step is one graph replay: reset, trace of every pair,
    estimation of every pair."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R

    dev = torch.device("cuda:0")
    cfg = R.batch_config()
    scenes = [P.Scene.from_dict(sd, device=dev) for sd in cfg["scenes"]]
    pairs = []
    for si, sd in enumerate(cfg["scenes"]):
        for p in sd["pairs"]:
            k = len(pairs)
            pairs.append(dict(scene=si, source=p["source"], listener=p["listener"], radius=p["radius"],
                              n_rays=p["n_rays"], max_bounces=p["max_bounces"], seed=cfg["seed_base"] + k,
                              pair_id=k))
    t0 = time.perf_counter()
    b = P.Batch(scenes, pairs, n_bins=cfg["n_bins"], sh_order=cfg["sh_order"], bin_width_s=cfg["bin_width_s"],
                autotune=True, use_graph=True, device=dev)
    plan_s = time.perf_counter() - t0
    info = b.info()
    for _ in range(a.warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = P.stats_host(b.stats)
    segs = int(st["n_segments"].sum())
    ms = wall * 1e3 / a.steps
    out = {
        "metric": "ray-bounces/s", "value": segs * a.steps / wall, "unit": "ray-bounces/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch: 256 source-listener pairs over 16 procedural scenes (1.5k-254k triangles), "
                               "rays 1k-64k per pair, 50-200 bounces, SH order 3, 2000 x 1 ms bins; step = one "
                               "graph replay (reset + trace + estimate)",
                   "pairs": len(pairs), "total_rays": int(info["total_rays"]),
                   "tris": [int(len(sd["tris"])) for sd in cfg["scenes"]]},
        "irs_per_s": len(pairs) / (ms * 1e-3), "segments_per_step": segs, "plan_s": plan_s,
        "launch_shape": {k: info[k] for k in ("waves_per_cu", "order", "chunk_rays", "stack_entries", "fixed_point",
                                             "n_candidates", "best_ms", "worst_ms", "stack_need", "from_cache")},
    }
    print(json.dumps(out), flush=True)


def learned_model(a, P):
    """The estimator's network per --learn-arch: two towers (default) or a dense first layer."""
    if a.learn_arch == "tower":
        model = P.Model(P.LEARN_DIMS_TOWER, max_batch=256, seed=1)
        model.set_tower(P.LEARN_DIMS_TOWER[0] - P.STAT_FEATURES, P.LEARN_TOWER)
        return model
    return P.Model(P.LEARN_DIMS, max_batch=256, seed=1)


def run_learn(a):
    """The learned reverb estimator against the plain method (see
    paper_1803_00430_amd/learn.py).  Rooms: shoeboxes and L-rooms (dims
    U[3,40] m, per-band absorption U[0.02,0.6], scattering U[0.1,0.9]).
    Training set: `--learn-train` rooms x `--learn-views` inputs, input = a
    1,024-ray trace (200 x 10 ms bins x 4 bands x 16 SH coefficients + 64
    trace statistics), target = the estimator's output on an independent
    `--learn-target-rays`-ray trace.  Error = mean over
    held-out rooms x bands of |RT60 - RT60_ref| / RT60_ref, RT60_ref from a
    third independent 262,144-ray trace.  Plain: the smallest ray count of a
    sweep whose error is <= 5% (N*), timed as one graph-captured batch over the
    held-out rooms.  Learned: 1k-ray batch + features + network + decoding,
    rooms whose sigma exceeds kappa (chosen on a calibration split for <= 5%)
    re-traced at N*; timed end to end."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R
    from paper_1803_00430_amd import learn as L

    q = a.quiet
    t_all = time.perf_counter()
    rooms = {"train": [R.learn_room(10000 + i) for i in range(a.learn_train)],
             "cal": [R.learn_room(150000 + i) for i in range(a.learn_eval)],
             "eval": [R.learn_room(200000 + i) for i in range(a.learn_eval)]}
    scenes = {k: L.make_scenes(v) for k, v in rooms.items()}
    t0 = time.perf_counter()
    data = L.make_dataset(scenes["train"], rooms["train"], n_target=a.learn_target_rays,
                          inputs_per_room=a.learn_views, chunk=1024, log=lambda m: log(m, q))
    t_data = time.perf_counter() - t0
    cal = L.make_dataset(scenes["cal"], rooms["cal"], chunk=1024)
    refs = {k: L.trace_rooms(scenes[k], rooms[k], n_rays=262144, seed_offset=L.SEED_REFERENCE, chunk=1024,
                             **L.CONVERGED)["params"] for k in ("cal", "eval")}
    def plain_sweep(method, Ns):
        sw = {}
        for N in Ns:
            tr = L.trace_rooms(scenes["eval"], rooms["eval"], n_rays=N, seed_offset=L.SEED_SWEEP + N, chunk=1024,
                               method=method, order=2 if method == "listener" else 0, **L.CONVERGED)
            sw[N] = L.rt60_error_summary(L.rt60_error(tr["params"], refs["eval"], 4))
            log(f"plain ({method}) N={N}: {sw[N]}", q)
        ok = [N for N in sw if sw[N]["mean"] <= 0.05]
        return sw, (min(ok) if ok else max(sw))

    sweep, n_star = plain_sweep("source", (1024, 4096, 16384, 32768, 65536, 131072, 262144))
    sweep_l, n_star_l = plain_sweep("listener", (4096, 8192, 16384, 32768, 65536))
    fbm = a.learn_fallback
    n_fb = n_star_l if fbm == "listener" else n_star
    model = learned_model(a, P)
    t0 = time.perf_counter()
    losses = L.train(model, data, epochs=a.learn_epochs, lr=3e-4, weight_decay=1e-2, batch=128,
                     log=lambda m: log(m, q))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained in {t_train:.1f} s", q)
    fb = L.trace_rooms(scenes["cal"], rooms["cal"], n_rays=n_fb, seed_offset=L.SEED_SWEEP + n_fb, chunk=1024,
                       method=fbm, order=2 if fbm == "listener" else 0, **L.CONVERGED)
    prm, sig, _ = L.predict(model, cal["features"], cal["e_in"], 4, 1e9)
    kappa, fb_frac_cal, err_cal = L.choose_kappa(sig.max(dim=1).values.cpu().numpy(),
                                                 L.rt60_error(prm, refs["cal"], 4),
                                                 L.rt60_error(fb["params"], refs["cal"], 4),
                                                 target=a.learn_target_err)
    log(f"kappa {kappa:.4f}: calibration fallback {fb_frac_cal:.3f}, error {err_cal:.4f}", q)
    # held-out: ungated network error, then the gated path, timed
    cheap_data = L.trace_rooms(scenes["eval"], rooms["eval"], n_rays=1024, seed_offset=L.SEED_INPUT,
                               want_features=True, chunk=1024, **L.INPUT)
    prm, _, _ = L.predict(model, cheap_data["features"], cheap_data["e_in"], 4, 1e9)
    err_net = L.rt60_error_summary(L.rt60_error(prm, refs["eval"], 4))
    prm, unc, cheap = L.learned_estimate(model, scenes["eval"], rooms["eval"], kappa, n_fb, fallback=fbm)
    err_learned = L.rt60_error_summary(L.rt60_error(prm, refs["eval"], 4))
    fb_frac = float(unc.float().mean())
    log(f"held-out: network {err_net}, learned {err_learned}, fallback {fb_frac:.3f}", q)
    for _ in range(a.warmup):
        L.learned_estimate(model, scenes["eval"], rooms["eval"], kappa, n_fb, cheap=cheap, fallback=fbm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        L.learned_estimate(model, scenes["eval"], rooms["eval"], kappa, n_fb, cheap=cheap, fallback=fbm)
    torch.cuda.synchronize()
    t_learned = (time.perf_counter() - t0) / a.steps
    log(f"learned: {len(rooms['eval']) / t_learned:.1f} IRs/s", q)
    ips_plain, _ = L.timed_plain(scenes["eval"], rooms["eval"], n_star, steps=a.steps)
    log(f"plain source: {ips_plain:.1f} IRs/s", q)
    ips_plain_l, _ = L.timed_plain(scenes["eval"], rooms["eval"], n_star_l, steps=a.steps, method="listener",
                                   order=2)
    log(f"plain listener: {ips_plain_l:.1f} IRs/s", q)
    n_ev = len(rooms["eval"])
    out = {
        "metric": "IRs/s at <=5% RT60 error, learned vs plain ray trace", "value": n_ev / t_learned,
        "unit": "IRs/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": t_learned * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 trace, bf16 mlp",
        "data": "synthetic",
        "config": {"workload": f"learn: {n_ev} held-out shoebox/L-rooms (dims U[3,40] m); step = learned estimate "
                               f"of every room (1k-ray trace + MLP + {fbm}-origin fallback at its N*); "
                               f"{a.learn_train} training rooms x {a.learn_views} inputs (100k rooms named for this "
                               f"workload), {a.learn_target_rays}-ray targets, 262,144-ray references",
                   "train_rooms": a.learn_train, "eval_rooms": n_ev, "views": a.learn_views,
                   "target_rays": a.learn_target_rays, "arch": a.learn_arch, "dims": list(model.dims)},
        "plain": {"n_star": n_star, "irs_per_s": ips_plain, "sweep": {str(k): v for k, v in sweep.items()}},
        "plain_listener": {"n_star": n_star_l, "irs_per_s": ips_plain_l,
                           "sweep": {str(k): v for k, v in sweep_l.items()}},
        "learned": {"irs_per_s": n_ev / t_learned, "rt60_err": err_learned, "fallback_fraction": fb_frac,
                    "fallback_method": fbm, "fallback_rays": n_fb,
                    "kappa": kappa, "network_only_rt60_err": err_net, "cal_fallback_fraction": fb_frac_cal,
                    "cal_rt60_err": err_cal},
        "speedup_learned_vs_plain": (n_ev / t_learned) / ips_plain,
        "speedup_learned_vs_best_plain": (n_ev / t_learned) / max(ips_plain, ips_plain_l),
        "training": {"dataset_s": t_data, "dataset_segments": data["segments"], "train_s": t_train,
                     "epochs": a.learn_epochs, "final_loss": losses[-1]},
        "total_s": time.perf_counter() - t_all,
    }
    model.close()
    print(json.dumps(out), flush=True)


def run_rooms(a):
    """The plain method traced two ways over --learn-eval held-out rooms of the
    learn workload (shoeboxes and L-rooms, dims U[3,40] m): from the source
    to the listener sphere, and from the listener point with next-event
    queries toward the source ball (r = 0.5 m).  For each, the smallest ray
    count of a sweep whose mean RT60 error against independent 262,144-ray
    source-origin references is <= 5% (N*), then IRs/s at N* as one
    graph-captured batch (reset, trace, estimate) over all rooms.  The
    listener batch deals the rooms' rays round-robin in 1,024-ray chunks
    (every reflection deposits, and the interleave spreads the atomics over
    many histograms); the source batch keeps the rooms in order."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R
    from paper_1803_00430_amd import learn as L

    q = a.quiet
    rooms = [R.learn_room(200000 + i) for i in range(a.learn_eval)]
    scenes = L.make_scenes(rooms)
    fixed = a.rooms_rays > 0
    ref = None if fixed else L.trace_rooms(scenes, rooms, n_rays=262144, seed_offset=L.SEED_REFERENCE, chunk=1024,
                                           **L.CONVERGED)["params"]
    res = {}
    plans = (("source", 0, (16384, 32768, 65536, 131072)), ("listener", 2, (4096, 8192, 16384, 32768, 65536)))
    if fixed:
        plans = tuple((m, o, (a.rooms_rays,)) for m, o, _ in plans if m == a.method)
    for method, order, Ns in plans:
        sweep = {}
        for N in Ns:
            if fixed:
                break
            tr = L.trace_rooms(scenes, rooms, n_rays=N, seed_offset=L.SEED_SWEEP + N, chunk=1024, method=method,
                               order=order, **L.CONVERGED)
            sweep[N] = L.rt60_error_summary(L.rt60_error(tr["params"], ref, 4))
            log(f"{method} N={N}: {sweep[N]}", q)
        ok = [N for N in sweep if sweep[N]["mean"] <= 0.05]
        n_star = Ns[0] if fixed else (min(ok) if ok else max(sweep))
        b = P.Batch(scenes, [dict(p, pair_id=k) for k, p in
                             enumerate(L.room_pairs(rooms, n_star, L.SEED_SWEEP + n_star))],
                    n_bins=L.CONVERGED["n_bins"], sh_order=L.SH_ORDER, bin_width_s=L.CONVERGED["bin_width_s"],
                    autotune=False, use_graph=True, late=False, method=method, order=order)
        for _ in range(max(1, a.warmup)):
            b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            b.run()
        torch.cuda.synchronize()
        dt_step = (time.perf_counter() - t0) / a.steps
        st = P.stats_host(b.stats)
        err = None if fixed else L.rt60_error_summary(L.rt60_error(b.params, ref, 4))
        res[method] = {"n_star": n_star, "irs_per_s": len(rooms) / dt_step, "ms_per_replay": dt_step * 1e3,
                       "rt60_err_at_n_star": err, "segments_per_replay": int(st["n_segments"].sum()),
                       "next_event_queries_per_replay": int(st["n_next_event"].sum()),
                       "deposit_rows_per_replay": int(st["n_deposit_rows"].sum()),
                       "sweep": {str(k): v for k, v in sweep.items()}}
        b.close()
        log(f"{method}: N* {n_star}, {res[method]['irs_per_s']:.1f} IRs/s", q)
    if fixed:
        print(json.dumps({"workload": "rooms", "method": a.method, **res[a.method]}), flush=True)
        return
    lst = res["listener"]
    # the replay is reset + trace + estimate; the trace kernel is all but < 1 ms of it (rocprofv3)
    row_bytes = 2 * 4 * 4 * (L.SH_ORDER + 1) ** 2  # read and write of one bins x coefficients row
    achieved = lst["deposit_rows_per_replay"] * row_bytes / (lst["ms_per_replay"] * 1e-3) / 1e9
    out = {
        "metric": "IRs/s at <=5% RT60 error, plain ray trace from the listener (next-event estimation) "
                  "vs from the source", "value": lst["irs_per_s"], "unit": "IRs/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": lst["ms_per_replay"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"rooms: {len(rooms)} held-out shoebox/L-rooms (dims U[3,40] m, one source, "
                               f"r = 0.5 m); step = one graph replay over all rooms at the method's N*; "
                               f"262,144-ray references", "rooms": len(rooms)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_trace_lstp",
                     "bytes_counted": "histogram atomics only (read + write of each deposited row); node and "
                                      "triangle fetches of the two traversals per reflection are not counted"},
        "listener": lst, "source": res["source"],
        "speedup_listener_vs_source": lst["irs_per_s"] / res["source"]["irs_per_s"],
    }
    print(json.dumps(out), flush=True)


def run_reverb(a):
    """Audio-rate rendering of the SH reverberator (Section 4.1; 8 combs and 4
    all-passes, Section 5): every step renders the next block of band audio
    for all sources, their delay lines carried from step to step; the
    parameters (reverb_setup) are built once before, as at a propagation
    update, and timed on their own."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R
    dev = torch.device("cuda:0")
    S, n, order, B, fs = a.reverb_sources, a.reverb_block, a.reverb_order, 4, 44100.0
    nc = (order + 1) ** 2
    desc = P.reverb_desc(B, order, fs, 343.0, 0.3)
    log(f"reverb: {S} sources x {n} samples, {B} bands, SH order {order}, {fs:.0f} Hz", a.quiet)
    inp = R.reverb_inputs(5, S, B, order, n_bins=40)
    prm = np.zeros(S, P.REVERB_PARAMS_DTYPE)
    for k in ("rt60", "g_reverb", "dir_loudness", "mean_free_path_m", "predelay_s", "first_arrival_s"):
        prm[k] = inp[k]
    params = torch.from_numpy(prm.view(np.uint8).reshape(S, -1).copy()).to(dev)
    hist = torch.from_numpy(inp["hist"]).to(dev)
    z = torch.from_numpy(inp["z"]).to(dev)
    ang = torch.from_numpy(inp["angles"]).to(dev)
    setup = P.alloc_reverb_setup(S, dev)
    state = P.reverb_state(S, desc, dev)
    x = torch.from_numpy(R.band_audio(6, S, B, n)).to(dev)
    out = torch.empty((S, nc, n), dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.reverb_setup(params, hist, inp["bin_width_s"], z, ang, desc, setup=setup, first=True)
    e1.record()
    torch.cuda.synchronize()
    setup_ms = e0.elapsed_time(e1)
    sh = P.reverb_setup_host(setup)
    for _ in range(a.warmup):
        P.reverb_render(setup, x, state, desc, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ev[i][0].record()
        P.reverb_render(setup, x, state, desc, out=out)
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    ms_step = wall * 1e3 / a.steps
    value = S * n * a.steps / wall
    ap_m = [int(np.floor(t * fs + 0.5)) for t in (4.9e-3, 4.1e-3, 3.4e-3, 2.9e-3)]
    # algorithmic HBM bytes per launch: each comb line read and written once per sample, the band
    # input read and the channels written once, the all-pass lines (short, cache-resident within a
    # launch) read and written once, the setup rows read once
    per_src = (n * B * 8 * nc * 8 + n * B * 4 + n * nc * 4 + 2 * B * nc * 4 * sum(ap_m)
               + 4 * (8 * nc * nc + B * nc * nc + 8 * nc + 8 * B + B + 8) + 64)
    bytes_launch = S * per_src
    achieved = bytes_launch / (k_ms * 1e-3) / 1e9
    default = (S, n, order) == (4096, 1024, 1)
    traffic = (REVERB_TRAFFIC["bytes"] if default and REVERB_TRAFFIC["sources_sha256"] ==
               trace_sources_sha256(REVERB_SOURCES) else None)
    res = {
        "metric": "reverb source-samples/s", "value": value, "unit": "source-samples/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"reverb: {S} sources x {n}-sample blocks at {fs:.0f} Hz, {B} bands, SH order "
                               f"{order} ({nc} channels), 8 combs with SH rotations + 4 all-passes + loudness "
                               f"matrix; parameters from seeded estimates (RT60 U(0.2,3) s, mean free path "
                               f"U(2,40) m); step = one block for every source",
                   "sources": S, "block": n, "bands": B, "sh_order": order, "sample_rate": fs},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_reverb_render",
                     "bytes_per_source_sample": per_src / n, "kernel_ms": k_ms},
        "realtime_sources": value / fs,
        "setup_ms": setup_ms,
        "mean_comb_delay_ms": float(sh["t_comb"][:S].mean() * 1e3),
    }
    if not a.no_cpu_baseline:
        import oracle  # noqa: F401  (the oracle's SH basis is loaded through it)
        from oracle import reverb as RV
        ns, nsamp = 4, 16384
        xs = R.band_audio(7, ns, B, nsamp).astype(np.float64)
        c0 = time.perf_counter()
        for s_ in range(ns):
            po = dict(rt60=inp["rt60"][s_, :B].astype(np.float64), g_reverb=inp["g_reverb"][s_, :B].astype(np.float64),
                      dir_loudness=inp["dir_loudness"][s_, :B, :nc].astype(np.float64),
                      predelay_s=float(inp["predelay_s"][s_]), first_arrival_s=float(inp["first_arrival_s"][s_]),
                      mean_free_path_m=float(inp["mean_free_path_m"][s_]))
            so = RV.setup(po, inp["hist"][s_].astype(np.float64), inp["bin_width_s"], inp["z"][s_].astype(np.float64),
                          inp["angles"][s_].astype(np.float64), order=order, n_bands=B, fs=fs, c=343.0, t_max=0.3)
            RV.render(xs[s_], so, order)
        c_wall = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": ns * nsamp / c_wall, "unit": "source-samples/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"sources 0..{ns - 1}, {nsamp} samples each ({c_wall:.1f} s), FP64 "
                                         f"per-sample loops, setup included"}
    if a.calib_copy_mib > 0:
        m = a.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(m, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = 4 * m
    print(json.dumps(res), flush=True)


def run_paths(a):
    """Early-reflection paths per frame (Section 5: the first two reflection
    orders with the diffuse path cache, the N_ER = 100 strongest paths over
    all sources rendered and the rest added to the late IR).  The city's 8
    sources, static, are traced every 0.1 s frame with fresh rays: each frame
    runs trace_ir_paths, the path cache update (tau_ER = 1 s), the
    prioritization and the late-IR estimate, against trace_ir + estimate
    alone.  The frame-to-frame change of every source's rendered early energy
    is measured with the cache and without it (alpha = 1)."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R
    dev = torch.device("cuda:0")
    cfg = R.city_config()
    S, K, T, n, dt = len(cfg["sources"]), cfg["max_bounces"], cfg["n_bins"], cfg["sh_order"], cfg["bin_width_s"]
    B = cfg["absorption"].shape[1]
    N = a.rays or cfg["n_rays"]
    n_er, thr, emin, max_rec = 100, 1e-12, 1e-14, 1 << 18
    alpha = P.temporal_alpha(0.1, 1.0)
    scene = P.Scene.from_dict(cfg, device=dev)
    hist, late, stats, _ = P.alloc_trace_outputs(S, T, B, n, device=dev)
    params = P.alloc_params(S, device=dev)
    rec = torch.zeros((max_rec, P.PATH_RECORD_WORDS), dtype=torch.float32, device=dev)
    n_rec = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.zeros((n_er, 128), dtype=torch.uint8, device=dev)
    n_out = torch.zeros(1, dtype=torch.int32, device=dev)
    out2 = torch.zeros((n_er, 128), dtype=torch.uint8, device=dev)
    n_out2 = torch.zeros(1, dtype=torch.int32, device=dev)
    cache, nocache = P.PathCache(65536), P.PathCache(65536)
    log(f"paths: city, {S} static sources x {N} rays, K={K}, N_ER={n_er}, alpha={alpha:.4f}", a.quiet)
    frames = a.frames if a.frames != 8 else 30
    ev_names = ("trace_paths", "cache_update", "select", "estimate")
    times = {k: [] for k in ev_names}
    plain_ms, walls, recs, cached, e_on, e_off = [], [], [], [], [], []
    for f in range(a.warmup + frames):
        prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt,
                             seed=cfg["seed"] + 1000 + f)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        P.trace_ir_paths(scene, cfg["sources"], cfg["listener"], cfg["radius"], prm, hist, late, stats, rec, n_rec)
        ev[1].record()
        cache.update(rec, n_rec, alpha, f == 0, emin)
        ev[2].record()
        cache.select(thr, n_er, out, n_out, hist_late=late, stats=stats, n_src=S, n_bins=T, n_bands=B,
                     bin_width_s=dt)
        ev[3].record()
        P.estimate_reverb(hist, late, stats, T, B, n, dt, params, rt60_source=1)
        ev[4].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        nocache.update(rec, n_rec, 1.0, True, emin)
        nocache.select(thr, n_er, out2, n_out2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.trace_ir(scene, cfg["sources"], cfg["listener"], cfg["radius"], prm, hist, late, stats)
        P.estimate_reverb(hist, late, stats, T, B, n, dt, params)
        torch.cuda.synchronize()
        pl = time.perf_counter() - t1
        if f < a.warmup:
            continue
        for i, k in enumerate(ev_names):
            times[k].append(ev[i].elapsed_time(ev[i + 1]))
        walls.append(wall * 1e3)
        plain_ms.append(pl * 1e3)
        recs.append(int(n_rec.item()))
        cached.append(cache.info()["n_paths"])
        for dst, o_, no_ in ((e_on, out, n_out), (e_off, out2, n_out2)):
            pth = P.early_paths_host(o_, int(no_.item()))
            e = np.zeros(S)
            for p_ in pth:
                e[p_["source"]] += float(p_["e"][:B].sum())
            dst.append(e)

    def jitter(es):
        es = np.array(es)
        m = es.mean(axis=0)
        ok = m > 0
        return float(np.mean(np.abs(np.diff(es[:, ok], axis=0)) / m[ok]))

    # traversal bytes per segment from one visit-counting trace of the same rays
    prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=cfg["seed"] + 1000,
                         flags=P.TRACE_COUNT_VISITS)
    P.trace_ir(scene, cfg["sources"], cfg["listener"], cfg["radius"], prm, hist, late, stats)
    torch.cuda.synchronize()
    st = P.stats_host(stats)
    segs = int(st["n_segments"].sum())
    bps = (128.0 * float(st["n_node_visits"].sum()) + 48.0 * float(st["n_tri_tests"].sum())) / segs
    tr_ms = float(np.mean(times["trace_paths"]))
    achieved = segs * bps / (tr_ms * 1e-3) / 1e9
    ms = float(np.mean(walls))
    res = {
        "metric": "early-path frames/s (trace with path records + path cache + prioritization + late-IR estimate)",
        "value": 1e3 / ms, "unit": "frames/s", "n_gpus": 1, "steps": frames, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"paths: city of {len(cfg['tris'])} triangles, {S} static sources x {N} rays, "
                               f"{K} bounces, SH order {n}, {T} x 1 ms bins, 0.1 s frames, tau_ER 1 s, N_ER {n_er} "
                               f"over all sources", "sources": S, "rays_per_source": N, "n_er": n_er,
                   "frames": frames},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_trace (path-record variant)",
                     "bytes_per_ray_bounce": bps, "kernel_ms": tr_ms},
        "breakdown_ms": {k: float(np.mean(v)) for k, v in times.items()},
        "plain_trace_estimate_ms": float(np.mean(plain_ms)),
        "records_per_frame": float(np.mean(recs)), "cached_paths": float(np.mean(cached)),
        "early_energy_jitter": {"with_cache": jitter(e_on), "without_cache": jitter(e_off)},
    }
    cache.close()
    nocache.close()
    scene.close()
    print(json.dumps(res), flush=True)


def run_city_frames(a):
    """City frames with moving sources: the 8 sources walk through the streets
    (3 m per 0.1 s frame, turning away from buildings), the listener stays.
    Each frame is traced and estimated three times over the same walk: with
    the workload's fixed 32,768 rays per source; under a segment budget per
    frame (Section 5) whose ray count follows the previous frame's segments
    per ray (`budget_ray_count`, "predicted"); and under the same budget
    applied within the frame by trace_ir (first pass of 16,384 rays per
    source, then the rays that fill each source's share, "in_frame").
    Reports the spread of the per-frame segment counts and frame times."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R

    q = a.quiet
    dev = torch.device("cuda:0")
    cfg = R.city_config()
    n_frames = a.frames if a.frames != 8 else 40
    walk = R.city_source_walk(cfg, n_frames + a.warmup)
    scene = P.Scene.from_dict(cfg, device=dev)
    S, K, T, n, dt = len(cfg["sources"]), cfg["max_bounces"], cfg["n_bins"], cfg["sh_order"], cfg["bin_width_s"]
    B = cfg["absorption"].shape[1]
    N0 = cfg["n_rays"]
    hist, late, stats, _ = P.alloc_trace_outputs(S, T, B, n, device=dev)
    params = P.alloc_params(S, device=dev)
    res = {}
    for mode in ("fixed", "predicted", "in_frame"):
        segs_l, rays_l, times = [], [], []
        prev_s = prev_r = 0
        for f in range(a.warmup + n_frames):
            if mode == "in_frame":
                prm = P.trace_params(n_rays_total=N0 // 2, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt,
                                     seed=cfg["seed"] + f, segment_budget=a.segment_budget // S, max_rays=4 * N0)
            else:
                # budget_ray_count sees the frame's totals over the sources; every source gets an equal share
                N = N0 if mode == "fixed" else P.budget_ray_count(a.segment_budget, prev_s, prev_r, S * 1024,
                                                                    S * 4 * N0, S * N0) // S
                prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt,
                                     seed=cfg["seed"] + f)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.trace_ir(scene, walk[f], cfg["listener"], cfg["radius"], prm, hist, late, stats)
            P.estimate_reverb(hist, late, stats, T, B, n, dt, params)
            torch.cuda.synchronize()
            t = time.perf_counter() - t1
            st = P.stats_host(stats)
            prev_s, prev_r = int(st["n_segments"].sum()), int(st["n_rays"].sum())
            if f >= a.warmup:
                segs_l.append(prev_s)
                rays_l.append(prev_r)
                times.append(t)
        segs_a, times_a = np.array(segs_l, np.float64), np.array(times) * 1e3
        res[mode] = {"segments_mean": float(segs_a.mean()), "segments_min": int(segs_a.min()),
                     "segments_max": int(segs_a.max()), "segments_cv": float(segs_a.std() / segs_a.mean()),
                     "rays_min": int(min(rays_l)), "rays_max": int(max(rays_l)),
                     "ms_mean": float(times_a.mean()), "ms_p99": float(np.percentile(times_a, 99)),
                     "ms_cv": float(times_a.std() / times_a.mean())}
        log(f"{mode}: {res[mode]}", q)
    bud = res["in_frame"]
    out = {
        "metric": "city frames with moving sources: per-frame segments under a segment budget",
        "value": 1e3 / bud["ms_mean"], "unit": "frames/s", "n_gpus": 1, "steps": n_frames, "warmup": a.warmup,
        "ms_per_step": bud["ms_mean"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"city frames: {len(cfg['tris'])} triangles, 8 sources walking 3 m per frame "
                               f"through the streets, {K} bounces, SH order {n}, {T} x 1 ms bins; fixed "
                               f"{N0} rays per source vs a budget of {a.segment_budget} segments per frame",
                   "segment_budget": a.segment_budget, "frames": n_frames},
        "fixed": res["fixed"], "predicted": res["predicted"], "in_frame": bud,
    }
    scene.close()
    print(json.dumps(out), flush=True)


def run_hospital_reference(a):
    """The hospital's accuracy question: is there a reference to judge the
    plain methods against?  The listener-origin trace (next-event queries
    toward every source ball, Section 5) is run twice at --ref-rays with
    independent seeds; its seed-to-seed RT60 disagreement says whether it has
    converged.  The source-origin trace at the workload's 131,072 rays per
    source and the listener-origin trace at 65,536 rays are then scored
    against the first reference: mean over sources x bands of
    |RT60 - RT60_ref| / RT60_ref where the reference fit is valid, an invalid
    estimate counting as error 1 (as in the learn workload)."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R

    q = a.quiet
    dev = torch.device("cuda:0")
    cfg = R.hospital_config()
    scene = P.Scene.from_dict(cfg, device=dev)
    S, K, T, n, dt = len(cfg["sources"]), cfg["max_bounces"], cfg["n_bins"], cfg["sh_order"], cfg["bin_width_s"]
    B = cfg["absorption"].shape[1]
    hist, late, stats, _ = P.alloc_trace_outputs(S, T, B, n, device=dev)
    params = P.alloc_params(S, device=dev)

    def run(method, rays, seed):
        prm = P.trace_params(n_rays_total=rays, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=seed)
        t1 = time.perf_counter()
        tr = P.trace_listener if method == "listener" else P.trace_ir
        tr(scene, cfg["sources"], cfg["listener"], cfg["radius"], prm, hist, late, stats)
        P.estimate_reverb(hist, late, stats, T, B, n, dt, params)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3
        ph = P.params_host(params)
        log(f"{method} {rays} rays seed {seed}: {ms:.0f} ms", q)
        return ph["rt60"][:, :B].astype(np.float64), ph["rt60_range"][:, :B], ms

    def err(rt, ref):
        ok = ref > 0
        e = np.where(rt > 0, np.abs(rt - ref) / np.where(ok, ref, 1.0), 1.0)[ok]
        return {"mean": float(e.mean()), "p90": float(np.quantile(e, 0.9)), "valid_estimates": int((rt > 0).sum()),
                "scored": int(ok.sum()), "of": int(ok.size)}

    run("listener", 4096, 1)  # warm-up
    ref_a, rng_a, ms_ref = run("listener", a.ref_rays, (1 << 36) + 1)
    ref_b, rng_b, _ = run("listener", a.ref_rays, (1 << 36) + 2)
    both = (ref_a > 0) & (ref_b > 0)
    dis = np.abs(ref_a - ref_b)[both] / (0.5 * (ref_a + ref_b)[both])
    same = both & (rng_a == rng_b)
    dis_same = np.abs(ref_a - ref_b)[same] / (0.5 * (ref_a + ref_b)[same])
    self_dis = {"mean": float(dis.mean()), "p90": float(np.quantile(dis, 0.9)), "valid_both": int(both.sum()),
                "of": int(both.size), "same_fit_range": int(same.sum()),
                "mean_where_same_range": float(dis_same.mean()) if same.any() else None,
                "ranges_a": {str(k): int((rng_a == k).sum()) for k in range(-1, 4)}}
    plain_src, _, ms_src = run("source", cfg["n_rays"], cfg["seed"])
    plain_lst, _, ms_lst = run("listener", 65536, cfg["seed"] + 5)
    res = {"reference_self_disagreement": self_dis,
           "source_131072": dict(err(plain_src, ref_a), ms_per_frame=ms_src),
           "listener_65536": dict(err(plain_lst, ref_a), ms_per_frame=ms_lst),
           "reference_ms": ms_ref}
    judged = self_dis["mean"] <= 0.05
    out = {"metric": "hospital RT60 error against a listener-origin reference", "value": res["source_131072"]["mean"],
           "unit": "relative RT60 error", "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"hospital: {len(cfg['tris'])} triangles, {S} sources at their frame-0 positions, "
                                  f"{K} bounces, SH order {n}, {T} x 1 ms bins, late-only RT60; reference = "
                                  f"listener-origin trace at {a.ref_rays} rays (two seeds)"},
           "reference_converged_within_5pct": judged, **res}
    scene.close()
    print(json.dumps(out), flush=True)


def run_hospital(a):
    """Large interactive scene: a hospital-like interior of ~1M triangles
    (rooms 4-12 m on a grid, corridors, doorways, clutter), 64 sources moving
    along the corridors at 1.4 m/s, one listener; per frame (0.1 s of motion)
    every source is traced with 131,072 rays, 200 bounces, SH order 3, 4
    bands, 3000 bins of 1 ms, and its reverb parameters are estimated.  The
    scene's BVH is built once (static geometry).  Reports per-frame p50/p99
    latency and IRs/s of the plain method."""
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R

    q = a.quiet
    dev = torch.device("cuda:0")
    cfg = R.hospital_config()
    t0 = time.perf_counter()
    scene = P.Scene.from_dict(cfg, device=dev)
    build_ms = (time.perf_counter() - t0) * 1e3
    S = len(cfg["sources"])
    N, K, T, n, dt = cfg["n_rays"], cfg["max_bounces"], cfg["n_bins"], cfg["sh_order"], cfg["bin_width_s"]
    if a.rays > 0:
        N = a.rays
    B = cfg["absorption"].shape[1]
    hist, late, stats, _ = P.alloc_trace_outputs(S, T, B, n, device=dev)
    params = P.alloc_params(S, device=dev)
    prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=cfg["seed"])
    listener = a.method == "listener"
    if listener and a.learned:
        raise SystemExit("--learned runs with the source method only")
    if a.temporal and (a.learned or a.convergence):
        raise SystemExit("--temporal runs without --learned and --convergence")
    x_max = float(cfg["verts"][:, 0].max()) - 2.5
    g = np.random.default_rng(7)
    heading = np.where(g.uniform(0, 1, S) < 0.5, -1.0, 1.0)

    def sources_at(f):
        src = cfg["sources"].astype(np.float64).copy()
        x = src[:, 0] - 0.5 + heading * 1.4 * 0.1 * f
        period = 2.0 * (x_max - 1.0)
        x = np.mod(x, period)
        src[:, 0] = 0.5 + np.where(x <= period / 2, x, period - x)
        return src.astype(np.float32)

    frame_dt = 0.1  # seconds of source motion per frame
    temporal = a.temporal
    if temporal:
        # IR caches (all orders with tau_ER = 1 s, late with tau_LR = 3 s) and Eq. 4
        a_er, a_lr = P.temporal_alpha(frame_dt, 1.0), P.temporal_alpha(frame_dt, 3.0)
        hist_c, late_c = torch.empty_like(hist), torch.empty_like(late)
        params_f = P.alloc_params(S, device=dev)
    n_done = [0]

    def frame(f, p=prm):
        if listener:
            P.trace_listener(scene, sources_at(f), cfg["listener"], cfg["radius"], p, hist, late, stats)
        else:
            P.trace_ir(scene, sources_at(f), cfg["listener"], cfg["radius"], p, hist, late, stats)
        if temporal:
            first = n_done[0] == 0
            P.ir_cache_update(hist_c, hist, a_er, first)
            P.ir_cache_update(late_c, late, a_lr, first)
            P.estimate_reverb(hist_c, late_c, stats, T, B, n, dt, params_f)
            P.reverb_params_smooth(params, params_f, B, a_er, a_lr, first)
        else:
            P.estimate_reverb(hist, late, stats, T, B, n, dt, params)
        n_done[0] += 1

    for f in range(a.warmup):
        frame(-1 - f)
    torch.cuda.synchronize()
    times, segs, rt_frames = [], 0, []
    for f in range(a.frames):
        t1 = time.perf_counter()
        frame(f)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        rt_frames.append(params.clone())
        st_ = P.stats_host(stats)["n_segments"]
        segs += int(st_[0] if listener else st_.sum())  # the listener's ray set is repeated per source
        log(f"frame {f}: {times[-1] * 1e3:.1f} ms", q)
    times = np.array(times)
    ms = times.mean() * 1e3
    queries = int(P.stats_host(stats)["n_next_event"][0]) if listener else 0
    rts = [P.params_host(x)["rt60"][:, :B].astype(np.float64) for x in rt_frames]
    jit = []
    for r0, r1 in zip(rts[:-1], rts[1:]):
        ok = (r0 > 0) & (r1 > 0)
        jit.append(np.abs(r1 - r0)[ok] / (0.5 * (r0 + r1)[ok]))
    jit = np.concatenate(jit) if jit else np.zeros(0)
    jitter = {"mean": float(jit.mean()), "p90": float(np.quantile(jit, 0.9))} if jit.size else None
    conv = None
    if a.convergence:
        rt, el = [], []
        for extra in (1 << 40, 2 << 40):
            prm2 = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt,
                                  seed=cfg["seed"] + extra)
            frame(0, prm2)
            torch.cuda.synchronize()
            ph = P.params_host(params)
            rt.append(ph["rt60"][:, :B].astype(np.float64))
            el.append(ph["e_late"][:, :B].astype(np.float64))
        ok = (rt[0] > 0) & (rt[1] > 0)
        dis = np.abs(rt[0] - rt[1])[ok] / (0.5 * (rt[0] + rt[1])[ok])
        ok_e = (el[0] + el[1]) > 0
        dis_e = np.abs(el[0] - el[1])[ok_e] / (0.5 * (el[0] + el[1])[ok_e])
        conv = {"mean": float(dis.mean()), "p90": float(np.quantile(dis, 0.9)), "valid": int(ok.sum()),
                "of": int(ok.size), "e_late_mean": float(dis_e.mean()),
                "e_late_p90": float(np.quantile(dis_e, 0.9))}
        log(f"RT60 disagreement between two seeds: mean {conv['mean']:.4f}, p90 {conv['p90']:.4f}; "
            f"late energy: mean {conv['e_late_mean']:.4f}, p90 {conv['e_late_p90']:.4f}", q)
    learned = run_hospital_learned(a, P, scene, cfg, sources_at, params, frame) if a.learned else None
    how = (f"traced from the listener point with {N} rays and next-event queries toward every source ball "
           f"(r = {cfg['radius']} m)" if listener else f"{N} rays per source to the listener sphere")
    if temporal:
        how += ", smoothed across frames (IR caches tau 1 s / 3 s, Eq. 4 RT60 smoothing, 0.1 s frames)"
    out = {
        "metric": "per-frame latency p50/p99 and IRs/s (plain ray trace)", "value": S / times.mean(),
        "unit": "IRs/s", "n_gpus": 1, "steps": a.frames, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"hospital: {len(cfg['tris'])} triangles, {S} moving sources, {how}, "
                               f"{K} bounces, SH order {n}, {B} bands, {T} x 1 ms bins; step = one frame "
                               f"(trace + estimate of every source; BVH built once)", "method": a.method},
        "p50_ms": float(np.percentile(times, 50) * 1e3), "p99_ms": float(np.percentile(times, 99) * 1e3),
        "build_ms": build_ms, "ray_bounces_per_s": segs / times.sum(),
    }
    out["rt60_frame_jitter"] = jitter
    out["config"]["temporal"] = bool(temporal)
    if listener:
        out["next_event_queries_per_frame"] = queries
    if conv:
        out["rt60_seed_disagreement"] = conv
    if learned:
        out["learned"] = learned
    scene.close()
    print(json.dumps(out), flush=True)


def run_hospital_learned(a, P, scene, cfg, sources_at, params_plain, plain_frame):
    """The learned estimator inline in the hospital frames: per frame, every
    source is traced with 1,024 rays (200 bins of 10 ms), its features go
    through the network, and sources whose uncertainty exceeds kappa are
    traced again with the full 131,072 rays and estimated by the plain method.
    The network is trained first on shoebox / L-room data (as the learn
    workload, with --learn-train rooms), kappa tuned on calibration rooms.
    Accuracy: RT60 against the plain frame (131,072 rays) of the same source
    positions."""
    import torch

    import rpr_scenes as R
    from paper_1803_00430_amd import learn as L

    q = a.quiet
    t0 = time.perf_counter()
    # the hospital is out of the training rooms' distribution and falls back on every source (§6),
    # so its inline model trains on at most 32,768 rooms
    tr = [R.learn_room(10000 + i) for i in range(min(a.learn_train, 32768))]
    ca = [R.learn_room(150000 + i) for i in range(512)]
    tr_sc, ca_sc = L.make_scenes(tr), L.make_scenes(ca)
    data = L.make_dataset(tr_sc, tr, n_target=a.learn_target_rays, inputs_per_room=a.learn_views, chunk=1024)
    cal = L.make_dataset(ca_sc, ca, n_target=a.learn_target_rays, chunk=1024)
    ref = L.trace_rooms(ca_sc, ca, n_rays=262144, seed_offset=L.SEED_REFERENCE, chunk=1024, **L.CONVERGED)
    fb = L.trace_rooms(ca_sc, ca, n_rays=cfg["n_rays"], seed_offset=L.SEED_SWEEP + cfg["n_rays"], chunk=1024,
                       **L.CONVERGED)
    model = learned_model(a, P)
    L.train(model, data, epochs=a.learn_epochs, lr=3e-4, weight_decay=1e-2, batch=128)
    prm, sig, _ = L.predict(model, cal["features"], cal["e_in"], 4, 1e9)
    kappa, _, _ = L.choose_kappa(sig.max(dim=1).values.cpu().numpy(), L.rt60_error(prm, ref["params"], 4),
                                 L.rt60_error(fb["params"], ref["params"], 4), target=a.learn_target_err)
    t_prep = time.perf_counter() - t0
    log(f"learned model ready in {t_prep:.0f} s, kappa {kappa:.3f}", q)
    S, B, n = len(cfg["sources"]), cfg["absorption"].shape[1], cfg["sh_order"]
    nc = (n + 1) ** 2
    T_in, dt_in = L.INPUT["n_bins"], L.INPUT["bin_width_s"]
    hc, lc, sc_, _ = P.alloc_trace_outputs(S, T_in, B, n, late=False)
    # the network's input convention: 1,024 rays traced to the end of a 2 s window (bounce limit 1000)
    prm_cheap = P.trace_params(n_rays_total=1024, max_bounces=L.MAX_BOUNCES, sh_order=n, n_bins=T_in,
                               bin_width_s=dt_in, seed=cfg["seed"] + (1 << 32))
    prm_full = P.trace_params(n_rays_total=cfg["n_rays"], max_bounces=cfg["max_bounces"], sh_order=n,
                              n_bins=cfg["n_bins"], bin_width_s=cfg["bin_width_s"], seed=cfg["seed"] + (1 << 33))

    def learned_frame(f):
        src = sources_at(f)
        P.trace_ir(scene, src, cfg["listener"], cfg["radius"], prm_cheap, hc, None, sc_)
        feats, e = P.featurize(hc, T_in, B, nc, stats=sc_)
        out_p, _, unc = L.predict(model, feats, e, B, kappa, in_place=True)
        idx = torch.nonzero(unc).flatten().to(torch.int32)
        k = int(idx.numel())
        if k:
            hf, lf, sf, _ = P.alloc_trace_outputs(k, cfg["n_bins"], B, n)
            P.trace_ir(scene, src[idx.cpu().numpy()], cfg["listener"], cfg["radius"], prm_full, hf, lf, sf)
            pf = P.alloc_params(k)
            P.estimate_reverb(hf, lf, sf, cfg["n_bins"], B, n, cfg["bin_width_s"], pf)
            P.params_scatter(pf, idx, out_p)
        return out_p, k

    learned_frame(-1)
    torch.cuda.synchronize()
    times, errs, fbs = [], [], []
    for f in range(a.frames):
        t1 = time.perf_counter()
        out_p, k = learned_frame(f)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        fbs.append(k / S)
        plain_frame(f)  # reference: the plain method at the same source positions
        torch.cuda.synchronize()
        errs.append(L.rt60_error(out_p, params_plain, B))
        log(f"learned frame {f}: {times[-1] * 1e3:.1f} ms, fallback {k}/{S}", q)
    times = np.array(times)
    err = L.rt60_error_summary(np.concatenate(errs))
    model.close()
    return {"irs_per_s": S / times.mean(), "p50_ms": float(np.percentile(times, 50) * 1e3),
            "p99_ms": float(np.percentile(times, 99) * 1e3), "fallback_fraction": float(np.mean(fbs)),
            "rt60_err_vs_plain_frame": err, "kappa": kappa, "prep_s": t_prep}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import paper_1803_00430_amd as P
    import rpr_scenes as R

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # Python's cyclic garbage collector is kept out of the timed regions (as timeit does): a
    # collection walks every live object (torch's included) and, when one lands in a step, adds
    # about 2 ms of host time that belongs to no GPU work.  The objects alive now are frozen out
    # of later collections and the collector stays off for this short-lived process; the steps
    # create no reference cycles, so reference counting frees everything they allocate.
    gc.collect()
    gc.freeze()
    gc.disable()
    if a.workload == "batch":
        run_batch(a)
        return
    if a.workload == "learn":
        run_learn(a)
        return
    if a.workload == "hospital":
        if a.reference:
            run_hospital_reference(a)
        else:
            run_hospital(a)
        return
    if a.workload == "rooms":
        run_rooms(a)
        return
    if a.workload == "reverb":
        run_reverb(a)
        return
    if a.workload == "paths":
        run_paths(a)
        return
    if a.workload == "probe":
        run_probe(a)
        return
    if a.segment_budget > 0:
        run_city_frames(a)
        return
    cfg = R.city_config()
    S = len(cfg["sources"])
    N, K, T, n, dt = cfg["n_rays"], cfg["max_bounces"], cfg["n_bins"], cfg["sh_order"], cfg["bin_width_s"]
    B = cfg["absorption"].shape[1]
    log(f"city: {len(cfg['tris'])} triangles, {S} sources x {N} rays, K={K}, T={T}, n={n}", a.quiet)

    # inputs resident in HBM before anything is timed
    verts = torch.as_tensor(cfg["verts"], device=dev)
    tris = torch.as_tensor(cfg["tris"], device=dev)
    tmat = torch.as_tensor(cfg["tri_mat"], device=dev)
    absb = torch.as_tensor(cfg["absorption"], device=dev)
    scat = torch.as_tensor(cfg["scattering"], device=dev)
    hist, late, stats, _ = P.alloc_trace_outputs(S, T, B, n, device=dev)
    params = P.alloc_params(S, device=dev)
    prm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=cfg["seed"],
                         waves_per_cu=a.waves_per_cu)
    stream = torch.cuda.current_stream()

    # one counting pass (untimed): nodes and triangles fetched per ray-bounce
    scene = P.Scene(verts, tris, tmat, absb, scat, device=dev)
    info = scene.info()
    cprm = P.trace_params(n_rays_total=N, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=cfg["seed"],
                          flags=P.TRACE_COUNT_VISITS)
    P.trace_ir(scene, cfg["sources"], cfg["listener"], cfg["radius"], cprm, hist, late, stats)
    torch.cuda.synchronize()
    st = P.stats_host(stats)
    segs = int(st["n_segments"].sum())
    vn = float(st["n_node_visits"].sum()) / segs
    vt = float(st["n_tri_tests"].sum()) / segs
    bytes_per_seg = 128.0 * vn + 48.0 * vt  # 4-wide node = 128 B, triangle record = 48 B
    scene.close()
    log(f"BVH depth {info['max_depth']}, stack {info['stack_need']}; {segs} segments/step; "
        f"{vn:.1f} nodes + {vt:.1f} triangles per segment",
        a.quiet)

    # Steps are independent (same scene, same rays), so consecutive steps are
    # pipelined on several streams (--streams) with their own outputs and their
    # own scene, which each step rebuilds in place from the triangles
    # (scene_rebuild: the whole BVH build, into the scene's own arrays,
    # enqueued on the step's stream without waiting; the step's trace waits for
    # it).  Step i+1's rebuild is enqueued before step i's trace, so builds and
    # traces of neighbouring steps run side by side and the host never waits
    # for a build it has just enqueued.  Every step does all of its own work;
    # --serial runs them one after another on one stream.
    n_pipe = 1 if a.serial else max(1, a.streams)
    streams = [stream] if a.serial else [torch.cuda.Stream(device=dev) for _ in range(n_pipe)]
    outs = [(hist, late, stats, params)] + [(*P.alloc_trace_outputs(S, T, B, n, device=dev)[:3],
                                             P.alloc_params(S, device=dev)) for _ in range(n_pipe - 1)]
    pipe_scenes = [P.Scene(verts, tris, tmat, absb, scat, device=dev) for _ in range(n_pipe)]
    rec = []  # per timed step: (build ms, trace events, estimate events)

    def build(i):
        st_ = streams[i % n_pipe]
        with torch.cuda.stream(st_):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[3].record(st_)
            pipe_scenes[i % n_pipe].rebuild(verts, tris, tmat, absb, scat)
            ev[0].record(st_)
        return ev

    def trace_estimate(i, ev):
        st_, (h_, l_, s_, p_) = streams[i % n_pipe], outs[i % n_pipe]
        with torch.cuda.stream(st_):
            P.trace_ir(pipe_scenes[i % n_pipe], cfg["sources"], cfg["listener"], cfg["radius"], prm, h_, l_, s_)
            ev[1].record(st_)
            P.estimate_reverb(h_, l_, s_, T, B, n, dt, p_)
            ev[2].record(st_)

    def run_steps(k, record):
        if k == 0:
            return
        ahead = n_pipe > 1  # one scene per stream: step i+1's rebuild does not touch step i's scene
        ev = build(0)
        for i in range(k):
            nxt = build(i + 1) if ahead and i + 1 < k else None
            trace_estimate(i, ev)
            if record:
                rec.append(ev)
            ev = nxt if ahead else (build(i + 1) if i + 1 < k else None)

    run_steps(a.warmup, False)
    # timed region: exactly `steps` steps (each: rebuild, trace, estimate), synchronised on both sides
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(a.steps, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s_ in pipe_scenes:
        s_.close()
    t_build = [ev[3].elapsed_time(ev[0]) for ev in rec]
    t_trace = [ev[0].elapsed_time(ev[1]) for ev in rec]
    t_est = [ev[1].elapsed_time(ev[2]) for ev in rec]

    st = P.stats_host(stats)
    segs = int(st["n_segments"].sum())
    ms_step = wall * 1e3 / a.steps
    value = segs * a.steps / wall
    trace_ms = float(np.mean(t_trace))
    traffic = TRACE_TRAFFIC["bytes"] if TRACE_TRAFFIC["sources_sha256"] == trace_sources_sha256() else None
    pg = P.params_host(params)

    # After the timed region: the trace alone, launch after launch on one stream
    # (the duration a profiler reports for k_trace under --serial), and the
    # memory probe at the traversal's working set (the roof it runs under).
    sc = P.Scene(verts, tris, tmat, absb, scat, device=dev)
    s_ms = []
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        P.trace_ir(sc, cfg["sources"], cfg["listener"], cfg["radius"], prm, hist, late, stats)
        e1.record()
        e1.synchronize()
        if i > 0:
            s_ms.append(e0.elapsed_time(e1))
    sc.close()
    serial_ms = float(np.median(s_ms))
    work_bytes = 128 * int(info["n_nodes"]) + 48 * int(info["n_tris"])
    roof = trace_roof(P, torch, work_bytes, P.device_cus())
    alg_bytes = segs * bytes_per_seg  # algorithmic bytes of one step's trace
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9  # over the step time the job sustains
    achieved_serial = alg_bytes / (serial_ms * 1e-3) / 1e9

    out = {
        "metric": "ray-bounces/s", "value": value, "unit": "ray-bounces/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "city: procedural city of 99,996 triangles (extruded boxes, tessellated), "
                               "8 sources x 32,768 rays, 100 bounces, 4 bands, SH order 3, 3000 x 1 ms bins; "
                               "step = BVH build + trace + estimate" +
                               ("" if n_pipe == 1 else f"; consecutive steps pipelined on {n_pipe} streams"),
                   "pipelined_streams": n_pipe,
                   "n_tris": int(info["n_tris"]), "sources": S, "rays_per_source": N, "max_bounces": K,
                   "sh_order": n, "bands": B, "bins": T, "bin_width_s": dt,
                   **({"waves_per_cu": a.waves_per_cu} if a.waves_per_cu else {})},
        # k_trace's algorithmic bytes (nodes and triangle records fetched) per step over the
        # pipelined step time, against the measured rate at which the chip serves scattered
        # 128-byte lines from a working set of the tree's size (L2 + Infinity Cache: the tree is
        # far below HBM, whose traffic `traffic` is ~1% of these bytes); `serial` is the trace
        # launched alone, one launch after another
        "roofline": {"bound": "cache", "achieved": achieved, "peak": roof["gather_gbs"], "unit": "GB/s",
                     "frac": achieved / roof["gather_gbs"], "traffic": traffic,
                     "kernel": "k_trace", "kernel_ms": ms_step, "algorithmic_bytes": alg_bytes,
                     "bytes_per_ray_bounce": bytes_per_seg,
                     "node_visits_per_ray_bounce": vn, "tri_tests_per_ray_bounce": vt,
                     "peak_source": "memory_probe gather at the tree's working set", "probe": roof,
                     "hbm_peak": HBM_PEAK_GBS, "hbm_frac": achieved / HBM_PEAK_GBS,
                     "serial": {"kernel_ms": serial_ms, "achieved": achieved_serial,
                                "frac": achieved_serial / roof["gather_gbs"]},
                     "per_launch_overlapped_ms": trace_ms},
        # per timed step, by events on the step's stream (with several streams the phases overlap the
        # neighbouring steps, so they do not add up to ms_per_step)
        "breakdown_ms": {"build": float(np.mean(t_build)), "trace": trace_ms, "estimate": float(np.mean(t_est))},
        "trace_ray_bounces_per_s": segs / (trace_ms * 1e-3),
        # every source's IR is traced and estimated each step; `valid_irs_per_s` counts only the IRs
        # whose every band came back with a fit (see `estimates`)
        "irs_per_s": S / (ms_step * 1e-3),
        "valid_irs_per_s": int(sum(((pg["status"][i][:B] & 7) == 0).all() for i in range(S))) / (ms_step * 1e-3),
        "segments_per_step": segs,
        # the fit needs a decay range: in the open city most listener spheres catch only a few
        # bins of energy from 32,768 source rays, and those estimates come back invalid (RT60 0)
        "estimates": {
            "valid_sources": int(sum(((pg["status"][i][:B] & 7) == 0).all() for i in range(S))),
            "no_energy_sources": int(sum(((pg["status"][i][:B] & 1) != 0).any() for i in range(S))),
            "no_range_sources": int(sum(((pg["status"][i][:B] & 4) != 0).any() for i in range(S))),
            "rt60_s_valid": [[float(x) for x in pg["rt60"][i][:B]] for i in range(S)
                             if ((pg["status"][i][:B] & 7) == 0).all()],
        },
    }
    if not a.no_cpu_baseline:
        import oracle
        R_s = a.cpu_rays
        runs = []
        for _ in range(3):
            c0 = time.perf_counter()
            o = oracle.trace_ir(cfg, cfg["sources"], cfg["listener"], cfg["radius"], n_rays_total=N, ray_begin=0,
                                ray_end=R_s, max_bounces=K, sh_order=n, n_bins=T, bin_width_s=dt, seed=cfg["seed"])
            runs.append(time.perf_counter() - c0)
        c_wall = float(np.median(runs))
        osegs = sum(x["n_segments"] for x in o["stats"])
        out["cpu_baseline"] = {"value": osegs / c_wall, "unit": "ray-bounces/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "cpu": cpu_model(),
                               "sample": f"city, rays 0..{R_s - 1} of each of the 8 sources ({osegs} ray-bounces), "
                                         f"FP64 brute force; median of 3 runs "
                                         f"({', '.join(f'{r:.1f}' for r in runs)} s)"}
    if a.calib_copy_mib > 0:
        n = a.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)  # an elementwise kernel: reads and writes `n` floats
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 4 * n
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
