#!/usr/bin/env python3
"""Benchmark of libpgm: image pairs/s of pyramidal gradient matching at 1024x436.

One step = one whole pass of the method (pyramids, gradient images, random numbers,
coarse-to-fine PatchMatch with the forward-backward check at every level, level-0 output and
compaction) over one synthetic 1024x436 RGB pair already resident in HBM, issued as plain
per-pair launches on one stream (`value`). Further passes run the same method on B identical-size
pairs per step through pgm_match_batch (`batched_uniform`), on 64 pairs of four sizes grouped
into one pgm_match_groups graph launch (`batched`), and through the request server with
Poisson arrivals (`served`, p50/p99 latency); for context, the paper's own parameters (dense
field, patches 15/11) on the same pairs (`paper_preset`). Prints one JSON line.

Measurement: the timed region is bracketed by torch.cuda.synchronize(). The dominant kernel
(the propagation + random-search half-sweep) is then timed live with HIP events around each
run of its launches over a second pass of the same steps, which gives its average launch time
and its distance evaluations; its roofline is VALU-bound at one v_sad_u16 per lane per clock.
The CPU baseline is the oracle (single thread, synchronous schedule) on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "image pairs/s at 1024x436 plain vs batched; p50/p99 served latency"
# MI355X: 256 CUs x 4 SIMD16 x 2.4 GHz = 39.3 T lane operations per second. One v_sad_u16 per
# lane-clock adds two absolute differences of packed 16-bit gradients, so an 8x8 patch of 6
# channels (384 absolute differences) is 192 such operations.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
OPS_PER_EVAL = 8 * 8 * 6 // 2


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--pairs", type=int, default=2, help="distinct resident pairs cycled over the steps")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--batch", type=int, default=32, help="pairs per step of the batched pass (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--groups-pairs", type=int, default=64, help="pairs of the uneven-size batch (0 = skip)")
    ap.add_argument("--groups-steps", type=int, default=10)
    ap.add_argument("--served", type=int, default=240, help="requests per served run (0 = skip)")
    ap.add_argument("--served-pool", type=int, default=24, help="distinct generated request pairs")
    ap.add_argument("--paper-steps", type=int, default=20, help="steps of the paper-preset pass (0 = skip)")
    ap.add_argument("--config-steps", type=int, default=100,
                    help="steps of the 256x192 and 1242x375 plain passes (0 = skip)")
    ap.add_argument("--served-pool-mib", type=int, default=2048, help="HBM budget of the request server's pool")
    ap.add_argument("--cpu-all-seconds", type=float, default=8.0,
                    help="wall time of the all-core oracle throughput run (0 = skip)")
    ap.add_argument("--cpu-scan-seconds", type=float, default=6.0,
                    help="CPU time of the oracle's sequential-scan timing (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a known-size kernel for HBM counter scaling)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: turn the counter_collection.csv files of a FETCH_SIZE and a WRITE_SIZE "
                         "rocprofv3 run of the plain pass (with --copy-calibration) into TRAFFIC_FILE")
    ap.add_argument("--copy-mib", type=int, default=256, help="size of the calibration copy in those runs")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_hbm_traffic_1024x436.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1704_03217_amd", "csrc", "pgm_kernels.hip")


def _source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def summarize_counters(fetch_csv, write_csv, copy_mib):
    """HBM bytes per k_sweep launch of the plain pass from two rocprofv3 --pmc runs, each
    counter scaled by what it reads for the calibration copy of copy_mib MiB."""
    import csv

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"].startswith(counter)]
        return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows]

    out = {}
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = load(path, counter)
        copies = [v for k, g, v in rows if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"no calibration copy in {path}")
        scale = (copy_mib << 20) / (max(copies) * 1024.0)     # bytes per counted KiB
        # the half-sweep variant of the configuration-2 parameters (8x8 patches, integer SAD)
        sweeps = [v for k, g, v in rows if "k_sweep<6, 8, true, 0" in k]
        if not sweeps:
            raise SystemExit(f"no k_sweep<6, 8, true, 0> dispatches in {path}")
        out[name] = dict(kib_per_launch=sum(sweeps) / len(sweeps), scale=scale, launches=len(sweeps),
                         bytes_per_launch=scale * 1024.0 * sum(sweeps) / len(sweeps))
    res = {"kernel": "k_sweep", "workload": "plain pass, one 1024x436 pair per step (bench.py --batch 0)",
           "fetch_bytes_per_launch": round(out["fetch"]["bytes_per_launch"]),
           "write_bytes_per_launch": round(out["write"]["bytes_per_launch"]),
           "fetch_scale": out["fetch"]["scale"], "write_scale": out["write"]["scale"],
           "launches": out["fetch"]["launches"], "kernel_source_sha256": _source_hash()}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def measured_traffic():
    """HBM bytes per k_sweep launch from the committed counter summary, or None when it is
    missing or was taken on another version of the kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_source_sha256") != _source_hash():
            return None
        return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def sweep_roofline(pgm, ctx, steps, run, torch, traffic=None, ops_per_eval=None, peak=None, unit="TOP/s",
                   op="v_sad_u16 (two 16-bit absolute differences), 192 per 8x8x6 patch distance", bound="alu"):
    """Run `steps` steps with per-launch HIP events on; return (roofline of the half-sweep kernel
    that does the most distance evaluations, per-kind breakdown). achieved = evaluations x
    ops_per_eval / launches / average launch duration."""
    ops_per_eval = OPS_PER_EVAL if ops_per_eval is None else ops_per_eval
    peak = VALU_PEAK_TOPS if peak is None else peak
    pgm.pgm_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        run(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    breakdown = {}
    for kind, name in enumerate(pgm.KIND_NAMES):
        n, ms, ev = pgm.pgm_profile_read(ctx, kind)
        if n:
            breakdown[name] = dict(launches_per_step=n / steps, ms_per_step=ms / steps,
                                   avg_launch_us=1000.0 * ms / n, evals=ev)
    pgm.pgm_profile(ctx, False)
    # the half-sweep kernel that does the most distance evaluations (deterministic, unlike the
    # times): k_sweep, k_sweep_multi (2-4 half-sweeps of a small level per launch) or
    # k_sweep_pair (two per launch)
    cand = [k for k in ("sweep", "sweep_multi", "sweep_pair") if k in breakdown]
    which = max(cand, key=lambda k: breakdown[k]["evals"]) if cand else None
    sw = breakdown.get(which) if which else None
    if which != "sweep":
        traffic = None   # the counted HBM bytes are those of k_sweep launches
    roof = None
    if sw:
        n_launch = sw["launches_per_step"] * steps
        ops_per_launch = sw["evals"] * float(ops_per_eval) / n_launch
        achieved = ops_per_launch / (sw["avg_launch_us"] * 1e-6) / 1e12
        roof = {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 2),
                "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
                # the HBM side of the same launches, from the counted bytes (when current)
                "hbm_GBps": (round(traffic / (sw["avg_launch_us"] * 1e-6) / 1e9, 1) if traffic else None),
                "hbm_frac": (round(traffic / (sw["avg_launch_us"] * 1e-6) / 8.0e12, 4) if traffic else None),
                "kernel": {"sweep": "k_sweep (propagation + random search half-sweep)",
                           "sweep_multi": "k_sweep_multi (2-4 propagation + random search half-sweeps of a small "
                                          "level per launch)",
                           "sweep_pair": "k_sweep_pair (two propagation + random search half-sweeps per launch)"}[which],
                "op": op,
                "avg_launch_us": round(sw["avg_launch_us"], 3),
                "ops_per_launch": round(ops_per_launch),
                "profiled_ms_per_step": round(1000.0 * (t1 - t0) / steps, 4)}
    kernels = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
               for k, v in breakdown.items()}
    return roof, kernels


def _gen(args):
    import synth
    config, index, size = args
    return synth.config_pair(config, index, size)


def generate(jobs):
    """Seeded synthetic pairs, generated in worker processes."""
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(8, max(1, len(jobs)))) as ex:
        return list(ex.map(_gen, jobs))


def sized_params(pgm, w, preset=None):
    """Matching parameters of the uneven batch (preset 4) or of served pairs (preset 5):
    configuration 2's matching with |d| <= ceil(w / 5), through max_disp = -5."""
    return pgm.pgm_default_params(pgm.PRESET_CONFIG4 if preset is None else preset)


def run_groups(pgm, torch, dev, args, stream, pre):
    """64 pairs of uneven sizes, grouped by size into one pgm_match_groups call per step
    (captured into one HIP graph and replayed)."""
    sizes, pairs = pre["groups"]
    by = {}
    for sz, pr in zip(sizes, pairs):
        by.setdefault(tuple(sz), []).append(pr)
    need = 0
    for (w, h), prs in by.items():
        q = pgm.pgm_query(sized_params(pgm, w), w, h)
        need += (q.workspace_shared_bytes + len(prs) * q.workspace_pair_bytes + 255) // 256 * 256
    m = pgm.Matcher(0, need + (1 << 20))
    items, keep = [], []
    for (w, h), prs in sorted(by.items()):
        p = sized_params(pgm, w)
        a = torch.from_numpy(np.stack([q.img1 for q in prs])).to(dev)
        b = torch.from_numpy(np.stack([q.img2 for q in prs])).to(dev)
        o = m.outputs_batch(p, w, h, len(prs), count_evals=False)
        items.append((p, a, b, o))
    nev = torch.zeros(1, dtype=torch.int64, device=dev)
    # the launch schedule, picked by the library's tuner on the largest group (untimed; the
    # schedules give identical results)
    big = max(items, key=lambda it: it[1].shape[0] * it[1].shape[1] * it[1].shape[2])
    sched = m.tune(big[0], big[1], big[2], big[3], repeats=2, stream=stream)
    # eager reference, then graph replays (the first one captures)
    m.match_groups_into(items, n_evals=nev, stream=stream)
    torch.cuda.synchronize()
    evals_per_step = int(nev.item())
    ref = [o["fwd"].clone() for *_, o in items]
    for k in range(2):
        m.match_groups_into(items, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    same = all(torch.equal(o["fwd"], r) for (*_, o), r in zip(items, ref))
    print(f"[bench] uneven batch: timing {args.groups_steps} graph launches", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.groups_steps):
        m.match_groups_into(items, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n = args.groups_pairs * args.groups_steps
    roof = None
    if not args.no_profile_pass:   # eager launches (profiling records events around them)
        roof, _ = sweep_roofline(pgm, m.ctx, args.groups_steps, lambda k: m.match_groups_into(items, stream=stream),
                                 torch)
    m.close()
    return {"value": round(n / (t1 - t0), 3), "unit": "pairs/s", "pairs_per_step": args.groups_pairs,
            "steps": args.groups_steps, "ms_per_step": round(1000.0 * (t1 - t0) / args.groups_steps, 4),
            "sizes": {f"{w}x{h}": len(v) for (w, h), v in sorted(by.items())},
            "dist_evals_per_s": round(evals_per_step * args.groups_steps / (t1 - t0), 1),
            "graph_equals_eager": same, "schedule_flags": sched, "roofline": roof,
            "workload": "64 pairs, sizes uniform over 320x240, 640x480, 1024x436, 1242x375 (rectangle-layer "
                        "generator, |d| <= w/5), preset 4 (config-2 matching with |d| <= ceil(w/5)); grouped by size, "
                        "groups concurrent on 4 streams, one HIP graph launch per step"}


def run_paper_preset(pgm, torch, m, imgs, stream, steps):
    """Context: the paper's own parameters (dense stride-1 field, patches 15/11, Table II colour
    spaces, small-region removal) on the same resident 1024x436 pairs, one pair per call."""
    p = pgm.pgm_default_params(pgm.PRESET_PAPER)
    w, h = 1024, 436
    outs = [m.outputs(p, w, h, bwd=True, compact=True, count_evals=False) for _ in imgs]
    counted = m.outputs(p, w, h, bwd=True, compact=True, count_evals=True)
    m.match_into(p, imgs[0][0], imgs[0][1], counted, stream=stream)
    torch.cuda.synchronize()
    evals = int(counted["n_evals"].item())
    for k in range(2):
        a, b = imgs[k % len(imgs)]
        m.match_into(p, a, b, outs[k % len(outs)], stream=stream)
    print(f"[bench] paper preset: timing {steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        a, b = imgs[k % len(imgs)]
        m.match_into(p, a, b, outs[k % len(outs)], stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return {"value": round(steps / (t1 - t0), 3), "unit": "pairs/s", "steps": steps,
            "ms_per_pair": round(1000.0 * (t1 - t0) / steps, 4), "dist_evals_per_pair": evals,
            "dist_evals_per_s": round(evals * steps / (t1 - t0), 1),
            "workload": "paper preset on 1024x436: dense stride-1 field, patches 15 (forward) / 11 "
                        "(backward), L=3, Table II colour spaces, small-region removal (9 px)"}


def run_served(pgm, torch, dev, args, pre):
    """Poisson request streams through the request server, whose queued requests of one shape
    share launch sequences (continuous batching), and through plain per-pair launches (each
    request alone, in arrival order, on one stream) for the same requests at the same arrival
    times: capacity (all requests at once), then arrivals at 50% and 80% of the batching
    server's capacity; latency from arrival to observed completion."""
    sizes, pool = pre["served"]
    imgs = [(torch.from_numpy(q.img1).to(dev), torch.from_numpy(q.img2).to(dev)) for q in pool]
    prm = [sized_params(pgm, w, pgm.PRESET_CONFIG5) for (w, h) in sizes]
    rng = np.random.default_rng(5001)
    order = rng.integers(0, len(pool), args.served)
    budget = args.served_pool_mib << 20

    def run(srv, arrivals):
        lat = np.zeros(len(arrivals))
        subm, done = 0, 0
        t0 = time.perf_counter()
        while done < len(arrivals):
            now = time.perf_counter() - t0
            while subm < len(arrivals) and arrivals[subm] <= now:
                k = int(order[subm])
                srv.submit(prm[k], imgs[k][0], imgs[k][1], tag=subm)
                subm += 1
            for tag, _ in srv.poll():
                lat[tag] = (time.perf_counter() - t0) - arrivals[tag]
                done += 1
        return lat, time.perf_counter() - t0

    servers = {"batched": pgm.Server(0, budget, 4), "plain": pgm.Server(0, budget, 1, max_batch=1)}
    res = {}
    for name, srv in servers.items():
        run(srv, np.zeros(min(16, args.served)))    # warm-up
        s0 = srv.stats()
        lat, span = run(srv, np.zeros(args.served))
        s1 = srv.stats()
        res[name] = {"capacity_pairs_per_s": round(args.served / span, 2),
                     "launch_sequences": s1[0] - s0[0], "requests": s1[1] - s0[1]}
    capacity = res["batched"]["capacity_pairs_per_s"]
    arrivals = {}
    for frac in (0.5, 0.8):
        qps = frac * capacity
        arr = np.cumsum(rng.exponential(1.0 / qps, args.served))
        arrivals[frac] = (qps, arr - arr[0])
    for name, srv in servers.items():
        for frac, (qps, arr) in arrivals.items():
            print(f"[bench] served ({name}) at {qps:.0f} pairs/s", file=sys.stderr, flush=True)
            s0 = srv.stats()
            lat, span = run(srv, arr)
            s1 = srv.stats()
            res[name][f"at_{int(frac * 100)}pct"] = {
                "qps": round(qps, 2), "p50_ms": round(1000 * float(np.percentile(lat, 50)), 3),
                "p99_ms": round(1000 * float(np.percentile(lat, 99)), 3),
                "pairs_per_s": round(args.served / span, 2),
                "mean_requests_per_launch_sequence": round((s1[1] - s0[1]) / max(1, s1[0] - s0[0]), 3)}
        srv.close()
    out = {"unit": "ms", "capacity_pairs_per_s": capacity, "requests": args.served, "pool_bytes": budget,
           "distinct_pairs": len(pool), "batched_server": res["batched"], "plain_per_pair": res["plain"],
           "workload": "Poisson arrivals; sizes log-uniform in area over [320x240, 2048x1024], aspect "
                       "U[1.3, 3.3] (rectangle-layer generator, |d| <= w/5); preset 5 (config-2 matching with "
                       "|d| <= ceil(w/5)); requests drawn from the distinct generated pairs; batched_server: "
                       "4 streams, requests of one shape share launch sequences (at most 16, at most 8 "
                       "sequences in flight); plain_per_pair: pgm_match per request in arrival order on one "
                       "stream; pool = the stated HBM budget"}
    for frac in (0.5, 0.8):
        out[f"at_{int(frac * 100)}pct"] = res["batched"][f"at_{int(frac * 100)}pct"]
    return out


def run_config_pass(pgm, torch, dev, config, preset, steps, ops_per_eval, peak, unit, op, bound):
    """Plain passes of another workload (one pair per call): pairs/s, evaluations/s and the
    half-sweep's roofline fraction."""
    import synth
    pairs = [synth.config_pair(config, i) for i in range(2)]
    params = pgm.pgm_default_params(preset)
    h, w = pairs[0].img1.shape[:2]
    imgs = [(torch.from_numpy(p.img1).to(dev), torch.from_numpy(p.img2).to(dev)) for p in pairs]
    m = pgm.Matcher(0, pgm.pgm_query(params, w, h).workspace_bytes + (1 << 20))
    outs = [m.outputs(params, w, h, count_evals=False) for _ in imgs]
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step(k):
        m.match_into(params, *imgs[k % 2], outs[k % 2], stream=stream)

    for k in range(10):
        step(k)
    torch.cuda.synchronize()
    print(f"[bench] config {config} ({w}x{h}): timing {steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    counted = [m.outputs(params, w, h, count_evals=True) for _ in imgs]
    for k in range(2):
        m.match_into(params, *imgs[k], counted[k], stream=stream)
    torch.cuda.synchronize()
    per_pair = [int(o["n_evals"].item()) for o in counted]
    evals = sum(per_pair[k % 2] for k in range(steps))
    roof, _ = sweep_roofline(pgm, m.ctx, steps, step, torch, None, ops_per_eval, peak, unit, op, bound)
    m.close()
    return {"value": round(steps / (t1 - t0), 3), "unit": "pairs/s", "steps": steps,
            "ms_per_step": round(1000.0 * (t1 - t0) / steps, 4), "dist_evals_per_pair": evals / steps,
            "dist_evals_per_s": round(evals / (t1 - t0), 1), "roofline": roof}


def _oracle_worker(args):
    """One process of the all-core oracle run: runs until `seconds` of wall time are spent."""
    params_d, pair_ids, seconds, schedule, config = args
    import oracle
    import synth
    pairs = [synth.config_pair(config, i) for i in pair_ids]
    t0 = time.perf_counter()
    runs = 0
    while time.perf_counter() - t0 < seconds:
        p = pairs[runs % len(pairs)]
        oracle.match(params_d, p.img1, p.img2, schedule=schedule, trace=False)
        runs += 1
    return runs, time.perf_counter() - t0


def cpu_all_cores(params_d, seconds, config=2):
    """Throughput of independent oracle processes, one per host core (different pairs)."""
    import multiprocessing as mp
    import oracle
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    n = max(1, min(n, 16))   # the host share of one GPU
    ctx = mp.get_context("spawn")
    with ctx.Pool(n) as pool:
        res = pool.map(_oracle_worker, [(params_d, [k % 2], seconds, oracle.SYNC, config) for k in range(n)])
    runs = sum(r for r, _ in res)
    wall = max(t for _, t in res)
    return {"value": round(runs / wall, 4), "unit": "pairs/s", "cores": n, "processes": n, "runs": runs,
            "sample": f"{n} independent single-threaded oracle processes (synchronous schedule), each "
                      f"looping over a 1024x436 config-2 pair for {seconds:.0f} s of wall time"}


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.copy_mib)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the pairs are independent and this build runs on a single "
              "MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1704_03217_amd as pgm
    import synth

    # every synthetic pair is generated (in worker processes) before the GPU is first touched
    print(f"[bench] generating {args.pairs} synthetic 1024x436 pairs", file=sys.stderr, flush=True)
    pre = {}
    jobs = [(2, i, None) for i in range(args.pairs)]
    if args.groups_pairs > 0:
        gsizes = [tuple(sz) for sz in synth.batch_sizes(4000, args.groups_pairs)]
        jobs += [(4, k, sz) for k, sz in enumerate(gsizes)]
        print(f"[bench] generating {len(gsizes)} uneven-size pairs", file=sys.stderr, flush=True)
    if args.served > 0:
        ssizes = [tuple(sz) for sz in synth.served_sizes(5000, args.served_pool)]
        jobs += [(5, k, sz) for k, sz in enumerate(ssizes)]
        print(f"[bench] generating {len(ssizes)} served-size pairs", file=sys.stderr, flush=True)
    made = generate(jobs)
    pairs = made[: args.pairs]
    rest = made[args.pairs:]
    if args.groups_pairs > 0:
        pre["groups"] = (gsizes, rest[: len(gsizes)])
        rest = rest[len(gsizes):]
    if args.served > 0:
        pre["served"] = (ssizes, rest)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    params = pgm.pgm_default_params(pgm.PRESET_CONFIG2)
    w, h = 1024, 436
    imgs = [(torch.from_numpy(p.img1).to(dev), torch.from_numpy(p.img2).to(dev)) for p in pairs]
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nbytes} bytes done", file=sys.stderr, flush=True)
        del src, dst
    m = pgm.Matcher(0, 256 << 20)
    # the timed passes write every output of the path; distance evaluations (a report, not
    # part of the method) are counted in separate passes over the same pairs
    outs = [m.outputs(params, w, h, bwd=True, compact=True, count_evals=False) for _ in imgs]
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step(k):
        a, b = imgs[k % len(imgs)]
        m.match_into(params, a, b, outs[k % len(outs)], stream=stream)

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    counted = [m.outputs(params, w, h, bwd=True, compact=True, count_evals=True) for _ in imgs]
    for k, (a, b) in enumerate(imgs):
        m.match_into(params, a, b, counted[k], stream=stream)
    torch.cuda.synchronize()
    per_pair = [int(o["n_evals"].item()) for o in counted]
    evals = sum(per_pair[k % len(imgs)] for k in range(args.steps))
    del counted
    value = args.steps / elapsed
    n_inl = int(outs[0]["n_inliers"].item())

    roofline, kernels = None, {}
    if not args.no_profile_pass:
        print(f"[bench] profiled pass of {args.steps} steps (HIP events around each run of launches of one kind)", file=sys.stderr,
              flush=True)
        roofline, kernels = sweep_roofline(pgm, m.ctx, args.steps, step, torch, measured_traffic())

    batched = None
    if args.batch > 0:
        B = args.batch
        print(f"[bench] batched pass: {B} pairs per step, {args.batch_steps} steps", file=sys.stderr, flush=True)
        s_q = pgm.pgm_query(params, w, h)
        mb = pgm.Matcher(0, s_q.workspace_shared_bytes + B * s_q.workspace_pair_bytes + (1 << 20))
        A = torch.stack([imgs[k % len(imgs)][0] for k in range(B)]).contiguous()
        Bm = torch.stack([imgs[k % len(imgs)][1] for k in range(B)]).contiguous()
        ob = mb.outputs_batch(params, w, h, B, count_evals=False)

        # the launch schedule for this workload, picked by the library's tuner (untimed)
        sched = mb.tune(params, A, Bm, ob, repeats=2, stream=stream)

        def bstep(k):
            mb.match_batch_into(params, A, Bm, ob, stream=stream)

        for k in range(max(2, args.warmup // 4)):
            bstep(k)
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        for k in range(args.batch_steps):
            bstep(k)
        torch.cuda.synchronize()
        b1 = time.perf_counter()
        obc = mb.outputs_batch(params, w, h, B, count_evals=True)
        mb.match_batch_into(params, A, Bm, obc, stream=stream)
        torch.cuda.synchronize()
        bev = int(obc["n_evals"].item()) * args.batch_steps
        del obc
        # every pair of the batch equals its plain result
        same = bool(torch.equal(ob["fwd"][: outs[0]["fwd"].numel()], outs[0]["fwd"]))
        broof, bkern = (None, {})
        if not args.no_profile_pass:
            broof, bkern = sweep_roofline(pgm, mb.ctx, args.batch_steps, bstep, torch)
        batched = {"value": round(B * args.batch_steps / (b1 - b0), 3), "unit": "pairs/s", "global_batch": B,
                   "steps": args.batch_steps, "ms_per_step": round(1000.0 * (b1 - b0) / args.batch_steps, 4),
                   "dist_evals_per_s": round(bev / (b1 - b0), 1), "pair0_equals_plain": same,
                   "schedule_flags": sched,
                   "roofline": broof, "kernels": bkern}
        mb.close()

    configs = {}
    if args.config_steps > 0:
        configs["config1_256x192"] = run_config_pass(pgm, torch, dev, 1, pgm.PRESET_CONFIG1, args.config_steps,
                                                     OPS_PER_EVAL, VALU_PEAK_TOPS, "TOP/s",
                                                     "v_sad_u16 (two 16-bit absolute differences), 192 per 8x8x6 "
                                                     "patch distance", "alu")
        configs["config1_256x192"]["workload"] = (
            "plain, one 256x192 pair per step: 4 textured rectangles with integer motion |d| <= 20; L=3, stride 3, "
            "8x8 patch, 4 iterations, int16 gradients with int32 SAD, fwd+bwd tau=1")
        # float direction features: each patch element is a subtraction and an addition in
        # double precision (exact, see the kernels), 2 x 384 fp64 operations per distance. The
        # fp64 vector peak of 78.6 TFLOP/s counts a fused multiply-add as two; additions retire
        # one per lane per clock, 39.3 T per second, which is the peak used here.
        configs["config3_1242x375"] = run_config_pass(pgm, torch, dev, 3, pgm.PRESET_CONFIG3, args.config_steps,
                                                      2 * 8 * 8 * 6, VALU_PEAK_TOPS, "TOP/s",
                                                      "fp64 subtract + add per element of the unit-vector features, "
                                                      "768 per 8x8x6 patch distance", "alu")
        configs["config3_1242x375"]["workload"] = (
            "plain, one 1242x375 pair per step: ground plane with perspective flow, far background, 3 boxes, "
            "|d| <= 250; direction-only float features (unit gradient vectors), L=5, stride 3, 8x8, 6 iterations")
    groups = run_groups(pgm, torch, dev, args, stream, pre) if args.groups_pairs > 0 else None
    served = run_served(pgm, torch, dev, args, pre) if args.served > 0 else None
    paper = run_paper_preset(pgm, torch, m, imgs, stream, args.paper_steps) if args.paper_steps > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        params_d = pgm.params_dict(params)
        runs, spent = 0, 0.0
        while spent < args.cpu_seconds and runs < 64:
            p = pairs[runs % len(pairs)]
            c0 = time.perf_counter()
            oracle.match(params_d, p.img1, p.img2, schedule=oracle.SYNC, trace=False)
            spent += time.perf_counter() - c0
            runs += 1
            print(f"[bench] oracle run {runs}: {spent:.1f} s", file=sys.stderr, flush=True)
        cpu = {"value": round(runs / spent, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"{runs} oracle runs (single-threaded C, synchronous schedule) over {len(pairs)} "
                         f"1024x436 config-2 pairs, {spent:.1f} s",
               "cpu": _cpu_name(), "host_cores": os.cpu_count()}
        if args.cpu_scan_seconds > 0:
            runs, spent = 0, 0.0
            while spent < args.cpu_scan_seconds and runs < 64:
                p = pairs[runs % len(pairs)]
                c0 = time.perf_counter()
                oracle.match(params_d, p.img1, p.img2, schedule=oracle.SCAN, trace=False)
                spent += time.perf_counter() - c0
                runs += 1
            cpu["scan_schedule"] = {"value": round(runs / spent, 4), "unit": "pairs/s", "cores": 1,
                                    "sample": f"{runs} runs of the paper's sequential raster order, {spent:.1f} s"}
        if args.cpu_all_seconds > 0:
            print("[bench] oracle on every host core", file=sys.stderr, flush=True)
            cpu["all_cores"] = cpu_all_cores(params_d, args.cpu_all_seconds)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {"workload": "plain: one 1024x436 RGB pair per step, per-pair launches on one stream; "
                               "L=5, seed stride 3, 8x8 patch, 6 iterations per level, W=2, Sobel 5, "
                               "int16 gradients with int32 SAD, fwd+bwd check tau=1",
                   "global_batch": 1, "pairs_cycled": len(pairs)},
        "dist_evals_per_s": round(evals / elapsed, 1),
        "dist_evals_per_pair": evals / args.steps,
        "n_inliers_pair0": n_inl,
        "roofline": roofline,
        "kernels": kernels,
        "batched": groups,
        "batched_uniform": batched,
        "configs": configs,
        "served": served,
        "paper_preset": paper,
        "cpu_baseline": cpu,
        # the paper's own matching times (Table III), context only: other hardware, the dense
        # per-pixel method with 15/11 patches, the MPI Sintel and KITTI 2012 training sets
        "paper_runtimes_context": {
            "hardware": "Intel Pentium G3240 @3.1 GHz, 4 GB, one thread (Sec. IV)",
            "seconds_per_pair": {"PGM-C Sintel": 3.49, "PGM-C KITTI2012": 4.55, "PGM-G Sintel": 1.82,
                                 "PGM-G KITTI2012": 2.05, "PGM-CD Sintel": 1.56, "PGM-CD KITTI2012": 1.60,
                                 "PGM-GD Sintel": 1.08, "PGM-GD KITTI2012": 1.16}},
    }
    m.close()
    print(json.dumps(out), flush=True)


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
