"""Benchmark: TF update with partitioned distance maps vs full recompute.

Workload (default): tube-tree volume 1024x1024x795 uint8, bricks 4^3
(256x256x199 grid), 64 uniform partitions, the sequence of 200 random TFs
(1-3 trapezoid ramps).  One step is one pass of the whole path over that
input with the volume already resident in HBM:

  brick [min,max] -> 64 PDMs (one-time initialisation, Sec. 3.1)
  for each of the 200 TFs:
      TF update  (active set + Eq. 1 min-combine)  -> D'
      plain method (occupancy from the volume + distance map) -> D
      plain method from the cached brick [min,max] (no volume read) -> D

`value` is the partitioned TF update's throughput: (|S|+1)*G algorithmic
bytes per update, summed over the timed steps' updates, divided by the sum
of their durations (HIP events recorded on the stream the library launches
on), in GB/s.  The whole step's bytes over its wall time is `step_GBps`;
each call's p50/p90/p99 are reported beside it.  `roofline` is reported for
the kernel that takes most of the step (the plain method's occupancy pass
over the volume) and, as `roofline_tf_update`, for the min-combine kernel.
`served` is a short serving leg with admissions and evictions under load
(see served_leg()).  `cpu_baseline` is the CPU oracle timed on a slab of the
same volume on all host threads, `cpu_baseline_one_thread` on one thread
(see cpu_baseline()).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--tfs T]
                       [--no-cpu-baseline] [--no-served] [--calib-copy-mib M]
                       [--workload tube_tree|batched|served|sweep|configs]

--workload served: a Poisson stream of TF changes (2k/s) over 24 resident
volumes (22 of the batched recipe and two 1024x1024x795 tube trees) served
with continuous batching; p50/p99 latency and updates/s, beside the same
schedule through a serial full-recompute queue (service times measured per
volume on the GPU).  Then short load levels (--serve-load-rates) on the warm
servers, where batches form: achieved updates/s, mean batch, p50/p99.

--workload sweep: partition counts 16..256, uniform and with a partition of
its own for rho_min, on the CT-like u16 volume, the tube tree and an
832x832x494 stag-beetle-shaped u8 volume (see run_sweep).

--workload configs: every configuration (64^3 u8, 512x512x460 u16, the
1024x1024x795 tube tree), every TF of its sequence: TF update and full
recompute warm (back to back) and cold (L2 and MALL flushed by a 1 GiB write
before each timed call), GB/s against 8 TB/s and against a device copy
measured in the same run, the build split by phase, |S| per TF, and the
oracle on all host threads and on one.

--workload batched: 48 volumes of uneven sizes (96-640 per axis, half u8 and
half 12-bit u16, 16/32/64 partitions).  Times the batched build (grouped or
single launch, chosen with the rest of the launch shape by the autotuner)
against a per-volume launch loop, and the
one-launch TF update of all 48 volumes (a different TF each) against a
per-volume loop, each call timed alone and over calls issued back to back
(the value); checks that both ways give identical bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2407_21552_amd", "csrc", "pdm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tube_tree_1024x1024x795.md")

# paper's numbers (RTX 4090, OpenGL), kingsnake 1024x1024x795, 64 partitions
PAPER_CONTEXT = {
    "hardware": "NVIDIA RTX 4090 (paper, Table 1)",
    "dataset": "kingsnake 1024x1024x795, 64 partitions, TF1-TF6",
    "pdm_update_ms": [1.97, 1.99, 1.23, 1.23, 1.68, 1.26],
    "full_recompute_ms": [9.63, 7.28, 21.40, 14.59, 15.28, 9.76],
    "init_ms": 913.7,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the kernel source with comments and whitespace removed, so a
    comment edit does not orphan the counter record while any code change
    does."""
    import re
    text = open(KERNEL_SRC).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch measured with rocprofv3 counters (the JSON block
    of the traffic summary), valid only for the kernel source they were
    taken on."""
    try:
        text = open(TRAFFIC_FILE).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return rec


def range_table_leg(pdm, torch, stream, v, desc, bounds, alphas, masks, n, G, max_level):
    """Build the range table over the PDMs and run every TF through it (HIP
    events on the library's stream).  Checks D' against the plain update on
    every TF.  Bytes per update: (maps read + 1) * G."""
    maps = pdm.range_table_maps(n, max_level)
    table = torch.empty((maps, G), dtype=torch.uint8, device="cuda")
    ref = torch.empty_like(v.dist)
    out = torch.empty_like(v.dist)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    pdm.build_range_table(desc, v.pdms, n, max_level, table, stream)
    b0, b1 = ev(), ev()
    b0.record(stream)
    pdm.build_range_table(desc, v.pdms, n, max_level, table, stream)
    b1.record(stream)
    times, covers = [], []
    for a, m in zip(alphas, masks):
        pdm.tf_update(desc, v.pdms, bounds, a, ref, stream)
        e0, e1 = ev(), ev()
        e0.record(stream)
        pdm.tf_update_ranges(desc, v.pdms, table, bounds, max_level, a, out, stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        covers.append(len(pdm.range_cover(n, max_level, m)))
        assert torch.equal(out, ref), "range-table D' differs from the plain update"
    gbytes = sum((c + 1) * G for c in covers)
    return {"p50_ms": round(pct(times, 50), 4), "p99_ms": round(pct(times, 99), 4),
            "mean_ms": round(float(np.mean(times)), 4), "mean_maps_read": round(float(np.mean(covers)), 2),
            "GBps": round(gbytes / (sum(times) * 1e-3) / 1e9, 1),
            "table_maps": maps, "table_bytes": maps * G, "max_level": max_level,
            "table_build_ms": round(b0.elapsed_time(b1), 3),
            "identical_to_eq1_update": True}


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


def cpu_baseline(vol, bounds, alphas, levels, step_bytes_fn, slab_z=256, tfs=20, threads=None):
    """The CPU oracle (as it stands) on a bounded sample: the first `slab_z`
    z-slices of the volume, the full build plus `tfs` TFs through both the
    update and the plain method, on `threads` OpenMP threads (None: all the
    host's).  Each phase's oracle throughput (bytes/s on the slab) is applied
    to the full step's byte mix to give GB/s."""
    import oracle
    prev = oracle.threads()
    if threads is not None:
        oracle.set_threads(int(threads))
    try:
        return _cpu_baseline(oracle, vol, bounds, alphas, levels, step_bytes_fn, slab_z, tfs)
    finally:
        oracle.set_threads(prev)


def _cpu_baseline(oracle, vol, bounds, alphas, levels, step_bytes_fn, slab_z, tfs):
    slab = np.ascontiguousarray(vol[:slab_z])
    n = len(bounds) - 1
    t0 = time.perf_counter()
    bmin, bmax = oracle.bricks(slab)
    t1 = time.perf_counter()
    pd = oracle.pdms(slab, bounds, levels, brick_minmax=(bmin, bmax))
    t2 = time.perf_counter()
    upd_bytes = 0
    Gs = bmin.size
    for a in alphas[:tfs]:
        _, m = oracle.tf_update(pd, bounds, a, levels)
        upd_bytes += (len(oracle.active_list(m, n)) + 1) * Gs
    t3 = time.perf_counter()
    for a in alphas[:tfs]:
        oracle.full_recompute(slab, a, levels)
    t4 = time.perf_counter()
    s = slab.dtype.itemsize
    V = slab.size
    rate_bricks = (V * s + 2 * Gs * s) / (t1 - t0)
    rate_parts = (2 * Gs * s + n * Gs) / (t2 - t1)
    rate_upd = upd_bytes / (t3 - t2)
    rate_full = tfs * (V * s + Gs) / (t4 - t3)
    b = step_bytes_fn()
    return {
        "value": round(rate_upd / 1e9, 3),
        "unit": "GB/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"first {slab_z} of {vol.shape[0]} z-slices ({slab.shape[2]}x{slab.shape[1]}x"
                   f"{slab_z}; not the full volume), build + {tfs} TFs through update and full "
                   f"recompute, {t4 - t0:.1f} s; value = the oracle's TF-update rate, "
                   "(|S|+1)*G bytes per update over its time; per-phase rates scaled to "
                   "the full volume below"),
        "full_recompute_GBps": round(rate_full / 1e9, 3),
        "tf_update_ms_per_tf_full_volume": round(1e3 * b["tf_update"] / b["tfs"] / rate_upd, 3),
        "full_recompute_ms_per_tf_full_volume": round(
            1e3 * b["full_recompute"] / b["tfs"] / rate_full, 3),
        "build_ms_full_volume": round(1e3 * (b["bricks"] / rate_bricks + b["partitions"] / rate_parts), 1),
        "host": host_info(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tfs", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    ap.add_argument("--workload", default="tube_tree",
                    choices=("tube_tree", "batched", "served", "sweep", "configs"))
    ap.add_argument("--sweep-tfs", type=int, default=40)
    ap.add_argument("--config-tfs", type=int, default=200,
                    help="TFs per configuration for --workload configs (c1 has one)")
    ap.add_argument("--range-level", type=int, default=8,
                    help="top level of the range table (the TF updates through it are reported "
                         "beside the plain update)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-load-rates", default="20000,60000,150000",
                    help="comma-separated request rates of the served load levels")
    ap.add_argument("--serve-load-seconds", type=float, default=2.0)
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served leg of the default workload")
    ap.add_argument("--served-seconds", type=float, default=15.0,
                    help="length of the served leg of the default workload")
    ap.add_argument("--served-drift", type=float, default=1.0,
                    help="seconds per one-volume drift of the served leg's working set")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU layout is a design note, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_21552_amd as pdm
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "served":
        run_served(args)
        return
    if args.workload == "sweep":
        run_sweep(args)
        return
    if args.workload == "configs":
        run_configs(args)
        return
    cfg = W.config_info("c3")
    L, n = cfg["levels"], cfg["n"]
    log("generating tube-tree 1024x1024x795 u8 ...")
    vol = W.make_volume("c3")
    bounds = W.uniform_bounds(L, n)
    alphas = W.make_tfs("c3", args.tfs)
    T = len(alphas)

    t_vol = pdm.to_device(vol)
    v = pdm.Volume(t_vol, L, bounds)
    desc = v.desc
    G, V, s = v.G, vol.size, vol.dtype.itemsize
    d_full = torch.empty_like(v.dist)
    masks = [pdm.active_set(bounds, a, L) for a in alphas]
    s_sizes = [len(pdm.mask_to_list(m, n)) for m in masks]

    def step_bytes():
        b = {
            "bricks": V * s + 2 * G * s,
            "partitions": 2 * G * s + n * G,
            "tf_update": sum((k + 1) * G for k in s_sizes),
            "full_recompute": T * (V * s + G),
            "full_recompute_cached": T * (2 * G * s + G),
            "tfs": T,
        }
        b["total"] = (b["bricks"] + b["partitions"] + b["tf_update"] + b["full_recompute"]
                      + b["full_recompute_cached"])
        return b

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    d_cached = torch.empty_like(v.dist)

    def run_step(rec):
        e = [ev() for _ in range(4)]
        e[0].record(stream)
        pdm.build_bricks(desc, t_vol, v.bmin, v.bmax, None, stream)
        e[1].record(stream)
        pdm.pom_distance_x(desc, v.bmin, v.bmax, bounds, v.pdms, stream)
        e[2].record(stream)
        pdm.distance_yz(desc, v.pdms, n, stream)
        e[3].record(stream)
        rec["build"].append(e)
        for a in alphas:
            f = [ev() for _ in range(6)]
            f[0].record(stream)
            pdm.tf_update(desc, v.pdms, bounds, a, v.dist, stream)
            f[1].record(stream)
            pdm.plain_distance_x(desc, t_vol, a, d_full, stream)
            f[2].record(stream)
            pdm.distance_yz(desc, d_full, 1, stream)
            f[3].record(stream)
            pdm.plain_cached_distance_x(desc, v.bmin, v.bmax, a, d_cached, stream)
            f[4].record(stream)
            pdm.distance_yz(desc, d_cached, 1, stream)
            f[5].record(stream)
            rec["tf"].append(f)

    log(f"warmup {args.warmup} step(s) ...")
    for _ in range(args.warmup):
        run_step({"build": [], "tf": []})
    torch.cuda.synchronize()
    log(f"timing {args.steps} step(s) of build + {T} TFs ...")
    rec = {"build": [], "tf": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_step(rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps

    el = lambda a, b: a.elapsed_time(b)
    bricks_ms = [el(e[0], e[1]) for e in rec["build"]]
    pomx_ms = [el(e[1], e[2]) for e in rec["build"]]
    dyz_n_ms = [el(e[2], e[3]) for e in rec["build"]]
    upd_ms = [el(f[0], f[1]) for f in rec["tf"]]
    plx_ms = [el(f[1], f[2]) for f in rec["tf"]]
    dyz1_ms = [el(f[2], f[3]) for f in rec["tf"]]
    cx_ms = [el(f[3], f[4]) for f in rec["tf"]]
    cyz_ms = [el(f[4], f[5]) for f in rec["tf"]]
    full_ms = [a + b for a, b in zip(plx_ms, dyz1_ms)]
    cached_ms = [a + b for a, b in zip(cx_ms, cyz_ms)]
    upd_bytes = [(k + 1) * G for k in s_sizes] * args.steps
    sb = step_bytes()

    # parity spot checks on the last TF: D' <= D everywhere (Sec. 3.1), and
    # the plain method gives the same D from the volume and from the cached
    # brick ranges
    assert bool((v.dist <= d_full).all().item()), "D' > D"
    assert torch.equal(d_full, d_cached), "cached-range D differs from D"

    # the same TFs through the range table (outside the step: an option of
    # the update, not one of the method's steps)
    log("range table: build + the same TFs through it ...")
    rt = range_table_leg(pdm, torch, stream, v, desc, bounds, alphas, masks, n, G, args.range_level)

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read, {nb} bytes written")

    plain_bytes = V * s + G
    cached_bytes = 2 * G * s + G
    plain_avg_ms = float(np.mean(plx_ms))
    plain_gbps = plain_bytes / (plain_avg_ms * 1e-3) / 1e9
    upd_gbps = sum(upd_bytes) / (sum(upd_ms) * 1e-3) / 1e9
    traffic = load_traffic()

    def roofline(name, achieved, launches_bytes_note):
        r = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
             "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
             "traffic": None, "algorithmic": launches_bytes_note}
        if traffic and name in traffic.get("kernels", {}):
            k = traffic["kernels"][name]
            r["traffic"] = k["hbm_bytes_per_launch"]
            if k.get("algorithmic_bytes_per_launch"):
                # the counter runs' own launches (the combine's |S| differs per TF)
                r["traffic_vs_algorithmic"] = round(k["hbm_bytes_per_launch"]
                                                    / k["algorithmic_bytes_per_launch"], 4)
        return r

    total_by_kernel = {
        "k_plain_x": sum(plx_ms), "y/z scans, one map (k_dist_pairs)": sum(dyz1_ms) + sum(cyz_ms),
        "k_combine": sum(upd_ms), "k_plain_cached_x": sum(cx_ms), "k_bricks": sum(bricks_ms),
        "k_pom_x": sum(pomx_ms), "y/z scans, all partitions (k_dist_lines)": sum(dyz_n_ms)}

    def ms_stats(xs):
        return {"p50_ms": round(pct(xs, 50), 4), "p90_ms": round(pct(xs, 90), 4),
                "p99_ms": round(pct(xs, 99), 4), "mean_ms": round(float(np.mean(xs)), 4)}

    out = {
        "metric": "TF-update ms & GB/s (partitioned vs full recompute), 1024³ u8; p50/p99 served",
        "value": round(upd_gbps, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded tube-tree volume and trapezoid TFs standing in for kingsnake)",
        "config": {"workload": "tube-tree 1024x1024x795 u8, bricks 4^3 (256x256x199), "
                               f"64 uniform partitions, {T} TFs (1-3 ramps); step = build + "
                               f"{T} x (TF update + full recompute from the volume + full "
                               "recompute from the cached brick ranges)",
                   "volume_zyx": list(vol.shape), "partitions": n, "tfs": T, "brick": 4},
        "value_is": ("partitioned TF update (Sec. 3.1, Eq. 1): sum over the timed steps' updates of "
                     "(|S|+1)*G bytes / sum of their HIP-event durations"),
        "step_GBps": round(sb["total"] * args.steps / wall / 1e9, 2),
        "tf_update": {**ms_stats(upd_ms), "GBps": round(upd_gbps, 1),
                      "mean_active_partitions": round(float(np.mean(s_sizes)), 2)},
        "full_recompute": {**ms_stats(full_ms),
                           "occupancy_x_mean_ms": round(plain_avg_ms, 4),
                           "distance_yz_mean_ms": round(float(np.mean(dyz1_ms)), 4),
                           "GBps": round(T * plain_bytes * args.steps / (sum(full_ms) * 1e-3) / 1e9, 1)},
        "full_recompute_cached": {**ms_stats(cached_ms),
                                  "occupancy_x_mean_ms": round(float(np.mean(cx_ms)), 4),
                                  "distance_yz_mean_ms": round(float(np.mean(cyz_ms)), 4),
                                  "bytes_per_call": cached_bytes,
                                  "GBps": round(T * cached_bytes * args.steps / (sum(cached_ms) * 1e-3) / 1e9, 1),
                                  "identical_to_full_recompute": True},
        "speedup_update_vs_full": {"p50": round(pct(full_ms, 50) / pct(upd_ms, 50), 2),
                                   "mean": round(float(np.mean(full_ms)) / float(np.mean(upd_ms)), 2)},
        "speedup_update_vs_cached": {"p50": round(pct(cached_ms, 50) / pct(upd_ms, 50), 2),
                                     "mean": round(float(np.mean(cached_ms)) / float(np.mean(upd_ms)), 2)},
        "build": {"bricks_ms": round(float(np.median(bricks_ms)), 4),
                  "pom_x_ms": round(float(np.median(pomx_ms)), 4),
                  "distance_yz_ms": round(float(np.median(dyz_n_ms)), 4),
                  "total_ms": round(float(np.median(np.add(np.add(bricks_ms, pomx_ms), dyz_n_ms))), 4),
                  "bricks_GBps": round((V * s + 2 * G * s) / (np.median(bricks_ms) * 1e-3) / 1e9, 1)},
        "kernel_time_share": {k: round(t / sum(total_by_kernel.values()), 4)
                              for k, t in total_by_kernel.items()},
        "roofline": roofline("k_plain_x", plain_gbps,
                             f"V*s + G = {plain_bytes} B per launch (volume read + x-distance write)"),
        "roofline_tf_update": roofline("k_combine", upd_gbps,
                                       "(|S|+1)*G B per launch, summed over the TFs"),
        "tf_update_range_table": {
            **rt, "speedup_vs_eq1_update_p50": round(pct(upd_ms, 50) / rt["p50_ms"], 2),
            "speedup_vs_full_p50": round(pct(full_ms, 50) / rt["p50_ms"], 2)},
        "paper_context": PAPER_CONTEXT,
        "kernel_source_sha256_16": kernel_hash(),
    }
    if not args.no_served:
        torch.cuda.empty_cache()
        out["served"] = served_leg(args, torch, pdm, W, vol)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a slab (all host threads) ...")
        out["cpu_baseline"] = cpu_baseline(vol, bounds, alphas, L, step_bytes)
        log("timing the CPU oracle on a thinner slab (one thread) ...")
        out["cpu_baseline_one_thread"] = cpu_baseline(vol, bounds, alphas, L, step_bytes,
                                                      slab_z=32, tfs=10, threads=1)
    print(json.dumps(out), flush=True)


def served_leg(args, torch, pdm, W, tube_tree):
    """Continuous batching with admissions under load: a catalog of 32
    volumes (28 of the batched recipe, the step's tube tree and a second
    one) behind a server with 24 slots and a 200 GB budget.  Poisson
    requests at --serve-rate for --served-seconds; the working set of 24
    volumes drifts by one volume every --served-drift seconds, so new
    volumes are admitted (pinned host voxels copied on the admission stream,
    then built) and LRU volumes evicted while the stream runs.  Reports the
    served p50/p99 latency (arrival to completion, admissions included),
    updates/s, admissions and evictions, and the same schedule through a
    serial full-recompute queue (per-volume service times measured here)."""
    from paper_2407_21552_amd.serve import GpuExecutor, Server, VolumeSpec, requests_from
    log("served leg: generating a catalog of 32 volumes ...")
    cat, pinned = {}, {}

    def pin(a):
        a = np.ascontiguousarray(a)
        t = torch.from_numpy(a.view(np.int16) if a.dtype == np.uint16 else a)
        return t.pin_memory()

    specs = W.batch_specs(30, seed=6)
    order = list(range(24)) + [30, 31] + list(range(24, 30))
    for k, sp in enumerate(specs):
        pinned[k] = pin(W.batch_volume(sp))
        cat[k] = VolumeSpec(k, sp["shape"], sp["dtype"], sp["levels"],
                            W.uniform_bounds(sp["levels"], sp["n"]), lambda k=k: pinned[k])
    for k, host in ((30, tube_tree), (31, W.tube_tree_u8(seed=33))):
        pinned[k] = pin(host)
        cat[k] = VolumeSpec(k, host.shape, np.uint8, 256, W.uniform_bounds(256, 64),
                            lambda k=k: pinned[k])
    ids = order
    arrivals = W.poisson_requests(args.serve_rate, args.served_seconds, ids,
                                  {k: cat[k].levels for k in cat}, seed=12,
                                  window=(24, args.served_drift))
    ex = GpuExecutor(outputs_per_volume=8)
    srv = Server(ex, cat, budget_bytes=200 << 30, max_slots=24)
    # warm start: the first working set resident before the stream
    for k in ids[:24]:
        srv._ensure(k)
    torch.cuda.synchronize()
    for h in srv.resident.values():
        ex.ready(h)
    srv.stats.clear()
    sched = requests_from(arrivals)
    log(f"served leg: {len(sched)} requests over {args.served_seconds:.0f} s, working set drifting "
        f"every {args.served_drift:.1f} s ...")
    srv.t0 = srv.clock()
    srv.run(sched, timeout=args.served_seconds + 60)
    torch.cuda.synchronize()
    rep = srv.report()
    admitted = {r.vol_id for r in sched} - set(ids[:24])
    lat_cold = [r.done - r.arrival for r in srv.completed if r.vol_id in admitted]
    # per-volume service time of the plain method (volume resident), for the
    # serial full-recompute queue over the same schedule
    log("served leg: per-volume full recompute times ...")
    stream = torch.cuda.current_stream()
    full_s = {}
    for k, spec in cat.items():
        vol_dev = pinned[k].to("cuda")
        desc = pdm.volume_desc(spec.shape, spec.dtype, spec.levels)
        a = W.trapezoid_tf(spec.levels, 2, np.random.default_rng(k))
        d = torch.empty(pdm.grid_of(desc)[3], dtype=torch.uint8, device="cuda")
        pdm.full_recompute(desc, vol_dev, a, d, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            pdm.full_recompute(desc, vol_dev, a, d, stream)
        e1.record(stream)
        e1.synchronize()
        full_s[k] = e0.elapsed_time(e1) / 5 * 1e-3
        del vol_dev
    rnd = lambda x: None if x is None else round(x, 4)
    return {
        "workload": (f"Poisson {args.serve_rate:.0f}/s over {args.served_seconds:.0f} s; catalog of 32 "
                     "volumes (30 of U{96..640}^3 mixed u8/u16 with 16/32/64 partitions, 2 x "
                     "1024x1024x795 u8 tube trees with 64), 24 slots, 200 GB budget; the working set "
                     f"of 24 drifts by one volume every {args.served_drift:.1f} s (admission + LRU "
                     "eviction under load); up to 48 requests per launch"),
        "requests": len(sched),
        "p50_ms": rnd(rep["p50_ms"]), "p99_ms": rnd(rep["p99_ms"]), "mean_ms": rnd(rep["mean_ms"]),
        "updates_per_s": rnd(rep["updates_per_s"]), "completed": rep["completed"],
        "rejected": rep["rejected"], "launches": rep["launches"], "mean_batch": rnd(rep["mean_batch"]),
        "admissions": rep["admissions"], "evictions": rep["evictions"],
        "requests_to_admitted_volumes": len(lat_cold),
        "p99_ms_requests_to_admitted_volumes": rnd(float(np.percentile(lat_cold, 99)) * 1e3
                                                   if lat_cold else None),
        "serial_full_recompute": serial_queue(sched, full_s),
    }


def run_batched(args):
    """48 uneven volumes: the batched build (launch shape and grouped or
    single launch from the autotuner) and the one-launch TF update against
    per-volume launch loops."""
    import torch
    import paper_2407_21552_amd as pdm
    from paper_2407_21552_amd import autotune
    import workloads as W

    specs = W.batch_specs()
    vols, alphas = [], []
    log("generating and uploading 48 volumes ...")
    for k, sp in enumerate(specs):
        vol = W.batch_volume(sp)
        bounds = W.uniform_bounds(sp["levels"], sp["n"])
        v = pdm.Volume(pdm.to_device(vol), sp["levels"], bounds, voxel_dtype=sp["dtype"])
        vols.append(v)
        rng = np.random.default_rng(40_000 + k)
        alphas.append(W.trapezoid_tf(sp["levels"], int(rng.integers(1, 5)), rng))
        del vol
    stream = torch.cuda.current_stream()
    items = [(v.desc, v.volume, v.bmin, v.bmax, v.bounds, v.pdms) for v in vols]
    ws = torch.zeros(pdm.batch_workspace_bytes(len(items)), dtype=torch.uint8, device="cuda")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out))

    def loop_build():
        for v in vols:
            pdm.build_bricks(v.desc, v.volume, v.bmin, v.bmax, None, stream)
            pdm.build_partitions(v.desc, v.bmin, v.bmax, v.bounds, v.pdms, stream)

    log("per-volume build loop ...")
    loop_ms = timed(loop_build, args.steps)
    ref = [v.pdms.clone() for v in vols]
    log("autotuning the batched build ...")
    best, table = autotune.tune_batch_build(items, ws, reps=3, cache_path=None, stream=stream)
    for v in vols:
        v.pdms.fill_(0)
    batch_ms = timed(lambda: pdm.batch_build(items, ws, best, stream), args.steps)
    same_build = all(bool(torch.equal(a, v.pdms)) for a, v in zip(ref, vols))
    default_ms = timed(lambda: pdm.batch_build(items, ws, None, stream), args.steps)

    outs_loop = [torch.empty_like(v.dist) for v in vols]
    outs_batch = [torch.empty_like(v.dist) for v in vols]

    def loop_update():
        for v, a, o in zip(vols, alphas, outs_loop):
            pdm.tf_update(v.desc, v.pdms, v.bounds, a, o, stream)

    def back_to_back(fn, reps):
        # mean per call over calls issued without waiting: the host prepares a
        # call while the device still runs the previous one
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / reps

    upd_items = [(v.prepared, a, o) for v, a, o in zip(vols, alphas, outs_batch)]
    log("TF updates: per-volume loop vs one launch ...")
    upd_loop_ms = timed(loop_update, 20)
    masks = pdm.batch_tf_update_prepared(upd_items, stream)
    upd_batch_ms = timed(lambda: pdm.batch_tf_update_prepared(upd_items, stream), 20)
    same_update = all(bool(torch.equal(a, b)) for a, b in zip(outs_loop, outs_batch))
    upd_loop_b2b = back_to_back(loop_update, 20)
    upd_batch_b2b = back_to_back(lambda: pdm.batch_tf_update_prepared(upd_items, stream), 20)
    t0 = time.perf_counter()
    for _ in range(200):
        pdm.active_set(vols[0].bounds, alphas[0], vols[0].levels)
    host_set_us = (time.perf_counter() - t0) / 200 * 1e6

    G_tot = sum(v.G for v in vols)
    vox_bytes = sum(v.volume.numel() * v.volume.element_size() for v in vols)
    build_bytes = sum(v.volume.numel() * v.volume.element_size() + 4 * v.G * v.voxel_dtype.itemsize
                      + v.n * v.G for v in vols)
    upd_bytes = sum((len(pdm.mask_to_list(m, v.n)) + 1) * v.G for m, v in zip(masks, vols))
    out = {
        "metric": "batched build and TF update of 48 uneven volumes (ms), one launch vs per-volume loop",
        "value": round(upd_bytes / (upd_batch_b2b * 1e-3) / 1e9, 1),
        "unit": "GB/s (batched TF update, calls back to back)",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic (48 seeded volumes: ellipsoid u8 and CT-like 12-bit u16)",
        "config": {"workload": "48 volumes, dims U{96..640}, half u8 / half u16 (12-bit), "
                               "partitions from {16,32,64}, bricks 4^3",
                   "volumes": len(vols), "voxels_bytes": vox_bytes, "bricks_total": G_tot,
                   "pdm_bytes": sum(v.n * v.G for v in vols)},
        "build": {"per_volume_loop_ms": round(loop_ms, 3), "batched_tuned_ms": round(batch_ms, 3),
                  "batched_default_ms": round(default_ms, 3),
                  "best_grouped_ms": round(min(t for k, t in table.items()
                                               if '"single_launch": 0' in k), 3),
                  "best_single_launch_ms": round(min(t for k, t in table.items()
                                                     if '"single_launch": 1' in k), 3),
                  "speedup_vs_loop": round(loop_ms / batch_ms, 3),
                  "GBps_batched": round(build_bytes / (batch_ms * 1e-3) / 1e9, 1),
                  "tuned_config": best, "identical_to_loop": same_build,
                  "autotune_table_ms": {k: round(t, 3) for k, t in sorted(table.items(), key=lambda kv: kv[1])}},
        "tf_update": {"per_volume_loop_ms": round(upd_loop_ms, 4), "batched_ms": round(upd_batch_ms, 4),
                      "speedup_vs_loop": round(upd_loop_ms / upd_batch_ms, 3),
                      "GBps_batched": round(upd_bytes / (upd_batch_ms * 1e-3) / 1e9, 1),
                      "back_to_back_loop_ms": round(upd_loop_b2b, 4),
                      "back_to_back_batched_ms": round(upd_batch_b2b, 4),
                      "back_to_back_speedup": round(upd_loop_b2b / upd_batch_b2b, 3),
                      "bytes": upd_bytes,
                      "host_active_set_us": round(host_set_us, 2),
                      "identical_to_loop": same_update},
    }
    print(json.dumps(out), flush=True)


def host_info() -> dict:
    """CPU model and thread counts of the machine that runs the oracle."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline_rates(vol, bounds, alphas, levels, max_tfs, budget_s, one_thread_tfs,
                       one_thread_budget_s):
    """The CPU-baseline leg of the per-configuration workload: the oracle's
    throughput (bytes/s) on `vol`, the build with all host threads, then the
    TF update and the full recompute with all threads and with one (at most
    the given TF counts, about the given seconds per phase).  The PDMs built
    once serve both thread counts."""
    import oracle
    all_threads = oracle.threads()
    n = len(bounds) - 1
    s, V = vol.dtype.itemsize, vol.size
    t0 = time.perf_counter()
    bmin, bmax = oracle.bricks(vol)
    G = bmin.size
    pd = oracle.pdms(vol, bounds, levels, brick_minmax=(bmin, bmax))
    t1 = time.perf_counter()
    out = {"build_Bps": (V * s + 4 * G * s + n * G) / (t1 - t0), "threads": all_threads}

    def phases(max_k, budget):
        upd_bytes, k, t2 = 0, 0, time.perf_counter()
        for a in alphas[:max_k]:
            _, m = oracle.tf_update(pd, bounds, a, levels)
            upd_bytes += (len(oracle.active_list(m, n)) + 1) * G
            k += 1
            if time.perf_counter() - t2 > budget:
                break
        t3 = time.perf_counter()
        r = {"tf_update_Bps": upd_bytes / (t3 - t2), "tf_update_tfs": k}
        k = 0
        for a in alphas[:max_k]:
            oracle.full_recompute(vol, a, levels)
            k += 1
            if time.perf_counter() - t3 > budget:
                break
        r["full_recompute_Bps"] = k * (V * s + G) / (time.perf_counter() - t3)
        r["full_recompute_tfs"] = k
        return r

    out["all_threads"] = phases(max_tfs, budget_s)
    oracle.set_threads(1)
    try:
        out["one_thread"] = phases(one_thread_tfs, one_thread_budget_s)
    finally:
        oracle.set_threads(all_threads)
    return out


def run_configs(args):
    """Per configuration (c1 64^3 u8, c2 512x512x460 u16, c3 1024x1024x795 u8),
    every TF of its sequence: the TF update and the full recompute timed per
    call, warm (the previous call's data left in the caches; a spin kernel
    keeps the device busy across the start event) and cold (a 1 GiB scratch
    write before every timed call, outside the timing, so that neither L2 nor
    the 256 MB MALL holds anything of the call's inputs); GB/s as summed bytes over
    summed time; roofline fractions against 8 TB/s and against a device copy
    measured in the same process; the build split into bricks, POM + x pass
    and y/z passes (median of 5); |S| per TF; the CPU oracle on all host
    threads and on one (c3 on its first 256 z-slices, rates applied to the
    full volume).  The same in the EXACT reading (occupancy from the brick's
    voxels): its build, full recompute and update, and how much larger its
    distances run than RANGE's.  Last, c3's first 100 z-slices: one GPU's
    share when the volume is split into 8 z-slabs."""
    import torch
    import paper_2407_21552_amd as pdm
    import workloads as W

    stream = torch.cuda.current_stream()
    scratch = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    # copy ceiling: 1 GiB device-to-device, best of 5 (2 GiB moved)
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(3)
    best = 1e9
    for _ in range(6):
        a = ev()
        scratch.copy_(src)
        b = ev()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    copy_gbps = 2 * (1 << 30) / (best * 1e-3) / 1e9
    del src
    torch.cuda.empty_cache()
    log(f"device copy ceiling {copy_gbps:.0f} GB/s")

    def stats(ms, bytes_each, small):
        d = {"p50_ms": round(pct(ms, 50), 4), "p90_ms": round(pct(ms, 90), 4),
             "mean_ms": round(float(np.mean(ms)), 4)}
        if small:
            d["p50_us"] = round(1e3 * pct(ms, 50), 2)
            d["GBps"] = "n/m"
        else:
            gbps = sum(bytes_each) / (sum(ms) * 1e-3) / 1e9
            d["GBps"] = round(gbps, 1)
            d["frac_hbm_peak"] = round(gbps / HBM_PEAK_GBPS, 4)
            d["frac_copy_ceiling"] = round(gbps / copy_gbps, 4)
        return d

    results = []
    c3_vol = None
    # c3_slab8: the first 100 z-slices of c3 (25 brick layers), the share of
    # one GPU when the volume is split into 8 z-slabs (the update and the
    # slab-local build phases are that GPU's work as they stand; its z pass
    # would need the other slabs' columns)
    for name in ("c1", "c2", "c3", "c3_slab8"):
        c = W.config_info("c3" if name == "c3_slab8" else name)
        L, n = c["levels"], c["n"]
        if name == "c3_slab8":
            vol = np.ascontiguousarray(c3_vol[:100])
            c3_vol = None
        else:
            log(f"{name}: generating {c['shape']} ...")
            vol = W.make_volume(name)
            if name == "c3":
                c3_vol = vol
        bounds = W.uniform_bounds(L, n)
        alphas = W.make_tfs("c3" if name == "c3_slab8" else name, None if name == "c1" else args.config_tfs)
        T = len(alphas)
        t_vol = pdm.to_device(vol)
        v = pdm.Volume(t_vol, L, bounds, voxel_dtype=vol.dtype)
        desc, G, V, s = v.desc, v.G, vol.size, vol.dtype.itemsize
        small = name == "c1"
        d_full = torch.empty_like(v.dist)
        sizes = [len(pdm.mask_to_list(pdm.active_set(bounds, a, L), n)) for a in alphas]
        upd_b = [(k + 1) * G for k in sizes]
        full_b = [V * s + G] * T
        # build, median of 5
        bt = []
        for _ in range(6):
            e = [ev()]
            pdm.build_bricks(desc, t_vol, v.bmin, v.bmax, None, stream)
            e.append(ev())
            pdm.pom_distance_x(desc, v.bmin, v.bmax, bounds, v.pdms, stream)
            e.append(ev())
            pdm.distance_yz(desc, v.pdms, n, stream)
            e.append(ev())
            bt.append(e)
        torch.cuda.synchronize()
        bt = bt[1:]
        build = {k: round(float(np.median([e[i].elapsed_time(e[i + 1]) for e in bt])), 4)
                 for i, k in enumerate(("bricks_ms", "pom_x_ms", "distance_yz_ms"))}
        build["total_ms"] = round(sum(build.values()), 4)

        def busy(cold, k):
            # the device must be busy when the start event is recorded, or the
            # event fires while the host still prepares the call and the host
            # time is counted: a 1 GiB write (cold) or a spin that touches no
            # memory (warm)
            if cold:
                scratch.fill_(k & 255)
            else:
                torch.cuda._sleep(100_000)

        def timed(cold, fn):
            out = []
            for k, a in enumerate(alphas):
                busy(cold, k)
                e0 = ev()
                fn(a)
                e1 = ev()
                out.append((e0, e1))
            torch.cuda.synchronize()
            return [x.elapsed_time(y) for x, y in out]

        def full_phases(cold, exact=False):
            occ_x = pdm.plain_exact_distance_x if exact else pdm.plain_distance_x
            out = []
            for k, a in enumerate(alphas):
                busy(cold, k)
                e0 = ev()
                occ_x(desc, t_vol, a, d_full, stream)
                e1 = ev()
                pdm.distance_yz(desc, d_full, 1, stream)
                e2 = ev()
                out.append((e0, e1, e2))
            torch.cuda.synchronize()
            return ([x.elapsed_time(y) for x, y, _ in out], [y.elapsed_time(z) for _, y, z in out])

        upd = lambda a: pdm.tf_update(desc, v.pdms, bounds, a, v.dist, stream)
        cached = lambda a: pdm.full_recompute_cached(desc, v.bmin, v.bmax, a, d_full, stream)
        cached_b = [2 * G * s + G] * T
        timed(False, upd)  # warm-up
        timed(False, cached)
        rec = {}
        for mode in ("warm", "cold"):
            log(f"{name}: {T} TFs, {mode} ...")
            u = timed(mode == "cold", upd)
            ox, yz = full_phases(mode == "cold")
            fm = [a + b for a, b in zip(ox, yz)]
            cm = timed(mode == "cold", cached)
            rec[mode] = {"tf_update": stats(u, upd_b, small),
                         "full_recompute": {**stats(fm, full_b, small),
                                            "occupancy_x_mean_ms": round(float(np.mean(ox)), 4),
                                            "distance_yz_mean_ms": round(float(np.mean(yz)), 4)},
                         "full_recompute_cached": stats(cm, cached_b, True),
                         "speedup_p50": round(pct(fm, 50) / pct(u, 50), 2),
                         "speedup_vs_cached_p50": round(pct(cm, 50) / pct(u, 50), 2)}
        # EXACT reading (occupancy from the brick's voxels): build, full
        # recompute warm and cold, and the update over the EXACT PDMs; and how
        # much larger its distances run than RANGE's (EXACT occupancy is a
        # subset, so its distances are >= RANGE's)
        exact = None
        if name != "c3_slab8":
            pdms_x = torch.empty_like(v.pdms)
            d_xu = torch.empty_like(v.dist)
            bx = []
            for _ in range(6):
                e = [ev()]
                pdm.pom_exact_distance_x(desc, t_vol, bounds, pdms_x, stream)
                e.append(ev())
                pdm.distance_yz(desc, pdms_x, n, stream)
                e.append(ev())
                bx.append(e)
            torch.cuda.synchronize()
            bx = bx[1:]
            xb = {"pom_exact_x_ms": round(float(np.median([e[0].elapsed_time(e[1]) for e in bx])), 4),
                  "distance_yz_ms": round(float(np.median([e[1].elapsed_time(e[2]) for e in bx])), 4)}
            xb["total_ms"] = round(xb["pom_exact_x_ms"] + xb["distance_yz_ms"], 4)
            xupd = lambda a: pdm.tf_update(desc, pdms_x, bounds, a, d_xu, stream)
            timed(False, xupd)  # warm-up
            xrec = {}
            for mode in ("warm", "cold"):
                log(f"{name}: EXACT, {T} TFs, {mode} ...")
                u = timed(mode == "cold", xupd)
                ox, yz = full_phases(mode == "cold", exact=True)
                fm = [a + b for a, b in zip(ox, yz)]
                xrec[mode] = {"tf_update": stats(u, upd_b, small),
                              "full_recompute": {**stats(fm, full_b, small),
                                                 "occupancy_x_mean_ms": round(float(np.mean(ox)), 4),
                                                 "distance_yz_mean_ms": round(float(np.mean(yz)), 4)}}
            # tightness on three TFs: D' and D in both readings
            cmp_ = []
            for a in alphas[:3]:
                pdm.tf_update(desc, v.pdms, bounds, a, v.dist, stream)
                pdm.tf_update(desc, pdms_x, bounds, a, d_xu, stream)
                pdm.full_recompute(desc, t_vol, a, d_full, stream)
                dxf = torch.empty_like(d_full)
                pdm.full_recompute_exact(desc, t_vol, a, dxf, stream)
                torch.cuda.synchronize()
                r_dp, x_dp = v.dist.float(), d_xu.float()
                cmp_.append({"dprime_exact_gt_range_frac": float((d_xu > v.dist).float().mean()),
                             "dprime_mean_range": float(r_dp.mean()),
                             "dprime_mean_exact": float(x_dp.mean()),
                             "d_exact_gt_range_frac": float((dxf > d_full).float().mean()),
                             "exact_dprime_le_exact_d": bool((d_xu <= dxf).all())})
            exact = {"build": xb, **xrec,
                     "vs_range": {k: (round(float(np.mean([c[k] for c in cmp_])), 4) if k != "exact_dprime_le_exact_d"
                                      else all(c[k] for c in cmp_)) for k in cmp_[0]}}
            del pdms_x, d_xu
        entry = {"config": name, "shape_zyx": list(vol.shape), "dtype": str(vol.dtype), "levels": L,
                 "partitions": n, "G": G, "seeds": {"volume": c["seed"], "tf_base": c["tf_seed"]},
                 "tfs": T, "active_partitions": {"mean": round(float(np.mean(sizes)), 2),
                                                 "min": int(min(sizes)), "max": int(max(sizes)),
                                                 "per_tf": sizes},
                 "build": build, **rec}
        if exact is not None:
            entry["exact"] = exact
        if name == "c3_slab8":
            entry["note"] = ("one GPU's share of c3 split into 8 z-slabs; the update and the bricks, "
                             "POM + x and y phases are that GPU's work, the z pass would need the "
                             "other slabs' columns (one exchange per volume load)")
        if not args.no_cpu_baseline and name != "c3_slab8":
            host = vol if name != "c3" else np.ascontiguousarray(vol[:256])
            scale = vol.size / host.size
            log(f"{name}: CPU oracle, all threads and one ...")
            r = cpu_baseline_rates(host, bounds, alphas, L, T, 15.0, 20, 6.0)
            cpu = {"build_ms": round(1e3 * (V * s + 4 * G * s + n * G) / r["build_Bps"], 1),
                   "build_threads": r["threads"]}
            for label in ("all_threads", "one_thread"):
                q = r[label]
                cpu[label] = {"threads": r["threads"] if label == "all_threads" else 1,
                              "tf_update_ms_per_tf": round(1e3 * float(np.mean(upd_b)) / q["tf_update_Bps"], 3),
                              "full_recompute_ms_per_tf": round(1e3 * (V * s + G) / q["full_recompute_Bps"], 3),
                              "tfs_timed": [q["tf_update_tfs"], q["full_recompute_tfs"]]}
            entry["cpu_baseline"] = {**cpu, "kind": "oracle", "sample": "full volume" if scale == 1 else
                                   f"first 256 z-slices, rates applied to the full volume ({scale:.2f}x)"}
        results.append(entry)
        del v, t_vol, d_full, vol
        torch.cuda.empty_cache()
    c3 = next(r for r in results if r["config"] == "c3")["cold"]["tf_update"]
    out = {
        "metric": "TF update and full recompute per configuration (c1, c2, c3), warm and cold, "
                  "GB/s and roofline fractions",
        "value": c3["GBps"],
        "unit": "GB/s (c3 TF update, cold)",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u8",
        "data": "synthetic (seeded configurations c1-c3)",
        "config": {"workload": "c1 64^3 u8 n=8; c2 512x512x460 u16 (12-bit) n=32; "
                               "c3 1024x1024x795 u8 n=64; c3_slab8 its first 100 z-slices; "
                               "bricks 4^3", "tfs": args.config_tfs},
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "copy_ceiling": "1 GiB device-to-device copy (torch copy_, best of 5), 2 GiB moved",
        "host": host_info(),
        "configs": results,
    }
    print(json.dumps(out), flush=True)


def serial_queue(schedule, service_s):
    """Latencies of a single server taking requests in arrival order with the
    given per-volume service times (seconds)."""
    free = 0.0
    lat = []
    for r in schedule:
        start = max(free, r.arrival)
        free = start + service_s[r.vol_id]
        lat.append(free - r.arrival)
    lat = np.array(lat)
    span = free - schedule[0].arrival
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "updates_per_s": round(len(schedule) / span, 1)}


def run_served(args):
    import torch
    import paper_2407_21552_amd as pdm
    from paper_2407_21552_amd.serve import GpuExecutor, Server, VolumeSpec, requests_from
    import workloads as W

    log("generating the catalog (22 batch-recipe volumes + 2 tube trees) ...")
    cat, host = {}, {}
    for k, sp in enumerate(W.batch_specs(22, seed=6)):
        host[k] = W.batch_volume(sp)
        cat[k] = VolumeSpec(k, sp["shape"], sp["dtype"], sp["levels"],
                            W.uniform_bounds(sp["levels"], sp["n"]), lambda k=k: host[k])
    for j, seed in enumerate((3, 33)):
        k = 22 + j
        host[k] = W.tube_tree_u8(seed=seed)
        cat[k] = VolumeSpec(k, host[k].shape, np.uint8, 256, W.uniform_bounds(256, 64),
                            lambda k=k: host[k])
    arrivals = W.poisson_requests(args.serve_rate, args.serve_seconds, list(cat),
                                  {k: cat[k].levels for k in cat}, seed=12)
    rates = [float(r) for r in args.serve_load_rates.split(",") if r.strip()]

    def serve_on(srv, arr, seconds):
        # one stream on a warm server: counters and results start afresh
        srv.completed, srv.rejected = [], []
        srv.stats.clear()
        sched = requests_from(arr)
        srv.t0 = srv.clock()
        srv.run(sched, timeout=seconds + 60)
        torch.cuda.synchronize()
        return sched, srv.report()

    def serve(range_level):
        ex = GpuExecutor(outputs_per_volume=8, range_level=range_level)
        srv = Server(ex, cat, budget_bytes=200 << 30, max_slots=24)
        log(f"admitting all volumes (warm start), range level {range_level} ...")
        for k in cat:
            srv._ensure(k)
        torch.cuda.synchronize()
        for h in srv.resident.values():
            ex.ready(h)
        log(f"serving {len(arrivals)} requests over {args.serve_seconds:.0f} s ...")
        sched, rep = serve_on(srv, arrivals, args.serve_seconds)
        load = []
        for k, rate in enumerate(rates):
            arr = W.poisson_requests(rate, args.serve_load_seconds, list(cat),
                                     {v: cat[v].levels for v in cat}, seed=40 + k, tf_pool=16)
            log(f"load {rate:.0f}/s: {len(arr)} requests over {args.serve_load_seconds:.1f} s ...")
            _, r = serve_on(srv, arr, args.serve_load_seconds)
            load.append({"rate_hz": rate, **r})
        return srv, sched, rep, load

    srv_rt, _, rep_rt, load_rt = serve(args.range_level)
    del srv_rt
    torch.cuda.empty_cache()
    srv, sched, rep, load = serve(None)

    # per-volume service times of the plain method and of a single update
    log("measuring per-volume full recompute and single update times ...")
    stream = torch.cuda.current_stream()
    full_s, upd_s = {}, {}
    for k, h in srv.resident.items():
        v = h.vol
        vol_dev = pdm.to_device(host[k])
        a = W.trapezoid_tf(cat[k].levels, 2, np.random.default_rng(k))
        d = torch.empty_like(v.dist)
        for name, fn, store in (("full", lambda: pdm.full_recompute(v.desc, vol_dev, a, d, stream), full_s),
                                ("upd", lambda: pdm.tf_update(v.desc, v.pdms, v.bounds, a, d, stream), upd_s)):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(5):
                fn()
            e1.record(stream)
            e1.synchronize()
            store[k] = e0.elapsed_time(e1) / 5 * 1e-3
        del vol_dev
    out = {
        "metric": "served TF updates: p50/p99 latency (ms) and updates/s, continuous batching "
                  "(batched update of the active PDMs; range tables beside it)",
        "value": rep["updates_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic (22 batch-recipe volumes and two tube-tree volumes)",
        "config": {"workload": f"Poisson {args.serve_rate:.0f}/s over {args.serve_seconds:.0f} s, "
                               "24 resident volumes (22 U{96..640}^3 mixed u8/u16 + 2 x "
                               "1024x1024x795 u8), 200 GB budget, up to 48 requests per launch",
                   "requests": len(sched), "rate_hz": args.serve_rate},
        "served": rep,
        "served_range_tables": {**rep_rt, "range_level": args.range_level},
        "load": {"seconds": args.serve_load_seconds, "tfs_per_volume": 16,
                 "batched": load, "range_tables": load_rt},
        "serial_full_recompute": serial_queue(sched, full_s),
        "serial_single_update": serial_queue(sched, upd_s),
        "service_ms_mean": {"full_recompute": round(1e3 * float(np.mean(list(full_s.values()))), 4),
                            "tf_update": round(1e3 * float(np.mean(list(upd_s.values()))), 4)},
    }
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """Partition sweep: n = 16..256 with uniform partitions and with a
    partition of its own for the minimum intensity (Sec. 3.1 and Fig. 4), on
    the CT-like 512x512x460 u16, the 1024x1024x795 tube tree and an
    832x832x494 stag-beetle-shaped u8 volume whose background sits at
    rho_min.  Per point: init time (bricks + PDMs), PDM bytes n*G, TF-update
    and full-recompute times over the same TFs, and how much of the plain
    method's distance D the update keeps (D' == D fraction, mean D' / mean
    D; D' <= D always)."""
    import torch
    import paper_2407_21552_amd as pdm
    import workloads as W

    stream = torch.cuda.current_stream()
    T = args.sweep_tfs
    cases = [
        ("ct_like_512x512x460_u16", lambda: W.make_volume("c2"), 4096, lambda: W.make_tfs("c2", T)),
        ("tube_tree_1024x1024x795_u8", lambda: W.make_volume("c3"), 256, lambda: W.make_tfs("c3", T)),
        ("stag_beetle_832x832x494_u8", lambda: W.stag_beetle_u8(), 256, lambda: W.stag_tfs(T)),
    ]
    ns = [16, 32, 64, 128, 256]

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    points = []
    upd_bytes_total, upd_ms_total = 0.0, 0.0
    for name, make, L, make_tfs in cases:
        log(f"sweep: generating {name} ...")
        host = make()
        rho_min = int(host.min())
        dvol = pdm.to_device(host)
        alphas = make_tfs()
        del host
        for kind in ("uniform", "rho_min"):
            for n in ns:
                bounds = (W.uniform_bounds(L, n) if kind == "uniform"
                          else W.rhomin_bounds(L, n, rho_min))
                v = pdm.Volume(dvol, L, bounds)
                v.build(stream)
                builds = []
                for _ in range(3):
                    a = ev()
                    v.build(stream)
                    b = ev()
                    b.synchronize()
                    builds.append(a.elapsed_time(b))
                d_full = torch.empty_like(v.dist)
                upd, full, sizes, eq, ratio = [], [], [], [], []
                for k, alpha in enumerate(alphas):
                    e0 = ev()
                    mask = v.update_tf(alpha, stream=stream)
                    e1 = ev()
                    v.full_recompute(alpha, out=d_full, stream=stream)
                    e2 = ev()
                    e2.synchronize()
                    upd.append(e0.elapsed_time(e1))
                    full.append(e1.elapsed_time(e2))
                    act = pdm.mask_to_list(mask, v.n)
                    sizes.append(len(act))
                    assert bool((v.dist <= d_full).all().item()), "D' > D"
                    if k < 3:
                        # Eq. 1 against a plain PyTorch min over the active maps
                        want = (v.pdms[act].amin(0) if act else
                                torch.full_like(v.dist, 255))
                        assert torch.equal(v.dist, want), "D' differs from the min over S"
                    eq.append(float((v.dist == d_full).float().mean().item()))
                    df = float(d_full.float().mean().item())
                    ratio.append(float(v.dist.float().mean().item()) / df if df > 0 else 1.0)
                ub = sum((k + 1) * v.G for k in sizes)
                upd_bytes_total += ub
                upd_ms_total += sum(upd)
                points.append({
                    "volume": name, "partition": kind, "n": n, "rho_min": rho_min,
                    "init_ms": round(float(np.median(builds)), 3), "pdm_bytes": n * v.G,
                    "update_p50_ms": round(pct(upd, 50), 4), "update_mean_ms": round(float(np.mean(upd)), 4),
                    "update_GBps": round(ub / (sum(upd) * 1e-3) / 1e9, 1),
                    "mean_active": round(float(np.mean(sizes)), 2),
                    "full_mean_ms": round(float(np.mean(full)), 4),
                    "speedup_mean": round(float(np.mean(full)) / float(np.mean(upd)), 2),
                    "d_equal_frac": round(float(np.mean(eq)), 4),
                    "d_mean_ratio": round(float(np.mean(ratio)), 4)})
                log(json.dumps(points[-1]))
                del v, d_full
                torch.cuda.empty_cache()
        del dvol
        torch.cuda.empty_cache()
    out = {
        "metric": "partition sweep: init ms, PDM bytes, TF-update ms/GB/s and D' retention vs n, "
                  "uniform vs rho_min partition",
        "value": round(upd_bytes_total / (upd_ms_total * 1e-3) / 1e9, 1),
        "unit": "GB/s (TF update, all points)",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u8",
        "data": "synthetic (CT-like u16, tube tree u8, stag-beetle-shaped u8 with background at rho_min)",
        "config": {"workload": f"n in {ns}, uniform and rho_min partitions, {T} TFs per point, bricks 4^3",
                   "tfs": T},
        "points": points,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
