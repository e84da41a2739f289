#!/usr/bin/env python3
"""Benchmark of sketch-based facility location on one MI355X.

A step is one complete facility-location solve (fl_solve: validation, bottom-k
sketches of every vertex, gamma and the radius ladder, the opening loop, MIS
per rung, assignment and objective) on a synthetic R-MAT graph:
2^22 vertices, 64M edge samples with (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
unit weights, every vertex a client and a facility with opening cost uniform
in 1..1000, k = 64, eps = 0.1.  Inputs are resident in HBM before timing.

Printed (one JSON line): edge relaxations per second over whole solves
(sum_v |ADS(v)| deg(v) per solve, divided by the solve time), solves per
second, the HBM roofline of the sketch-round kernel, and the CPU oracle timed
on a bounded sample of the same graph.

Measured HBM traffic of the sketch-round kernel comes from two rocprofv3
counter runs of this script with --pmc-calibration (one with FETCH_SIZE, one
with WRITE_SIZE); `--traffic FETCH_DIR WRITE_DIR` turns their CSV output into
profiles/ads_round_rmat22_traffic.json.  Each counter is scaled by what it
reads for a plain 1 GiB device copy (torch.neg on int32) in the same run.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ADS edge-relaxations/s + facility-location solves/s, batched vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ads_round_rmat22_traffic.json")
ROUND_KERNEL = "k_ads_tasks"
CALIB_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(g, k, seed, sources):
    """The oracle's pruned-Dijkstra sketch construction, single-threaded, on the
    first `sources` sources in rank order of the same graph."""
    import oracle as O
    t0 = time.perf_counter()
    relax = O.ads_pruned_timed(g, k, seed, sources)
    dt = time.perf_counter() - t0
    return {"value": relax / dt, "unit": "edge-relaxations/s", "cores": 1, "kind": "oracle",
            "sample": f"pruned-Dijkstra sketches from the {sources} lowest-rank sources of the same "
                      f"graph ({relax} relaxations in {dt:.1f} s, 1 thread, {cpu_model()})"}


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("fl_ads.hip", "fl_ads.h", "fl_common.h"):
        h.update(open(os.path.join(ROOT, "paper_1503_03635_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def write_traffic(fetch_dir, write_dir):
    """Per-launch HBM bytes of the sketch-round kernel from two rocprofv3
    counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the
    counter's reading for the 1 GiB calibration copy of the same run."""
    import csv
    import glob

    def read(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        assert path, f"no counter_collection.csv under {d}"
        calib, launches = [], {}
        for row in csv.DictReader(open(path[0])):
            if row["Counter_Name"] != counter:
                continue
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            if "neg_kernel" in name:
                calib.append(val)
            elif ROUND_KERNEL in name:
                launches[row["Dispatch_Id"]] = launches.get(row["Dispatch_Id"], 0.0) + val
        assert calib and launches, f"{counter}: calibration copy or {ROUND_KERNEL} missing in {path[0]}"
        return calib[0], launches

    fc, fl_ = read(fetch_dir, "FETCH_SIZE")
    wc, wl = read(write_dir, "WRITE_SIZE")
    f_scale = CALIB_BYTES / (fc * 1024.0)
    w_scale = CALIB_BYTES / (wc * 1024.0)
    fetch = sum(fl_.values()) / len(fl_) * 1024.0 * f_scale
    write = sum(wl.values()) / len(wl) * 1024.0 * w_scale
    out = {"kernel": ROUND_KERNEL, "kernel_source_hash": kernel_hash(), "launches": len(fl_),
           "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "bytes_per_launch": round(fetch + write),
           "calibration": {"bytes": CALIB_BYTES, "fetch_kib": fc, "write_kib": wc,
                           "fetch_scale": f_scale, "write_scale": w_scale}}
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sources", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the measured traffic file from two rocprofv3 counter runs and exit")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"sharding of this method is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1503_03635_amd as fl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    g = gg.rmat_unit(args.scale, args.edge_factor, args.seed)
    log(f"[bench] generated R-MAT 2^{args.scale}: n={g.n} arcs={g.n_arcs} in {time.perf_counter() - t0:.1f}s")
    dg = fl.to_device(g, "cuda:0")
    torch.cuda.synchronize()
    if args.pmc_calibration:
        x = torch.ones(CALIB_BYTES // 4, dtype=torch.int32, device="cuda:0")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    outputs = fl._alloc_outputs(g.n, dg.col.device, False)

    for i in range(args.warmup):
        r = fl.solve(dg, args.k, args.seed, args.eps, outputs=outputs)
        log(f"[bench] warmup {i}: {r['stats']['ms_total']:.1f} ms")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = fl.solve(dg, args.k, args.seed, args.eps, outputs=outputs)
        stats.append(dict(r["stats"], total_cost=r["total_cost"], n_open=r["n_open"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, s in enumerate(stats):
        log(f"[bench] step {i}: total {s['ms_total']:.1f} ms | ads {s['ms_ads']:.1f} (kernel "
            f"{s['ms_ads_kernel']:.1f} in {s['ads_kernel_launches']} launches, {s['ads_rounds']} rounds) | "
            f"gamma {s['ms_gamma']:.1f} | open {s['ms_open']:.1f} ({s['rungs']} rungs) | mis "
            f"{s['ms_mis']:.1f} ({s['mis_rounds']} rounds) | assign {s['ms_assign']:.1f} | "
            f"open={s['n_open']} cost={s['total_cost']}")

    relax = sum(s["relax_alg"] for s in stats)
    entries = sum(s["ads_entries"] for s in stats)
    ms_per_step = elapsed / args.steps * 1e3
    value = relax / elapsed
    kern_ms = sum(s["ms_ads_kernel"] for s in stats)
    launches = sum(s["ads_kernel_launches"] for s in stats)
    # algorithmic bytes of the sketch rounds: 8 B per relaxation (each final
    # entry read once per neighbour) + 8 B per entry written, over the summed
    # duration of the round-kernel launches (HIP events on the launch stream)
    alg_bytes = 8.0 * relax + 8.0 * entries
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tf = json.load(open(TRAFFIC_FILE))
            if tf.get("kernel_source_hash") == kernel_hash():
                traffic = tf.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ROUND_KERNEL, "avg_launch_ms": round(kern_ms / max(launches, 1), 3),
            "alg_bytes_per_launch": round(alg_bytes / max(launches, 1)),
            "merge_ms_per_step": round(sum(s["ms_ads_merge"] for s in stats) / args.steps, 2)}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "edge-relaxations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_unit_k{args.k}", "n": g.n, "arcs": g.n_arcs,
                   "edge_samples": args.edge_factor << args.scale, "rmat": [0.57, 0.19, 0.19, 0.05],
                   "k": args.k, "eps": args.eps, "seed": args.seed, "costs": "uniform 1..1000",
                   "parallelism": "single GPU"},
        "solves_per_s": round(args.steps / elapsed, 4),
        "ads_entries_per_s": round(entries / elapsed, 1),
        "ads_relax_per_s_ads_phase": round(relax / (sum(s["ms_ads"] for s in stats) * 1e-3), 1),
        "relax_alg_per_solve": stats[0]["relax_alg"], "ads_entries_per_solve": stats[0]["ads_entries"],
        "phase_ms": {p: round(sum(s[f"ms_{p}"] for s in stats) / args.steps, 2)
                     for p in ("validate", "ads", "gamma", "open", "mis", "assign", "total")},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, args.k, args.seed, args.cpu_sources)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
