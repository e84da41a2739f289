#!/usr/bin/env python3
"""Benchmark of sketch-based facility location on one MI355X.

A step is one complete facility-location solve (fl_solve: validation, bottom-k
sketches of every vertex, gamma and the radius ladder, the opening loop, MIS
per rung, assignment and objective) of the large weighted workload: R-MAT
2^24 vertices with 268M edge samples, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
weights uniform 1..100, a seeded 10% of the vertices facilities with opening
costs lognormal(5, 1) rounded to integers, every vertex a client, k = 32,
eps = 0.1.  Inputs are generated on the device (seeded) and resident in HBM
before timing.

Printed (one JSON line): edge relaxations per second over whole solves
(sum_v |ADS(v)| deg(v) per solve, divided by the solve time), solves per
second, the HBM roofline of the sketch-round kernel, and the CPU oracle timed
on a bounded sample of the same graph.  Secondary legs in the same line: the
R-MAT 2^22 unit-weight workload (k = 64), batched vs plain solves of 1,024
power-law graphs, a continuous-batching server (capacity, a sustainable
Poisson rate, a saturation sweep and the configured 200 requests/s), and the
directed reading of the R-MAT 2^22 samples.

Measured HBM traffic of the sketch-round kernel comes from two rocprofv3
counter runs of this script with --pmc-calibration (one with FETCH_SIZE, one
with WRITE_SIZE); `--traffic FETCH_DIR WRITE_DIR --profile-workload W` turns
their CSV output into profiles/ads_round_<W>_traffic.json.  Each counter is
scaled by what it reads for a plain 1 GiB device copy (torch.neg on int32) in
the same run.
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
# VALU issue peak: each CU's 4 SIMDs complete one wave64 VALU instruction per
# 4 cycles each, i.e. one per CU per cycle: 256 CUs x 2.4 GHz
VALU_PEAK_INSTS = 256 * 2.4e9
# The sketch-round kernels of one distance round: the two-task kernel (k <=
# 32, rounds run from worklists) and the one-wave kernel that runs after it
# on the tasks it leaves (or on every task).  A "launch" below is one round:
# per-dispatch counters of both are summed and divided by the rounds (the
# one-wave kernel's dispatches).
ROUND_KERNEL = "k_ads_tasks"
ROUND_KERNELS = ("k_ads_tasks", "k_ads_pairs")
ROUND_LABEL = "k_ads_pairs + k_ads_tasks (one distance round)"
CALIB_BYTES = 1 << 30
LARGE = "rmat24_w100_fac10_lognormal_k32"
UNIT = "rmat22_unit_k64"


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


def profile_file(workload, kind):
    return os.path.join(ROOT, "profiles", f"ads_round_{workload}_{kind}.json")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("fl_ads.hip", "fl_ads.h", "fl_common.h"):
        h.update(open(os.path.join(ROOT, "paper_1503_03635_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def write_traffic(fetch_dir, write_dir, workload):
    """Per-launch HBM bytes of the sketch-round kernel from two rocprofv3
    counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the
    counter's reading for the 1 GiB calibration copy of the same run."""
    import csv
    import glob

    def read(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        assert path, f"no counter_collection.csv under {d}"
        calib, total, rounds = [], 0.0, set()
        for row in csv.DictReader(open(path[0])):
            if row["Counter_Name"] != counter:
                continue
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            if "neg_kernel" in name:
                calib.append(val)
            elif any(kn in name for kn in ROUND_KERNELS):
                total += val
                if ROUND_KERNEL in name:
                    rounds.add(row["Dispatch_Id"])
        assert calib and rounds, f"{counter}: calibration copy or {ROUND_KERNEL} missing in {path[0]}"
        return calib[0], total, len(rounds)

    fc, ftot, nr = read(fetch_dir, "FETCH_SIZE")
    wc, wtot, _ = read(write_dir, "WRITE_SIZE")
    f_scale = CALIB_BYTES / (fc * 1024.0)
    w_scale = CALIB_BYTES / (wc * 1024.0)
    fetch = ftot / nr * 1024.0 * f_scale
    write = wtot / nr * 1024.0 * w_scale
    out = {"kernel": ROUND_LABEL, "workload": workload, "kernel_source_hash": kernel_hash(),
           "launches": nr, "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "bytes_per_launch": round(fetch + write),
           "calibration": {"bytes": CALIB_BYTES, "fetch_kib": fc, "write_kib": wc,
                           "fetch_scale": f_scale, "write_scale": w_scale}}
    json.dump(out, open(profile_file(workload, "traffic"), "w"), indent=1)
    print(json.dumps(out))


def write_issue(sq_dir, workload):
    """Per-launch instruction counts of the sketch-round kernel from one
    rocprofv3 counter run (SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS,
    SQ_INSTS_VMEM_RD; wave instructions summed over the chip per dispatch)."""
    import csv
    import glob
    path = glob.glob(os.path.join(sq_dir, "**", "*counter_collection.csv"), recursive=True)
    assert path, f"no counter_collection.csv under {sq_dir}"
    tot, rounds = {}, set()
    for row in csv.DictReader(open(path[0])):
        name = row["Kernel_Name"]
        if not any(kn in name for kn in ROUND_KERNELS):
            continue
        if ROUND_KERNEL in name:
            rounds.add(row["Dispatch_Id"])
        tot[row["Counter_Name"]] = tot.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    assert rounds, f"{ROUND_KERNEL} missing in {path[0]}"
    out = {"kernel": ROUND_LABEL, "workload": workload, "kernel_source_hash": kernel_hash(), "launches": len(rounds)}
    for nm in sorted(tot):
        out[nm.lower() + "_per_launch"] = round(tot[nm] / len(rounds))
    json.dump(out, open(profile_file(workload, "issue"), "w"), indent=1)
    print(json.dumps(out))


def timed_solves(dg, k, eps, seed, warmup, steps, tag):
    """`warmup` untimed solves, then `steps` timed ones bracketed by device
    synchronisation; returns (per-solve stats, elapsed seconds, last result)."""
    import torch
    import paper_1503_03635_amd as fl
    outputs = fl._alloc_outputs(dg.n, dg.col.device, False)
    for i in range(warmup):
        r = fl.solve(dg, k, seed, eps, outputs=outputs)
        log(f"[bench] {tag} warmup {i}: {r['stats']['ms_total']:.1f} ms")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fl.solve(dg, k, seed, eps, outputs=outputs)
        stats.append(dict(r["stats"], total_cost=r["total_cost"], n_open=r["n_open"],
                          n_unreachable=r["n_unreachable"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, s in enumerate(stats):
        log(f"[bench] {tag} step {i}: total {s['ms_total']:.1f} ms | ads {s['ms_ads']:.1f} (kernel "
            f"{s['ms_ads_kernel']:.1f} in {s['ads_kernel_launches']} launches, merges {s['ms_ads_merge']:.1f}, "
            f"{s['ads_rounds']} rounds) | gamma {s['ms_gamma']:.1f} | open {s['ms_open']:.1f} ({s['rungs']} rungs) "
            f"| mis {s['ms_mis']:.1f} ({s['mis_rounds']} rounds) | assign {s['ms_assign']:.1f} | "
            f"open={s['n_open']} cost={s['total_cost']}")
    return stats, elapsed, (r, outputs)


def roofline(stats, arcs, weighted, workload):
    """HBM roofline of the sketch-round kernel.  Algorithmic bytes of a solve's
    sketch rounds: 8 B per relaxation (each final entry read once by each
    neighbour), 8 B per entry written, and one read of the arcs (4 B per arc,
    8 B with weights); per launch they are divided by the solve's launches,
    and `achieved` is that over the average launch duration (HIP events on the
    launch stream).  `traffic` is the measured HBM bytes per launch (committed
    counter runs of the same kernel source, else null)."""
    launches = sum(s["ads_kernel_launches"] for s in stats)
    kern_ms = sum(s["ms_ads_kernel"] for s in stats)
    relax = sum(s["relax_alg"] for s in stats)
    entries = sum(s["ads_entries"] for s in stats)
    alg_bytes = 8.0 * relax + 8.0 * entries + (8.0 if weighted else 4.0) * arcs * len(stats)
    avg_ms = kern_ms / max(launches, 1)
    per_launch = alg_bytes / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    traffic = issue = None
    tf_path, is_path = profile_file(workload, "traffic"), profile_file(workload, "issue")
    if os.path.exists(tf_path):
        try:
            tf = json.load(open(tf_path))
            if tf.get("kernel_source_hash") == kernel_hash():
                traffic = tf.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    if os.path.exists(is_path):
        try:
            isf = json.load(open(is_path))
            if isf.get("kernel_source_hash") == kernel_hash() and "sq_insts_valu_per_launch" in isf:
                rate = isf["sq_insts_valu_per_launch"] / (avg_ms * 1e-3)
                issue = {"valu_insts_per_launch": isf["sq_insts_valu_per_launch"],
                         "valu_insts_per_s": round(rate), "valu_peak_insts_per_s": VALU_PEAK_INSTS,
                         "valu_issue_frac": round(rate / VALU_PEAK_INSTS, 4)}
        except (OSError, ValueError, KeyError):
            issue = None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ROUND_LABEL, "avg_launch_ms": round(avg_ms, 3), "alg_bytes_per_launch": round(per_launch),
            "launches_per_solve": round(launches / len(stats), 1),
            "merge_ms_per_solve": round(sum(s["ms_ads_merge"] for s in stats) / len(stats), 2),
            "measured_hbm_gbs": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1),
            "issue": issue}


def leg_summary(stats, elapsed, dg, workload, extra):
    steps = len(stats)
    s0 = stats[0]
    out = {"workload": workload, "n": dg.n, "arcs": dg.n_arcs, "steps": steps,
           "ms_per_solve": round(elapsed / steps * 1e3, 2),
           "relax_per_s": round(sum(x["relax_alg"] for x in stats) / elapsed, 1),
           "solves_per_s": round(steps / elapsed, 4),
           "ads_entries_per_s": round(sum(x["ads_entries"] for x in stats) / elapsed, 1),
           "relax_alg_per_solve": s0["relax_alg"], "ads_entries_per_solve": s0["ads_entries"],
           "ads_rounds": s0["ads_rounds"], "rungs": s0["rungs"], "mis_rounds": s0["mis_rounds"],
           "phase_ms": {p: round(sum(x[f"ms_{p}"] for x in stats) / steps, 2)
                        for p in ("validate", "ads", "gamma", "open", "mis", "assign", "total")},
           "n_open": s0["n_open"], "n_unreachable": s0["n_unreachable"], "total_cost": s0["total_cost"]}
    out.update(extra)
    return out


def check_large(dg, res):
    """Checks that hold at any size: opened vertices are facilities, every
    served client is assigned to an opened one, and the objective is the
    opening costs plus the assigned distances."""
    import torch
    r, outputs = res
    fac = dg.fac_cost.to(torch.int64) & 0xFFFFFFFF
    is_open = outputs["open"].bool()
    assign = outputs["assign"].to(torch.int64) & 0xFFFFFFFF
    served = assign != 0xFFFFFFFF
    dist = outputs["dist"].to(torch.int64) & 0xFFFFFFFF
    return {"opened_are_facilities": bool((fac[is_open] != 0xFFFFFFFF).all()),
            "served_assigned_to_opened": bool(is_open[assign[served]].all()),
            "total_cost_matches": int(fac[is_open].sum()) + int(dist[served].sum()) == r["total_cost"]}


def cpu_baseline(dg, k, seed, sources, label):
    """The oracle's pruned-Dijkstra sketch construction, single-threaded, from
    the first `sources` sources in rank order of the same graph (host copy)."""
    import graphgen.device as gd
    import oracle as O
    g = gd.to_host(dg)
    t0 = time.perf_counter()
    relax = O.ads_pruned_timed(g, k, seed, sources)
    dt = time.perf_counter() - t0
    return {"value": relax / dt, "unit": "edge-relaxations/s", "cores": 1, "kind": "oracle",
            "sample": f"pruned-Dijkstra sketches from the {sources} lowest-rank sources of the same graph "
                      f"({label}; {relax} relaxations in {dt:.1f} s, 1 thread, {cpu_model()})"}


def batch_leg(count, plain_count, seed):
    """Batched vs plain on power-law graphs: count Chung-Lu graphs (exponent
    2.2, average degree 10, weights 1..20, n log-uniform in [500, 200000]),
    k = 32.  Batched: one fl_solve_batch over all of them (after one untimed
    call); plain: fl_solve one after another on the first plain_count."""
    import torch
    import graphgen.device as gd
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    dgs = gd.powerlaw_batch(count, seed)
    torch.cuda.synchronize()
    n_tot, m_tot = sum(d.n for d in dgs), sum(d.n_arcs for d in dgs)
    log(f"[bench] batch: {count} graphs, sum n {n_tot}, arcs {m_tot} in {time.perf_counter() - t0:.1f}s")
    fl.solve(dgs[0], 32, seed, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in dgs[:plain_count]:
        fl.solve(d, 32, seed, 0.1)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    fl.solve_batch(dgs, 32, seed, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = fl.solve_batch(dgs, 32, seed, 0.1)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    relax = sum(o["stats"]["relax_alg"] for o in outs)
    plain_sps = plain_count / t_plain
    batch_sps = count / t_batch
    log(f"[bench] batch: plain {plain_sps:.2f} solves/s, batched {batch_sps:.2f} solves/s")
    del dgs, outs
    fl.release_workspace()
    torch.cuda.empty_cache()
    return {"workload": f"powerlaw_batch{count}_k32", "graphs": count, "n_total": int(n_tot), "arcs_total": int(m_tot),
            "n_range": [500, 200000], "degree": "Chung-Lu exponent 2.2, average 10", "weights": "1..20",
            "batched_solves_per_s": round(batch_sps, 3), "plain_solves_per_s": round(plain_sps, 3),
            "plain_sample": plain_count, "speedup": round(batch_sps / plain_sps, 2),
            "batched_relax_per_s": round(relax / t_batch, 1), "batched_s": round(t_batch, 3),
            "design": "disjoint unions within a device-memory budget, up to 3 sub-unions at once on worker "
                      "streams; the host drives rungs and MIS steps (not one persistent captured launch)"}


def _serve_point(fl, srv, dgs, arrivals, seed):
    """Submit dgs[i] at arrivals[i] (seconds from now); latency from
    submission to completion per request, and the completion rate."""
    import numpy as np
    count = len(arrivals)
    t_sub = np.zeros(count)
    t_done = np.zeros(count)
    pending = {}
    t0 = time.perf_counter()
    i = 0
    while i < count or pending:
        now = time.perf_counter() - t0
        while i < count and arrivals[i] <= now:
            t_sub[i] = time.perf_counter() - t0
            pending[srv.submit(dgs[i % len(dgs)], 32, seed + i, 0.1)] = i
            i += 1
        for t in list(pending):
            r = srv.poll(t)
            if r is not None:
                j = pending.pop(t)
                t_done[j] = time.perf_counter() - t0
                assert r["status"] == 0, f"request {j} failed: {r['status']}"
        time.sleep(0.0005)
    lat = (t_done - t_sub) * 1e3
    span = t_done.max() - t_sub.min()
    # a burst (every arrival at 0) has no offered rate
    offered = round(count / arrivals[-1], 2) if arrivals[-1] > 0 else None
    return {"requests": count, "offered_per_s": offered,
            "completed_per_s": round(count / span, 3),
            "p50_ms": round(float(np.percentile(lat, 50)), 1), "p99_ms": round(float(np.percentile(lat, 99)), 1)}


def serve_leg(pool, seed, rate, slots, burst, point_s):
    """Continuous batching (Chung-Lu requests, exponent 2.2, average degree 12,
    weights 1..50, n log-uniform in [1000, 500000], k = 32) on a server with a
    200 GB budget: the capacity (a burst of requests submitted at once), p50
    and p99 latency at Poisson arrivals of half the capacity, a saturation
    sweep of rising rates, and the configured rate."""
    import numpy as np
    import torch
    import graphgen.device as gd
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    _, dgs = gd.poisson_requests(pool, seed, rate=rate)
    torch.cuda.synchronize()
    log(f"[bench] serve: pool of {pool} requests, sum n {sum(d.n for d in dgs)} in {time.perf_counter() - t0:.1f}s")
    rng = np.random.Generator(np.random.PCG64(seed + 99))
    out = {"workload": f"poisson_requests_k32", "n_range": [1000, 500000], "degree": "Chung-Lu exponent 2.2, average 12",
           "weights": "1..50", "hbm_budget_gb": 200, "slots": slots, "request_pool": pool}
    with fl.Server(hbm_budget_bytes=200 << 30, slots=slots) as srv:
        srv.wait(srv.submit(dgs[0], 32, seed, 0.1))
        cap = _serve_point(fl, srv, dgs, np.zeros(burst), seed)
        capacity = cap["completed_per_s"]
        out["capacity"] = dict(cap, note="all requests submitted at once")
        log(f"[bench] serve: capacity {capacity:.2f} solves/s")
        sweep = []
        for frac in (0.25, 0.5, 0.75, 1.0, 1.5):
            lam = frac * capacity
            cnt = max(12, int(lam * point_s))
            arr = np.cumsum(rng.exponential(1.0 / lam, size=cnt))
            p = _serve_point(fl, srv, dgs, arr, seed)
            p["rate_frac_of_capacity"] = frac
            sweep.append(p)
            log(f"[bench] serve: lambda {lam:.2f}/s -> {p}")
        out["sweep"] = sweep
        out["sustainable"] = dict(sweep[1], note="Poisson arrivals at half the measured capacity")
        cnt = max(pool, int(rate * point_s / 4))
        arr = np.cumsum(rng.exponential(1.0 / rate, size=cnt))
        cfg = _serve_point(fl, srv, dgs, arr, seed)
        out["configured_rate"] = dict(cfg, rate_per_s=rate,
                                      note="above capacity: latency is queueing in a saturated server")
        log(f"[bench] serve: configured {rate}/s -> {cfg}")
    del dgs
    fl.release_workspace()
    torch.cuda.empty_cache()
    return out


def directed_leg(scale, edge_factor, k, seed, steps):
    """The directed reading (FL_FLAG_DIRECTED) of the R-MAT 2^22 samples: the
    samples kept as arcs, unit weights, k and costs as in the unit workload."""
    import torch
    import graphgen.device as gd
    import paper_1503_03635_amd as fl
    dg = gd.rmat_unit(scale, edge_factor, seed, directed=True)
    torch.cuda.synchronize()
    stats, elapsed, _ = timed_solves(dg, k, 0.1, seed, 1, steps, "directed")
    out = leg_summary(stats, elapsed, dg, f"rmat{scale}_directed_unit_k{k}",
                      {"n_reach_guard": stats[0]["n_reach_guard"]})
    del dg
    fl.release_workspace()
    torch.cuda.empty_cache()
    return out


def mis_compare(seed):
    """Luby's MIS variant against the fixed-priority MIS (the comparison of the
    paper's Tab. 3, on synthetic graphs): MIS rounds and MIS time of full
    solves of R-MAT 2^20 and 2^22 (unit weights, costs 1..1000, k = 32) and
    of Forest Fire graphs (weights 1..100), median of three after one warm-up."""
    import torch
    import graphgen as gg
    import graphgen.device as gd
    import paper_1503_03635_amd as fl

    def point(dg, flags):
        fl.solve(dg, 32, seed, 0.1, flags=flags)
        runs = []
        for _ in range(3):
            r = fl.solve(dg, 32, seed, 0.1, flags=flags)
            torch.cuda.synchronize()
            runs.append(r)
        runs.sort(key=lambda r: r["stats"]["ms_mis"])
        st = runs[1]["stats"]
        return {"mis_rounds": st["mis_rounds"], "ms_mis": round(st["ms_mis"], 1), "n_open": runs[1]["n_open"],
                "cost": runs[1]["total_cost"], "rungs": st["rungs"]}

    rows = []
    for name, make in (("rmat20_unit", lambda: gd.rmat_unit(20, 16, seed)),
                       ("rmat22_unit", lambda: gd.rmat_unit(22, 16, seed)),
                       ("forestfire10k_w1..100", lambda: fl.to_device(gg.with_problem(
                           gg.forest_fire(10000, seed, wmax=100), seed, cost="uniform"), "cuda:0")),
                       ("forestfire20k_w1..100", lambda: fl.to_device(gg.with_problem(
                           gg.forest_fire(20000, seed, wmax=100), seed, cost="uniform"), "cuda:0"))):
        dg = make()
        fixed, luby = point(dg, 0), point(dg, fl.FL_FLAG_LUBY_MIS)
        row = {"graph": name, "n": dg.n, "arcs": dg.n_arcs, "fixed": fixed, "luby": luby,
               "rounds_ratio": round(luby["mis_rounds"] / max(fixed["mis_rounds"], 1), 2),
               "time_ratio": round(luby["ms_mis"] / max(fixed["ms_mis"], 1e-9), 2)}
        log(f"[mis] {row}")
        rows.append(row)
        del dg
        fl.release_workspace()
    return rows


def quality_experiment(seeds):
    """Solution quality (the analogue of the paper's Tab. 2 without its
    comparison system): GPU solve cost over the exact optimum, found here by
    exhaustive search over every non-empty facility subset with distances
    from scipy, on small graphs (n <= 12), for eps in {0.01, 0.1, 1} and
    k in {1, 4, n}."""
    import itertools
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    import graphgen as gg
    import paper_1503_03635_amd as fl

    def opt(g):
        w = g.w if g.w is not None else np.ones(g.n_arcs, np.uint32)
        A = sp.csr_matrix((w.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                          shape=(g.n, g.n))
        D = dijkstra(A, directed=True)
        F = np.nonzero(g.fac_cost != gg.NOT_FACILITY)[0]
        served = np.isfinite(D[:, F]).any(axis=1)
        best = None
        for r in range(1, len(F) + 1):
            for S in itertools.combinations(F, r):
                d = D[np.ix_(served, list(S))].min(axis=1)
                if not np.isfinite(d).all():
                    continue
                c = int(g.fac_cost[list(S)].astype(np.int64).sum()) + int(d.sum())
                best = c if best is None else min(best, c)
        return best

    table = {}
    for eps in (0.01, 0.1, 1.0):
        for kk in ("1", "4", "n"):
            ratios = []
            for seed in seeds:
                n = 8 + seed % 5
                g = gg.with_problem(gg.er(n, 3, seed, wmax=6), seed, cost="uniform", cost_lo=1, cost_hi=25)
                k = n if kk == "n" else int(kk)
                r = fl.solve(fl.to_device(g, "cuda:0"), k, seed, eps)
                o = opt(g)
                if o:
                    ratios.append(r["total_cost"] / o)
            a = np.array(ratios)
            table[f"eps{eps}_k{kk}"] = {"graphs": len(a), "mean": round(float(a.mean()), 4),
                                        "median": round(float(np.median(a)), 4), "max": round(float(a.max()), 4),
                                        "frac_optimal": round(float((a <= 1.0 + 1e-12).mean()), 3)}
            log(f"[quality] eps={eps} k={kk}: {table[f'eps{eps}_k{kk}']}")
    return table


def accuracy_experiment(ks, samples, seed):
    """HIP-estimator accuracy (the protocol of Sec. 5.1): for sampled vertices
    v and distances d, the relative error |N(v,d) - |B(v,d)|| / |B(v,d)| of the
    estimate from the GPU sketches, against exact ball sizes from scipy's
    Dijkstra.  Unweighted graphs use d = 1..20, weighted (1..100) graphs
    d = 100..2000 step 100, as in the paper's figures."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl
    cases = [("rmat14_unit", lambda: gg.rmat(14, 16 << 14, seed), list(range(1, 21))),
             ("rmat14_w1..100", lambda: gg.rmat(14, 16 << 14, seed, wmax=100), list(range(100, 2001, 100))),
             ("forestfire8k_unit", lambda: gg.forest_fire(8000, seed), list(range(1, 21))),
             ("forestfire8k_w1..100", lambda: gg.forest_fire(8000, seed, wmax=100), list(range(100, 2001, 100)))]
    out = {}
    rng = np.random.Generator(np.random.PCG64(seed))
    for name, make, dists in cases:
        g = make()
        w = g.w if g.w is not None else np.ones(g.n_arcs, np.uint32)
        A = sp.csr_matrix((w.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                          shape=(g.n, g.n))
        deg = g.degrees()
        cand = np.nonzero(deg > 0)[0]
        vs = rng.choice(cand, size=min(samples, len(cand)), replace=False)
        D = dijkstra(A, directed=True, indices=vs)
        exact = np.array([[np.count_nonzero(D[i] <= d) for d in dists] for i in range(len(vs))], np.float64)
        dg = fl.to_device(g, "cuda:0")
        res = {}
        for k in ks:
            s = fl.ads_build(dg, k, seed)
            torch.cuda.synchronize()
            off = s["off"].cpu().numpy().view(np.uint64).astype(np.int64)
            dist = s["dist"].cpu().numpy().view(np.uint32).astype(np.float64)
            thr = s["thresh"].cpu().numpy().view(np.uint32).astype(np.float64)
            a = np.where(thr == 0, 1.0, 4294967296.0 / np.maximum(thr, 1.0))
            est = np.zeros_like(exact)
            for i, v in enumerate(vs):
                dv, av = dist[off[v]:off[v + 1]], a[off[v]:off[v + 1]]
                for j, d in enumerate(dists):
                    est[i, j] = av[dv <= d].sum()
            rel = np.abs(est - exact) / exact
            res[f"k{k}"] = {"mean_rel_err": round(float(rel.mean()), 4),
                            "max_rel_err": round(float(rel.max()), 4),
                            "mean_rel_err_by_d": [round(float(x), 4) for x in rel.mean(axis=0)]}
            log(f"[accuracy] {name} k={k}: mean relative error {rel.mean():.4f}")
        out[name] = {"n": g.n, "arcs": g.n_arcs, "samples": int(len(vs)), "distances": dists, "by_k": res}
    return out


def sweep_experiment(seed):
    """Time vs k and vs eps (the paper's Fig. 3 and Fig. 4 on synthetic
    graphs): full solves of R-MAT 2^20 (16 edge samples per vertex, unit
    weights, costs 1..1000) for k in {16, 32, 64, 128} at eps = 0.1 and for eps in
    {0.01, 0.1, 1} at k = 32, and the same eps sweep on a Forest Fire graph
    (n = 20,000, weights 1..100).  Each point: one untimed solve, then the
    median of three."""
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl

    def point(dg, k, eps):
        fl.solve(dg, k, seed, eps)
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            r = fl.solve(dg, k, seed, eps)
            torch.cuda.synchronize()
            runs.append(r)
        runs.sort(key=lambda r: r["stats"]["ms_total"])
        st = runs[1]["stats"]
        return {"k": k, "eps": eps, "ms_total": round(st["ms_total"], 1), "ms_ads": round(st["ms_ads"], 1),
                "ms_open": round(st["ms_open"], 1), "ms_mis": round(st["ms_mis"], 1), "rungs": st["rungs"],
                "mis_rounds": st["mis_rounds"], "n_open": runs[1]["n_open"], "cost": runs[1]["total_cost"],
                "ads_entries": st["ads_entries"], "relax_alg": st["relax_alg"]}

    out = {}
    g = gg.rmat_unit(20, 16, seed)
    dg = fl.to_device(g, "cuda:0")
    out["rmat20_unit"] = {"n": g.n, "arcs": g.n_arcs,
                          "k_sweep": [point(dg, k, 0.1) for k in (16, 32, 64, 128)],
                          "eps_sweep": [point(dg, 32, e) for e in (0.01, 0.1, 1.0)]}
    log(f"[sweep] rmat20: {out['rmat20_unit']}")
    g = gg.with_problem(gg.forest_fire(20000, seed, wmax=100), seed, cost="uniform")
    dg = fl.to_device(g, "cuda:0")
    out["forestfire20k_w1..100"] = {"n": g.n, "arcs": g.n_arcs,
                                    "eps_sweep": [point(dg, 32, e) for e in (0.01, 0.1, 1.0)]}
    log(f"[sweep] forest fire: {out['forestfire20k_w1..100']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sources", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="unit,batched,serving,directed",
                    help="secondary legs, comma separated (unit, batched, serving, directed) or 'none'")
    ap.add_argument("--headline", choices=("large", "unit"), default="large",
                    help="workload of the timed steps (default: the large weighted one)")
    ap.add_argument("--unit-steps", type=int, default=3)
    ap.add_argument("--batch-count", type=int, default=1024, help="graphs of the batched measurement")
    ap.add_argument("--batch-plain", type=int, default=32, help="of them solved one by one for the plain rate")
    ap.add_argument("--serve-pool", type=int, default=64, help="distinct request graphs of the serving legs")
    ap.add_argument("--serve-burst", type=int, default=48, help="requests of the capacity measurement")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-point-s", type=float, default=4.0, help="seconds of arrivals per sweep point")
    ap.add_argument("--directed-steps", type=int, default=2)
    ap.add_argument("--sweep", action="store_true", help="run the k and eps sweeps instead and print their JSON")
    ap.add_argument("--accuracy", action="store_true",
                    help="run the HIP-estimator accuracy experiment instead and print its JSON")
    ap.add_argument("--mis-compare", action="store_true",
                    help="run Luby's MIS against the fixed-priority MIS instead and print their JSON")
    ap.add_argument("--quality", action="store_true",
                    help="run the cost / exhaustive optimum experiment instead and print its JSON")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--profile-workload", default=LARGE, help="workload the counter files describe")
    ap.add_argument("--issue", metavar="SQ_DIR",
                    help="write the instruction-count file from a rocprofv3 SQ counter run and exit")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the measured traffic file from two rocprofv3 counter runs and exit")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic, args.profile_workload)
        return
    if args.issue:
        write_issue(args.issue, args.profile_workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"sharding of this method is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        print(json.dumps({"sweep": sweep_experiment(args.seed)}), flush=True)
        return
    if args.accuracy:
        print(json.dumps({"accuracy": accuracy_experiment([4, 8, 16, 32, 64], 100, args.seed)}), flush=True)
        return
    if args.mis_compare:
        print(json.dumps({"mis_compare": mis_compare(args.seed)}), flush=True)
        return
    if args.quality:
        print(json.dumps({"quality": quality_experiment(list(range(1, 41)))}), flush=True)
        return

    import torch
    import graphgen.device as gd
    import paper_1503_03635_amd as fl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    legs = set() if args.legs == "none" else set(args.legs.split(","))
    if args.pmc_calibration:
        x = torch.ones(CALIB_BYTES // 4, dtype=torch.int32, device="cuda:0")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y

    # ---- the timed workload
    t0 = time.perf_counter()
    if args.headline == "large":
        workload, k, weighted = LARGE, 32, True
        dg = gd.rmat_weighted_fac10(24, 32, args.seed)
        cfg = {"workload": LARGE, "edge_samples": 16 << 24, "rmat": [0.57, 0.19, 0.19, 0.05], "weights": "1..100",
               "facilities": "seeded 10% of the vertices, costs lognormal(5, 1) rounded", "clients": "every vertex"}
    else:
        workload, k, weighted = UNIT, 64, False
        dg = gd.rmat_unit(22, 16, args.seed)
        cfg = {"workload": UNIT, "edge_samples": 16 << 22, "rmat": [0.57, 0.19, 0.19, 0.05], "weights": "unit",
               "facilities": "every vertex, costs uniform 1..1000", "clients": "every vertex"}
    torch.cuda.synchronize()
    log(f"[bench] {workload}: n={dg.n} arcs={dg.n_arcs} generated on the device in {time.perf_counter() - t0:.1f}s")
    stats, elapsed, res = timed_solves(dg, k, 0.1, args.seed, args.warmup, args.steps, workload)
    relax = sum(s["relax_alg"] for s in stats)
    entries = sum(s["ads_entries"] for s in stats)
    cfg.update({"n": dg.n, "arcs": dg.n_arcs, "k": k, "eps": 0.1, "seed": args.seed,
                "generator": "seeded, on the device (torch Philox)", "parallelism": "single GPU"})
    out = {
        "metric": METRIC, "value": round(relax / elapsed, 1), "unit": "edge-relaxations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic", "config": cfg,
        "solves_per_s": round(args.steps / elapsed, 4),
        "ads_entries_per_s": round(entries / elapsed, 1),
        "ads_relax_per_s_ads_phase": round(relax / (sum(s["ms_ads"] for s in stats) * 1e-3), 1),
        "relax_alg_per_solve": stats[0]["relax_alg"], "ads_entries_per_solve": stats[0]["ads_entries"],
        "ads_rounds": stats[0]["ads_rounds"], "rungs": stats[0]["rungs"], "mis_rounds": stats[0]["mis_rounds"],
        "n_open": stats[0]["n_open"], "total_cost": stats[0]["total_cost"],
        "phase_ms": {p: round(sum(s[f"ms_{p}"] for s in stats) / args.steps, 2)
                     for p in ("validate", "ads", "gamma", "open", "mis", "assign", "total")},
        "roofline": roofline(stats, dg.n_arcs, weighted, workload),
    }
    if args.headline == "large":
        out["checks"] = check_large(dg, res)
        log(f"[bench] checks {out['checks']}")
    del res
    fl.release_workspace()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(dg, k, args.seed, args.cpu_sources, workload)
    else:
        out["cpu_baseline"] = None
    del dg
    torch.cuda.empty_cache()

    # ---- secondary legs
    if "unit" in legs and args.headline == "large":
        dgu = gd.rmat_unit(22, 16, args.seed)
        torch.cuda.synchronize()
        st, el, _ = timed_solves(dgu, 64, 0.1, args.seed, 1, args.unit_steps, UNIT)
        out[UNIT] = leg_summary(st, el, dgu, UNIT, {"roofline": roofline(st, dgu.n_arcs, False, UNIT)})
        del dgu
        fl.release_workspace()
        torch.cuda.empty_cache()
    if "batched" in legs:
        out["batched"] = batch_leg(args.batch_count, min(args.batch_plain, args.batch_count), args.seed)
    if "serving" in legs:
        out["serving"] = serve_leg(args.serve_pool, args.seed, args.serve_rate, args.serve_slots, args.serve_burst,
                                   args.serve_point_s)
    if "directed" in legs:
        out["directed"] = directed_leg(22, 16, 64, args.seed, args.directed_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
