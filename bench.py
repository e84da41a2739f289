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
ISSUE_FILE = os.path.join(ROOT, "profiles", "ads_round_rmat22_issue.json")
# VALU issue peak: each CU's 4 SIMDs complete one wave64 VALU instruction per
# 4 cycles each, i.e. one per CU per cycle: 256 CUs x 2.4 GHz
VALU_PEAK_INSTS = 256 * 2.4e9
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


def write_issue(sq_dir):
    """Per-launch instruction counts of the sketch-round kernel from one
    rocprofv3 counter run (SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS,
    SQ_INSTS_VMEM_RD; wave instructions summed over the chip per dispatch)."""
    import csv
    import glob
    path = glob.glob(os.path.join(sq_dir, "**", "*counter_collection.csv"), recursive=True)
    assert path, f"no counter_collection.csv under {sq_dir}"
    per = {}
    for row in csv.DictReader(open(path[0])):
        if ROUND_KERNEL not in row["Kernel_Name"]:
            continue
        d = per.setdefault(row["Dispatch_Id"], {})
        d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    assert per, f"{ROUND_KERNEL} missing in {path[0]}"
    names = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD")
    out = {"kernel": ROUND_KERNEL, "kernel_source_hash": kernel_hash(), "launches": len(per)}
    for nm in names:
        out[nm.lower() + "_per_launch"] = round(sum(d.get(nm, 0.0) for d in per.values()) / len(per))
    json.dump(out, open(ISSUE_FILE, "w"), indent=1)
    print(json.dumps(out))


def batch_bench(count, plain_count, seed):
    """Batched vs plain on power-law graphs: count Chung-Lu graphs (exponent
    2.2, average degree 10, weights 1..20, n log-uniform in [500, 200000]),
    k = 32.  Batched: one fl_solve_batch over all of them (after one untimed
    call); plain: fl_solve one after another on the first plain_count."""
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    graphs = gg.powerlaw_batch(count, seed)
    dgs = [fl.to_device(g, "cuda:0") for g in graphs]
    torch.cuda.synchronize()
    log(f"[bench] batch: {count} graphs, sum n {sum(g.n for g in graphs)} in {time.perf_counter() - t0:.1f}s")
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
    return {"workload": f"powerlaw_batch{count}_k32", "graphs": count,
            "n_total": int(sum(g.n for g in graphs)), "arcs_total": int(sum(g.n_arcs for g in graphs)),
            "n_range": [500, 200000], "degree": "Chung-Lu exponent 2.2, average 10", "weights": "1..20",
            "batched_solves_per_s": round(batch_sps, 3), "plain_solves_per_s": round(plain_sps, 3),
            "plain_sample": plain_count, "speedup": round(batch_sps / plain_sps, 2),
            "batched_relax_per_s": round(relax / t_batch, 1), "batched_s": round(t_batch, 3)}


def directed_bench(scale, edge_factor, k, seed, steps):
    """The directed reading (FL_FLAG_DIRECTED): the R-MAT samples of the main
    workload kept as arcs, unit weights, k and costs as there.  One untimed
    solve, then `steps` timed ones."""
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    g = gg.rmat_unit_directed(scale, edge_factor, seed)
    dg = fl.to_device(g, "cuda:0")
    torch.cuda.synchronize()
    log(f"[bench] directed R-MAT 2^{scale}: n={g.n} arcs={g.n_arcs} in {time.perf_counter() - t0:.1f}s")
    outputs = fl._alloc_outputs(g.n, dg.col.device, False)
    r = fl.solve(dg, k, seed, 0.1, outputs=outputs)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fl.solve(dg, k, seed, 0.1, outputs=outputs)
        stats.append(dict(r["stats"], total_cost=r["total_cost"], n_open=r["n_open"],
                          n_unreachable=r["n_unreachable"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s0 = stats[0]
    log(f"[bench] directed: {elapsed / steps * 1e3:.1f} ms per solve, open={s0['n_open']} "
        f"unreachable={s0['n_unreachable']} reach_guard={s0['n_reach_guard']}")
    return {"workload": f"rmat{scale}_directed_unit_k{k}", "n": g.n, "arcs": g.n_arcs,
            "edge_samples": edge_factor << scale, "steps": steps,
            "ms_per_solve": round(elapsed / steps * 1e3, 2),
            "relax_per_s": round(sum(x["relax_alg"] for x in stats) / elapsed, 1),
            "relax_alg_per_solve": s0["relax_alg"], "ads_entries_per_solve": s0["ads_entries"],
            "phase_ms": {p: round(sum(x[f"ms_{p}"] for x in stats) / steps, 2)
                         for p in ("validate", "ads", "gamma", "open", "mis", "assign", "total")},
            "n_open": s0["n_open"], "n_unreachable": s0["n_unreachable"],
            "n_reach_guard": s0["n_reach_guard"]}


def large_bench(scale, edge_factor, k, seed, steps):
    """The large single-graph configuration: R-MAT 2^scale with
    edge_factor * 2^scale samples, weights 1..100, 10% of the vertices
    facilities with lognormal(5, 1) costs, every vertex a client, k as given.
    One untimed solve, then `steps` timed ones, and checks of the result that
    hold at any size: opened vertices are facilities, every served client is
    assigned to an opened one, and the total cost is the opening costs plus the
    assigned distances."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    g = gg.rmat_weighted_fac10(scale, edge_factor, seed)
    dg = fl.to_device(g, "cuda:0")
    torch.cuda.synchronize()
    log(f"[bench] large R-MAT 2^{scale} w1..100: n={g.n} arcs={g.n_arcs} in {time.perf_counter() - t0:.1f}s")
    outputs = fl._alloc_outputs(g.n, dg.col.device, False)
    t0 = time.perf_counter()
    r = fl.solve(dg, k, seed, 0.1, outputs=outputs)
    torch.cuda.synchronize()
    log(f"[bench] large: untimed solve {time.perf_counter() - t0:.1f}s")
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fl.solve(dg, k, seed, 0.1, outputs=outputs)
        stats.append(r["stats"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dev = outputs["open"].device
    fac = torch.from_numpy(g.fac_cost.astype(np.int64)).to(dev)
    is_open = outputs["open"].bool()
    assign = outputs["assign"].to(torch.int64) & 0xFFFFFFFF
    served = assign != 0xFFFFFFFF
    dist = outputs["dist"].to(torch.int64) & 0xFFFFFFFF
    checks = {
        "opened_are_facilities": bool((fac[is_open] != 0xFFFFFFFF).all()),
        "served_assigned_to_opened": bool(is_open[assign[served]].all()),
        "total_cost_matches": int(fac[is_open].sum()) + int(dist[served].sum()) == r["total_cost"],
    }
    s0 = stats[0]
    log(f"[bench] large: {elapsed / steps * 1e3:.1f} ms per solve, open={r['n_open']} checks={checks}")
    return {"workload": f"rmat{scale}_w100_fac10_lognormal_k{k}", "n": g.n, "arcs": g.n_arcs,
            "edge_samples": edge_factor << scale, "steps": steps,
            "ms_per_solve": round(elapsed / steps * 1e3, 2),
            "relax_per_s": round(sum(x["relax_alg"] for x in stats) / elapsed, 1),
            "relax_alg_per_solve": s0["relax_alg"], "ads_entries_per_solve": s0["ads_entries"],
            "ads_rounds": s0["ads_rounds"], "rungs": s0["rungs"], "mis_rounds": s0["mis_rounds"],
            "phase_ms": {p: round(sum(x[f"ms_{p}"] for x in stats) / steps, 2)
                         for p in ("validate", "ads", "gamma", "open", "mis", "assign", "total")},
            "n_open": r["n_open"], "n_unreachable": r["n_unreachable"], "total_cost": r["total_cost"],
            "checks": checks}


def serve_bench(count, seed, rate, slots):
    """Continuous batching: a Poisson stream of count requests at `rate`
    requests/s (Chung-Lu graphs, exponent 2.2, average degree 12, weights
    1..50, n log-uniform in [1000, 500000], k = 32) submitted to a server with
    a 200 GB budget; latency from submission to completion."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_03635_amd as fl
    t0 = time.perf_counter()
    arrivals, graphs = gg.poisson_requests(count, seed, rate=rate)
    dgs = [fl.to_device(g, "cuda:0") for g in graphs]
    torch.cuda.synchronize()
    log(f"[bench] serve: {count} requests, sum n {sum(g.n for g in graphs)} in {time.perf_counter() - t0:.1f}s")
    with fl.Server(hbm_budget_bytes=200 << 30, slots=slots) as srv:
        srv.wait(srv.submit(dgs[0], 32, seed, 0.1))
        t_sub = np.zeros(count)
        t_done = np.zeros(count)
        tickets = []
        pending = {}
        t0 = time.perf_counter()
        i = 0
        while i < count or pending:
            now = time.perf_counter() - t0
            while i < count and arrivals[i] <= now:
                t_sub[i] = time.perf_counter() - t0
                pending[srv.submit(dgs[i], 32, seed + i, 0.1)] = i
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
    log(f"[bench] serve: p50 {np.percentile(lat, 50):.0f} ms, p99 {np.percentile(lat, 99):.0f} ms, "
        f"{count / span:.2f} solves/s")
    return {"workload": f"poisson{int(rate)}_requests{count}_k32", "requests": count, "rate_per_s": rate,
            "n_range": [1000, 500000], "degree": "Chung-Lu exponent 2.2, average 12", "weights": "1..50",
            "hbm_budget_gb": 200, "slots": slots,
            "p50_ms": round(float(np.percentile(lat, 50)), 1), "p99_ms": round(float(np.percentile(lat, 99)), 1),
            "solves_per_s": round(count / span, 3), "offered_per_s": rate}


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
    weights, costs 1..1000) for k in {16, 32, 64} at eps = 0.1 and for eps in
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
                          "k_sweep": [point(dg, k, 0.1) for k in (16, 32, 64)],
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
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sources", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-count", type=int, default=128, help="graphs of the batched measurement (0: skip)")
    ap.add_argument("--batch-plain", type=int, default=32, help="of them solved one by one for the plain rate")
    ap.add_argument("--serve-count", type=int, default=64, help="requests of the serving measurement (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--directed-steps", type=int, default=2,
                    help="timed solves of the directed reading of the same R-MAT samples (0: skip)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the k and eps sweeps instead and print their JSON")
    ap.add_argument("--large", action="store_true",
                    help="run the large weighted configuration (R-MAT 2^24, weights 1..100, 10%% facilities, "
                         "k = 32) instead and print its JSON")
    ap.add_argument("--large-steps", type=int, default=1)
    ap.add_argument("--accuracy", action="store_true",
                    help="run the HIP-estimator accuracy experiment instead and print its JSON")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--issue", metavar="SQ_DIR",
                    help="write the instruction-count file from a rocprofv3 SQ counter run and exit")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the measured traffic file from two rocprofv3 counter runs and exit")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic)
        return
    if args.issue:
        write_issue(args.issue)
        return
    if args.sweep:
        print(json.dumps({"sweep": sweep_experiment(args.seed)}), flush=True)
        return
    if args.large:
        print(json.dumps({"large": large_bench(24, 16, 32, args.seed, args.large_steps)}), flush=True)
        return
    if args.accuracy:
        print(json.dumps({"accuracy": accuracy_experiment([4, 8, 16, 32, 64], 100, args.seed)}), flush=True)
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
    # the kernel's own limit, from committed counters: VALU wave instructions
    # per launch over the average launch time, against the issue peak
    issue = None
    if os.path.exists(ISSUE_FILE):
        try:
            isf = json.load(open(ISSUE_FILE))
            if isf.get("kernel_source_hash") == kernel_hash():
                rate = isf["sq_insts_valu_per_launch"] / (kern_ms / max(launches, 1) * 1e-3)
                issue = {"valu_insts_per_launch": isf["sq_insts_valu_per_launch"],
                         "valu_insts_per_s": round(rate), "valu_peak_insts_per_s": VALU_PEAK_INSTS,
                         "valu_issue_frac": round(rate / VALU_PEAK_INSTS, 4)}
        except (OSError, ValueError, KeyError):
            issue = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ROUND_KERNEL, "avg_launch_ms": round(kern_ms / max(launches, 1), 3),
            "alg_bytes_per_launch": round(alg_bytes / max(launches, 1)),
            "merge_ms_per_step": round(sum(s["ms_ads_merge"] for s in stats) / args.steps, 2),
            "issue": issue}
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
    if args.batch_count:
        out["batched"] = batch_bench(args.batch_count, min(args.batch_plain, args.batch_count), args.seed)
    if args.serve_count:
        out["serving"] = serve_bench(args.serve_count, args.seed, args.serve_rate, args.serve_slots)
    if args.directed_steps:
        del dg, outputs
        torch.cuda.empty_cache()
        out["directed"] = directed_bench(args.scale, args.edge_factor, args.k, args.seed, args.directed_steps)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, args.k, args.seed, args.cpu_sources)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
