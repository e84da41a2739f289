"""GPU: the continuous-batching server.  Requests submitted from several
threads at uneven times, admitted into groups as workers and memory free up,
each give exactly the result of fl_solve on the same request alone."""
import random
import threading
import time

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1503_03635_amd as fl

from gpu_util import host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    fl.lib()


def _h(r):
    return {"open": host(r["open"], np.uint8), "assign": u32(r["assign"]), "dist": u32(r["dist"]),
            "open_rung": u32(r["open_rung"]), "freeze_rung": u32(r["freeze_rung"]),
            "q": host(r["q"], np.float64).view(np.uint64), "total_cost": r["total_cost"],
            "n_open": r["n_open"], "status": r["status"], "rungs": r["stats"]["rungs"],
            "mis_rounds": r["stats"]["mis_rounds"]}


def _same(a, b, what):
    for key in a:
        if isinstance(a[key], np.ndarray):
            assert np.array_equal(a[key], b[key]), f"{what}: {key}"
        else:
            assert a[key] == b[key], f"{what}: {key} {a[key]} vs {b[key]}"


def _requests():
    graphs = gg.powerlaw_batch(10, 21, n_lo=200, n_hi=4000, avg_deg=8.0, wmax=20)
    graphs.append(gg.with_problem(gg.rmat(10, 8 << 10, 3), 3, cost="uniform"))
    graphs.append(gg.with_problem(gg.er(300, 5, 4, wmax=10), 4, cost="uniform", cost_hi=200,
                                  client_frac=0.5))
    ks = [8, 16, 8, 8, 16, 8, 32, 8, 16, 8, 8, 16]
    return [(fl.to_device(g), ks[i], 100 + i) for i, g in enumerate(graphs)]


def test_server_results_equal_single_solves():
    reqs = _requests()
    alone = []
    for dg, k, sd in reqs:
        r = fl.solve(dg, k, sd, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        alone.append(_h(r))
    print(f"[server] {len(reqs)} requests, 3 slots, 2 submitting threads", flush=True)
    tickets = [None] * len(reqs)
    with fl.Server(hbm_budget_bytes=8 << 30, slots=3) as srv:
        def submitter(idx):
            rng = random.Random(idx[0])
            for i in idx:
                time.sleep(rng.uniform(0, 0.02))
                dg, k, sd = reqs[i]
                tickets[i] = srv.submit(dg, k, sd, 0.1, diagnostics=True)
        th = [threading.Thread(target=submitter, args=(list(range(j, len(reqs), 2)),)) for j in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = [None] * len(reqs)
        # half by wait, half by polling
        for i in range(0, len(reqs), 2):
            got[i] = srv.wait(tickets[i])
        pending = set(range(1, len(reqs), 2))
        deadline = time.time() + 60
        while pending and time.time() < deadline:
            for i in list(pending):
                r = srv.poll(tickets[i])
                if r is not None:
                    got[i] = r
                    pending.discard(i)
            time.sleep(0.002)
        assert not pending, "requests did not finish"
    torch.cuda.synchronize()
    for i, (a, r) in enumerate(zip(alone, got)):
        assert r["status"] == 0, f"request {i} status {r['status']}"
        _same(_h(r), a, f"request {i}")


def test_server_small_budget_runs_one_group_at_a_time():
    """With room for about one request the server still finishes everything
    (groups wait for memory), with the same results."""
    reqs = _requests()[:5]
    alone = []
    for dg, k, sd in reqs:
        r = fl.solve(dg, k, sd, 0.1)
        torch.cuda.synchronize()
        alone.append((r["total_cost"], r["n_open"]))
    budget = 1 << 30
    print("[server] 1 GiB budget", flush=True)
    with fl.Server(hbm_budget_bytes=budget, slots=2) as srv:
        ts = [srv.submit(dg, k, sd, 0.1) for dg, k, sd in reqs]
        got = [srv.wait(t) for t in ts]
    for i, (r, a) in enumerate(zip(got, alone)):
        assert r["status"] == 0
        assert (r["total_cost"], r["n_open"]) == a, f"request {i}"


def test_server_rejects_bad_requests():
    dg = fl.to_device(gg.with_problem(gg.er(50, 4, 1, wmax=5), 1))
    with fl.Server(hbm_budget_bytes=1 << 30, slots=1) as srv:
        with pytest.raises(fl.FlError):
            srv.submit(dg, 0, 1, 0.1)          # k = 0
        with pytest.raises(fl.FlError):
            srv.submit(dg, 8, 1, -1.0)         # eps <= 0
        t = srv.submit(dg, 8, 1, 0.1)
        r = srv.wait(t)
        assert r["status"] == 0
