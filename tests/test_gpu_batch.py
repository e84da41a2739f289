"""GPU: fl_solve_batch solves several graphs together as one disjoint union.
Every element must get exactly what fl_solve gives it alone (and therefore
what the oracle gives): opened set, assignment, distances, rungs, q bit for
bit, cost, counts and the per-graph statistics."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as O
import paper_1503_03635_amd as fl

from gpu_util import host, u32

pytestmark = pytest.mark.gpu

PER_GRAPH_STATS = ("rungs", "mis_rounds", "relax_alg", "ads_entries", "gamma", "alpha0", "n_guard")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    fl.lib()


def _host(r):
    return {"open": host(r["open"], np.uint8), "assign": u32(r["assign"]), "dist": u32(r["dist"]),
            "open_rung": u32(r["open_rung"]), "freeze_rung": u32(r["freeze_rung"]),
            "q": host(r["q"], np.float64), "total_cost": r["total_cost"], "n_open": r["n_open"],
            "n_unreachable": r["n_unreachable"], "status": r["status"], "stats": r["stats"]}


def _assert_same(a, b, what):
    for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
        bad = np.nonzero(a[key] != b[key])[0]
        assert len(bad) == 0, f"{what}: {key} differs at {bad[:10]}"
    assert np.array_equal(a["q"].view(np.uint64), b["q"].view(np.uint64)), f"{what}: q differs"
    for key in ("total_cost", "n_open", "n_unreachable", "status"):
        assert a[key] == b[key], f"{what}: {key} {a[key]} vs {b[key]}"
    for key in PER_GRAPH_STATS:
        assert a["stats"][key] == b["stats"][key], f"{what}: stats.{key} {a['stats'][key]} vs {b['stats'][key]}"


def _mixed():
    return [
        ("ER 300 w1..10", gg.with_problem(gg.er(300, 5, 1, wmax=10), 1, cost="uniform", cost_hi=200)),
        ("RMAT 2^10 unit", gg.with_problem(gg.rmat(10, 8 << 10, 2), 2, cost="uniform")),
        ("Chung-Lu 800 w1..20", gg.with_problem(gg.chung_lu(800, 3, 2.2, 10.0, 20), 3, cost="uniform")),
        ("grid 12x12 w1..4", gg.with_problem(gg.grid(12, 12, wmax=4), 4, cost="uniform", cost_hi=60)),
        ("half clients", gg.with_problem(gg.er(200, 4, 5, wmax=6), 5, cost="uniform", cost_hi=100,
                                         client_frac=0.5, fac_frac=0.5)),
        ("path+star+isolated", gg.with_problem(gg.disjoint_union(gg.path(30), gg.star(20), gg.empty(3)), 6,
                                               cost="uniform", cost_hi=50)),
        ("RMAT 2^9 w1..100 10% fac", gg.with_problem(gg.rmat(9, 16 << 9, 7, wmax=100), 7, cost="lognormal",
                                                     fac_frac=0.1)),
        ("single vertex", _single()),
    ]


def _single():
    g = gg.empty(1)
    g.fac_cost = np.array([5], np.uint32)
    return g


def test_batch_equals_single_solves():
    cases = _mixed()
    dgs = [fl.to_device(g) for _, g in cases]
    seeds = [11 + i for i in range(len(cases))]
    print(f"[batch] {len(cases)} mixed graphs, k=16", flush=True)
    got = fl.solve_batch(dgs, 16, seeds, 0.1, diagnostics=True)
    torch.cuda.synchronize()
    for (name, g), dg, sd, r in zip(cases, dgs, seeds, got):
        alone = fl.solve(dg, 16, sd, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        _assert_same(_host(r), _host(alone), name)


def test_batch_equals_oracle():
    cases = _mixed()[:4]
    dgs = [fl.to_device(g) for _, g in cases]
    print("[batch] oracle parity, k=8", flush=True)
    got = fl.solve_batch(dgs, 8, 3, 0.1, diagnostics=True)
    torch.cuda.synchronize()
    for (name, g), r in zip(cases, got):
        rc, want = O.solve(g, 8, 3, 0.1)
        assert rc == 0
        h = _host(r)
        for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
            assert np.array_equal(h[key], want[key]), f"{name}: {key}"
        assert np.array_equal(h["q"].view(np.uint64), want["q"].view(np.uint64)), f"{name}: q"
        assert h["total_cost"] == want["total_cost"], name
        assert h["stats"]["rungs"] == want["n_rungs"], name
        assert h["stats"]["mis_rounds"] == want["mis_rounds"], name


def test_batch_groups_by_parameters():
    """Elements with different k and eps go to different groups; each still
    equals its single solve."""
    cases = _mixed()[:5]
    dgs = [fl.to_device(g) for _, g in cases]
    ks = [4, 16, 4, 16, 8]
    epss = [0.1, 0.1, 0.5, 0.1, 0.1]
    print("[batch] mixed k/eps", flush=True)
    got = fl.solve_batch(dgs, ks, 5, epss, diagnostics=True)
    torch.cuda.synchronize()
    for (name, g), dg, k, e, r in zip(cases, dgs, ks, epss, got):
        alone = fl.solve(dg, k, 5, e, diagnostics=True)
        torch.cuda.synchronize()
        _assert_same(_host(r), _host(alone), f"{name} k={k} eps={e}")


def test_batch_bad_element_reports_alone():
    """An invalid element gets its error; the others are solved as usual."""
    good = _mixed()[:3]
    bad = gg.with_problem(gg.er(60, 4, 9, wmax=5), 9)
    bad.col = bad.col.copy()
    bad.col[0] = (bad.col[0] + 1) % bad.n        # breaks symmetry (or sortedness)
    graphs = [good[0][1], bad, good[1][1], good[2][1]]
    dgs = [fl.to_device(g) for g in graphs]
    print("[batch] one invalid element", flush=True)
    got = fl.solve_batch(dgs, 8, 2, 0.1, diagnostics=True, check=False)
    torch.cuda.synchronize()
    assert got[1]["status"] == fl._lib.FL_EINVAL
    assert got[1]["n_open"] == 0
    for i in (0, 2, 3):
        alone = fl.solve(dgs[i], 8, 2, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        _assert_same(_host(got[i]), _host(alone), f"element {i}")


def test_batch_many_small_graphs():
    """A few dozen power-law graphs of uneven sizes in one call."""
    graphs = gg.powerlaw_batch(24, 3, n_lo=100, n_hi=3000, avg_deg=6.0, wmax=20)
    dgs = [fl.to_device(g) for g in graphs]
    print(f"[batch] {len(graphs)} power-law graphs", flush=True)
    got = fl.solve_batch(dgs, 8, 4, 0.1, diagnostics=True)
    torch.cuda.synchronize()
    for i, (dg, r) in enumerate(zip(dgs, got)):
        alone = fl.solve(dg, 8, 4, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        _assert_same(_host(r), _host(alone), f"graph {i} n={dg.n}")


def test_batch_weight_beyond_limit_reports_alone():
    """An element whose largest weight exceeds the slot ring's limit (255)
    gets FL_ENOTIMPL; the batch's weight pre-pass counts it at the limit when
    it sizes the group, and the other elements are solved as usual."""
    good = _mixed()[:3]
    heavy = gg.with_problem(gg.er(80, 4, 12, wmax=1000), 12, cost="uniform")
    assert int(heavy.w.max()) > 255
    graphs = [good[0][1], heavy, good[1][1], good[2][1]]
    dgs = [fl.to_device(g) for g in graphs]
    print("[batch] one element with weights above 255", flush=True)
    got = fl.solve_batch(dgs, 8, 6, 0.1, diagnostics=True, check=False)
    torch.cuda.synchronize()
    assert got[1]["status"] == fl._lib.FL_ENOTIMPL
    assert got[1]["n_open"] == 0
    for i in (0, 2, 3):
        alone = fl.solve(dgs[i], 8, 6, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        _assert_same(_host(got[i]), _host(alone), f"element {i}")
