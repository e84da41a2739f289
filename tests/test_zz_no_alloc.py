"""GPU: fl_solve_static, the solve that allocates no device memory (its
workspace is the library's fixed device array), gives exactly fl_solve's
results, call after call on the same array, and refuses inputs that do not
fit with FL_ENOMEM."""
import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1503_03635_amd as fl
from paper_1503_03635_amd import _lib

from gpu_util import host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    fl.lib()


def _host(r):
    return {"open": host(r["open"], np.uint8), "assign": u32(r["assign"]), "dist": u32(r["dist"]),
            "open_rung": u32(r["open_rung"]), "freeze_rung": u32(r["freeze_rung"]),
            "q": host(r["q"], np.float64).view(np.uint64), "total_cost": r["total_cost"],
            "n_open": r["n_open"], "n_unreachable": r["n_unreachable"], "status": r["status"],
            "stats": {k: r["stats"][k] for k in ("rungs", "mis_rounds", "relax_alg", "ads_entries", "gamma",
                                                  "alpha0", "n_guard", "n_reach_guard", "ads_rounds")}}


def _same(a, b, what):
    for key in ("open", "assign", "dist", "open_rung", "freeze_rung", "q"):
        bad = np.nonzero(a[key] != b[key])[0]
        assert len(bad) == 0, f"{what}: {key} differs at {bad[:10]}"
    for key in ("total_cost", "n_open", "n_unreachable", "status", "stats"):
        assert a[key] == b[key], f"{what}: {key} {a[key]} vs {b[key]}"


def _case(name, g, k, seed, outputs=None):
    dg = fl.to_device(g, "cuda:0")
    print(f"[no-alloc] {name}: n={g.n} arcs={g.n_arcs} k={k}", flush=True)
    want = _host(fl.solve(dg, k, seed, 0.1, diagnostics=True))
    got = _host(fl.solve_static(dg, k, seed, 0.1, diagnostics=outputs is None, outputs=outputs))
    torch.cuda.synchronize()
    _same(got, want, name)


def test_static_solve_equals_solve_twice_smaller_second():
    """Two calls in a row on the one array, the second on a smaller input."""
    _case("tiny ER n=2000 w1..10 k16", gg.tiny_er(1), 16, 1)
    _case("ER n=300 w1..10 k8", gg.with_problem(gg.er(300, 5, 7, wmax=10), 7, cost="uniform", cost_hi=200), 8, 2)


def test_static_solve_other_shapes():
    """Weighted hubs, the end phase, a directed graph, and outputs passed in
    (no torch allocation inside the call either)."""
    g = gg.with_problem(gg.star(5000, wmax=100, seed=3), 23, cost="lognormal", fac_frac=0.1)
    outs = fl._alloc_outputs(g.n, torch.device("cuda:0"), True)
    _case("star 5000 w1..100", g, 32, 1, outputs=outs)
    for name, h in gg.end_phase_problems()[:2] + gg.end_phase_problems()[4:5]:
        _case(name, h, 8, 3)
    _case("RMAT 2^12 unit k64", gg.with_problem(gg.rmat(12, 16 << 12, 5), 5, cost="uniform"), 64, 4)


def test_static_solve_refuses_what_does_not_fit():
    """A graph whose sketch rows exceed the array gets FL_ENOMEM, and the next
    call on the array works."""
    big = gg.with_problem(gg.er(200_000, 4, 3), 3, cost="uniform")
    print("[no-alloc] ER n=200000 k=32: refused before any device work", flush=True)
    r = fl.solve_static(fl.to_device(big, "cuda:0"), 32, 1, check=False)
    assert r["rc"] == _lib.FL_ENOMEM
    _case("ER n=300 after a refusal", gg.with_problem(gg.er(300, 5, 7, wmax=10), 7, cost="uniform"), 8, 5)
    # sketch rows of 70,000 x 432 entries fit, the threshold rows after them do not
    mid = gg.with_problem(gg.er(70_000, 4, 4), 4, cost="uniform")
    print("[no-alloc] ER n=70000 k=32: runs out inside the solve", flush=True)
    r = fl.solve_static(fl.to_device(mid, "cuda:0"), 32, 1, check=False)
    assert r["rc"] == _lib.FL_ENOMEM
    _case("ER n=2000 after a refusal", gg.tiny_er(2), 16, 6)


def test_static_solve_errors():
    g = gg.with_problem(gg.er(50, 4, 1, wmax=5), 1)
    with pytest.raises(fl.FlError) as e:
        fl.solve_static(fl.to_device(g), 129, 1)
    assert e.value.code == _lib.FL_ENOTIMPL
    bad = gg.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy(), g.fac_cost)
    bad.w[0] += 1
    with pytest.raises(fl.FlError) as e:
        fl.solve_static(fl.to_device(bad), 4, 1)
    assert e.value.code == _lib.FL_EINVAL
