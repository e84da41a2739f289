"""GPU parity on directed graphs (FL_FLAG_DIRECTED, the graphs Sec. 3.1 also
admits): the sketch of v holds the vertices that reach v, clients are served
by facilities they reach.  Sketches, every solve output, Luby's variant, the
batched and served paths, all bit for bit against the oracle or the single
solve."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as O
import paper_1503_03635_amd as fl

from gpu_util import assert_sketch_equal, assert_solve_equal, gpu_solve, host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    fl.lib()


def _star(n, inward, fac_hub_only):
    leaves = np.arange(1, n)
    hub = np.zeros(n - 1, np.int64)
    u, v = (leaves, hub) if inward else (hub, leaves)
    g = gg.from_arcs(n, u, v, None, None, name="instar" if inward else "outstar")
    if fac_hub_only:
        g.fac_cost = np.array([7] + [gg.NOT_FACILITY] * (n - 1), np.uint32)
    return g


SKETCH_CASES = [
    ("dER 600 w1..10", lambda: gg.er(600, 5, 1, wmax=10, directed=True), 8),
    ("dRMAT 2^12 unit", lambda: gg.rmat(12, 16 << 12, 2, directed=True), 16),
    ("dRMAT 2^11 w1..100", lambda: gg.rmat(11, 16 << 11, 3, wmax=100, directed=True), 32),
    ("dFF 3000 w1..20", lambda: gg.forest_fire(3000, 4, wmax=20, directed=True), 16),
    ("dpath+dcycle", lambda: gg.disjoint_union(gg.path(40, directed=True), gg.cycle(33, wmax=3, directed=True)), 4),
    ("in-star 3000 (hub gathers 2999 arcs)", lambda: _star(3000, True, False), 8),
    ("out-star 3000 (hub marks 2999 arcs)", lambda: _star(3000, False, False), 8),
]


@pytest.mark.parametrize("ci", range(len(SKETCH_CASES)))
def test_directed_sketches_bit_exact(ci):
    name, make, k = SKETCH_CASES[ci]
    g = make()
    print(f"[directed sketch] {name} n={g.n} arcs={g.n_arcs} k={k}", flush=True)
    assert_sketch_equal(g, k, 5)
    if ci in (1, 5):
        assert_sketch_equal(g, k, 6, flags=fl.FL_FLAG_NO_DENSE)


def _problems():
    return [
        ("dER 600 w1..10", gg.with_problem(gg.er(600, 5, 1, wmax=10, directed=True), 1, cost="uniform", cost_hi=200)),
        ("dRMAT 2^12 unit", gg.with_problem(gg.rmat(12, 16 << 12, 2, directed=True), 2, cost="uniform")),
        ("dRMAT 2^11 w1..100 10% fac", gg.with_problem(gg.rmat(11, 16 << 11, 3, wmax=100, directed=True), 3,
                                                       cost="lognormal", fac_frac=0.1)),
        ("dFF 3000 w1..20 60% clients", gg.with_problem(gg.forest_fire(3000, 4, wmax=20, directed=True), 4,
                                                        cost="uniform", client_frac=0.6)),
        ("dpath+dcycle", gg.with_problem(gg.disjoint_union(gg.path(40, directed=True),
                                                           gg.cycle(33, wmax=3, directed=True)), 5,
                                         cost="uniform", cost_hi=50)),
        ("in-star, facility at the hub", _star(3000, True, True)),
        ("out-star, facility at the hub", _star(3000, False, True)),
    ]


PROBLEMS = _problems()


@pytest.mark.parametrize("pi", range(len(PROBLEMS)))
@pytest.mark.parametrize("k,seed", [(16, 7), (4, 2)])
def test_directed_solve_bit_exact(pi, k, seed):
    name, g = PROBLEMS[pi]
    print(f"[directed solve] {name} n={g.n} arcs={g.n_arcs} k={k} seed={seed}", flush=True)
    got, want = assert_solve_equal(g, k, seed)
    if pi == 3 and (k, seed) == (16, 7):
        assert want["n_reach_guard"] > 0          # the reach guard is exercised


@pytest.mark.parametrize("pi", [0, 1, 3])
def test_directed_luby_bit_exact(pi):
    name, g = PROBLEMS[pi]
    print(f"[directed luby] {name}", flush=True)
    assert_solve_equal(g, 16, 7, flags=fl.FL_FLAG_LUBY_MIS)


def test_symmetric_arcs_read_as_directed_equal_undirected():
    """The same symmetric arrays with and without FL_FLAG_DIRECTED give the
    same outputs (every search direction coincides)."""
    g = gg.with_problem(gg.rmat(12, 16 << 12, 9, wmax=20), 9, cost="uniform")
    a = gpu_solve(g, 16, 3)
    b = gpu_solve(g, 16, 3, flags=fl.FL_FLAG_DIRECTED)
    for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["q"].view(np.uint64), b["q"].view(np.uint64))
    assert a["total_cost"] == b["total_cost"] and b["stats"]["n_reach_guard"] == 0


def _host(r):
    return {"open": host(r["open"], np.uint8), "assign": u32(r["assign"]), "dist": u32(r["dist"]),
            "q": host(r["q"], np.float64), "open_rung": u32(r["open_rung"]),
            "freeze_rung": u32(r["freeze_rung"]), "total_cost": r["total_cost"], "status": r["status"],
            "n_reach_guard": r["stats"]["n_reach_guard"], "mis_rounds": r["stats"]["mis_rounds"]}


def _same(a, b, what):
    for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
        assert np.array_equal(a[key], b[key]), f"{what}: {key}"
    assert np.array_equal(a["q"].view(np.uint64), b["q"].view(np.uint64)), f"{what}: q"
    for key in ("total_cost", "status", "n_reach_guard", "mis_rounds"):
        assert a[key] == b[key], f"{what}: {key}"


def test_directed_batch_equals_single_solves():
    """Directed and undirected graphs in one fl_solve_batch call: they go to
    different groups, and every element equals its own fl_solve."""
    graphs = [g for _, g in PROBLEMS[:5]] + [gg.with_problem(gg.er(300, 5, 8, wmax=6), 8, cost="uniform")]
    dgs = [fl.to_device(g) for g in graphs]
    print(f"[directed batch] {len(graphs)} graphs", flush=True)
    got = fl.solve_batch(dgs, 16, 7, 0.1, diagnostics=True)
    torch.cuda.synchronize()
    for i, (dg, r) in enumerate(zip(dgs, got)):
        alone = fl.solve(dg, 16, 7, 0.1, diagnostics=True)
        torch.cuda.synchronize()
        _same(_host(r), _host(alone), f"element {i}")


def test_directed_server_equals_single_solve():
    _, g = PROBLEMS[3]
    dg = fl.to_device(g)
    print("[directed server]", flush=True)
    with fl.Server(slots=2) as srv:
        t = srv.submit(dg, 16, 7, 0.1, diagnostics=True)
        r = srv.wait(t)
    torch.cuda.synchronize()
    alone = fl.solve(dg, 16, 7, 0.1, diagnostics=True)
    torch.cuda.synchronize()
    _same(_host(r), _host(alone), "server")


def test_directed_input_errors():
    """A self loop is rejected with the directed flag; asymmetric arrays are
    rejected without it; the batch reports the bad element alone."""
    g = gg.with_problem(gg.er(200, 4, 3, wmax=5, directed=True), 3)
    bad = gg.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy(), g.fac_cost, directed=True)
    r0 = int(np.nonzero(np.diff(g.row_ptr.astype(np.int64)) > 0)[0][0])
    bad.col[g.row_ptr[r0]] = r0
    assert bad.col[g.row_ptr[r0]] == r0 and O.validate(bad, 4, 0.1) == O.EINVAL
    print("[directed errors]", flush=True)
    r = fl.solve(fl.to_device(bad), 4, 1, check=False)
    assert r["rc"] == fl._lib.FL_EINVAL
    und = gg.Graph(g.n, g.row_ptr, g.col, g.w, g.fac_cost, directed=False)
    assert O.validate(und, 4, 0.1) == O.EINVAL
    r = fl.solve(fl.to_device(und), 4, 1, check=False)
    assert r["rc"] == fl._lib.FL_EINVAL
    outs = fl.solve_batch([fl.to_device(g), fl.to_device(bad)], 4, 1, check=False)
    torch.cuda.synchronize()
    assert outs[0]["status"] == 0 and outs[1]["status"] == fl._lib.FL_EINVAL


def _degenerate():
    out = []
    g = gg.with_problem(gg.empty(7, directed=True), 1, cost="uniform", cost_hi=20, fac_frac=0.5)
    out.append(("no arcs, half facilities", g))
    one = gg.empty(1, directed=True)
    one.fac_cost = np.array([3], np.uint32)
    out.append(("single vertex", one))
    # a DAG: arcs only from lower to higher ids, facilities at the top end only
    rng = np.random.default_rng(4)
    u = rng.integers(0, 400, 1600)
    v = rng.integers(0, 400, 1600)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    dag = gg.from_arcs(400, lo, hi, 9, rng, name="dag400")
    dag.fac_cost = np.where(np.arange(400) >= 350, rng.integers(1, 100, 400), gg.NOT_FACILITY).astype(np.uint32)
    out.append(("DAG, facilities downstream", dag))
    out.append(("directed path+cycle+isolated", gg.with_problem(gg.disjoint_union(
        gg.path(30, directed=True), gg.cycle(11, directed=True), gg.empty(4, directed=True)), 2, cost="uniform",
        cost_hi=40)))
    return out


@pytest.mark.parametrize("ci", range(4))
def test_directed_degenerate_cases(ci):
    name, g = _degenerate()[ci]
    print(f"[directed degenerate] {name}", flush=True)
    got, want = assert_solve_equal(g, 8, 3)
    if ci == 2:
        assert want["n_unreachable"] > 0      # clients with no facility downstream
