"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element, on seeded inputs.  Integer outputs must be bit-exact; the double
q(f) must agree to 1e-12 relative (bit-exact in practice)."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as O
import paper_1503_03635_amd as fl

from gpu_util import assert_sketch_equal, assert_solve_equal, gpu_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    fl.lib()


SKETCH_CASES = [
    ("tiny ER n=2000 w1..10", lambda: gg.tiny_er(1), 16),
    ("ER n=500 unit", lambda: gg.er(500, 6, 3), 4),
    ("RMAT 2^12 unit", lambda: gg.rmat(12, 16 << 12, 5), 64),
    ("RMAT 2^11 w1..100", lambda: gg.rmat(11, 8 << 11, 6, wmax=100), 32),
    ("grid 20x20 ties", lambda: gg.grid(20, 20), 8),
    ("clique 70 (hub rows)", lambda: gg.clique(70, wmax=3), 64),
    ("star 3000 (one hub)", lambda: gg.star(3000), 16),
    ("path 300 w1..255", lambda: gg.path(300, wmax=255, seed=2), 2),
    ("disjoint + isolated", lambda: gg.disjoint_union(gg.path(40), gg.star(30, wmax=5), gg.empty(5),
                                                      gg.cycle(17)), 3),
    ("Chung-Lu n=3000 w1..20", lambda: gg.chung_lu(3000, 4, 2.2, 10.0, 20), 32),
]


@pytest.mark.parametrize("name,make,k", SKETCH_CASES, ids=[c[0] for c in SKETCH_CASES])
def test_sketches_bit_exact(name, make, k):
    g = make()
    print(f"[sketch] {name} n={g.n} arcs={g.n_arcs} k={k}", flush=True)
    assert_sketch_equal(g, k, seed=7)


@pytest.mark.parametrize("k", [1, 2, 5, 64, 65, 100, 128])
def test_sketches_k_edges(k):
    g = gg.rmat(10, 6 << 10, 11)
    print(f"[sketch] rmat 2^10 k={k}", flush=True)
    assert_sketch_equal(g, k, seed=3)


def test_sketches_k_at_least_n():
    g = gg.er(60, 5, 2, wmax=4)
    print("[sketch] k >= n", flush=True)
    assert_sketch_equal(g, 64, seed=1)
    g = gg.er(120, 5, 3, wmax=4)
    print("[sketch] k >= n, two registers", flush=True)
    assert_sketch_equal(g, 128, seed=1)


# k above 64 holds the running bottom-k set in two registers per lane and a
# survivor buffer of twice the size: sketches and solves on unit and weighted
# graphs, hubs and worklist rounds
BIG_K_CASES = [
    ("RMAT 2^12 unit k128", lambda: gg.rmat(12, 16 << 12, 5), 128),
    ("RMAT 2^11 w1..100 k96", lambda: gg.rmat(11, 8 << 11, 6, wmax=100), 96),
    ("star 3000 k128", lambda: gg.star(3000), 128),
    ("star 5000 w1..100 k128", lambda: gg.star(5000, wmax=100, seed=3), 128),
    ("Chung-Lu n=3000 w1..20 k80", lambda: gg.chung_lu(3000, 4, 2.2, 10.0, 20), 80),
    ("grid 20x20 ties k128", lambda: gg.grid(20, 20), 128),
]


@pytest.mark.parametrize("name,make,k", BIG_K_CASES, ids=[c[0] for c in BIG_K_CASES])
def test_sketches_big_k(name, make, k):
    g = make()
    print(f"[sketch] {name} n={g.n} arcs={g.n_arcs}", flush=True)
    assert_sketch_equal(g, k, seed=7)
    assert_sketch_equal(g, k, seed=8, flags=fl.FL_FLAG_NO_DENSE)


@pytest.mark.parametrize("k", [65, 128])
def test_solve_big_k(k):
    for name, make in (("RMAT 2^11 unit", lambda: gg.with_problem(gg.rmat(11, 16 << 11, 8), 8, cost="uniform")),
                       ("RMAT 2^10 w1..100 10% fac", lambda: gg.with_problem(gg.rmat(10, 16 << 10, 9, wmax=100), 9,
                                                                            cost="lognormal", fac_frac=0.1))):
        print(f"[solve] {name} k={k}", flush=True)
        assert_solve_equal(make(), k, 1)



# k <= 32 starts with a survivor buffer of 512 ids per level; a level that
# accepts more restarts the build with the full buffer.  The hook
# FL_TEST_SMALL_SURVIVOR_BUFFER starts k <= 64 with the small buffer too, so
# that a modest input overflows it: the hub of a star with 10^5 leaves accepts
# about 64 (1 + ln(10^5 / 64)) = 535 leaves in its one level at k = 64.
@pytest.mark.parametrize("wmax", [None, 1], ids=["unit (dense rounds)", "weights 1 (worklist rounds)"])
def test_sketches_survivor_buffer_restart(wmax, monkeypatch, capfd):
    monkeypatch.setenv("FL_TEST_SMALL_SURVIVOR_BUFFER", "1")
    monkeypatch.setenv("FL_DEBUG", "1")
    g = gg.star(100_000, wmax=wmax, seed=3)
    print(f"[sketch] star 10^5 leaves wmax={wmax} k=64, small survivor buffer", flush=True)
    assert_sketch_equal(g, 64, seed=5)
    err = capfd.readouterr().err
    assert "survivor buffer 512 overflowed" in err

def test_sketches_schedule_invariant():
    """Dense rounds and frontier worklists give the same bytes."""
    g = gg.rmat(12, 16 << 12, 9)
    print("[sketch] dense vs frontier", flush=True)
    a = assert_sketch_equal(g, 32, seed=2, flags=0)
    b = assert_sketch_equal(g, 32, seed=2, flags=fl.FL_FLAG_NO_DENSE)
    for key in a:
        assert np.array_equal(a[key], b[key])



# At k <= 32 rounds run from worklists take two small tasks per wave; slices
# of split vertices and levels of more than 32 survivors go to the one-wave
# kernel.  Unit-weight inputs with hubs (long entry lists, split rows) on the
# worklist schedule, next to the weighted cases above and below.
TWO_TASK_UNIT_CASES = [
    ("star 9000 unit k32", lambda: gg.star(9000), 32),
    ("RMAT 2^13 unit k16", lambda: gg.rmat(13, 16 << 13, 12), 16),
]


@pytest.mark.parametrize("name,make,k", TWO_TASK_UNIT_CASES, ids=[c[0] for c in TWO_TASK_UNIT_CASES])
def test_sketches_two_task_unit_worklists(name, make, k):
    g = make()
    print(f"[sketch] {name} n={g.n} arcs={g.n_arcs} (worklist rounds)", flush=True)
    assert_sketch_equal(g, k, seed=4, flags=fl.FL_FLAG_NO_DENSE)

SOLVE_CASES = [
    ("tiny ER n=2000 w1..10 k16 cost50", lambda: gg.tiny_er(1), 16),
    ("ER n=400 w1..10 costs 1..200", lambda: gg.with_problem(gg.er(400, 5, 7, wmax=10), 7, cost="uniform",
                                                             cost_lo=1, cost_hi=200), 8),
    ("RMAT 2^11 unit costs 1..1000", lambda: gg.with_problem(gg.rmat(11, 16 << 11, 8), 8, cost="uniform"), 64),
    ("RMAT 2^10 w1..100 10% fac lognormal", lambda: gg.with_problem(gg.rmat(10, 16 << 10, 9, wmax=100), 9,
                                                                    cost="lognormal", fac_frac=0.1), 32),
    ("grid 15x15 w1..4", lambda: gg.with_problem(gg.grid(15, 15, wmax=4), 4, cost="uniform", cost_lo=1,
                                                 cost_hi=60), 8),
    # unit weights and many ties: MIS radii land exactly on the distances of
    # many clients (the sweeps keep labels at the radius only at targets)
    ("grid 20x20 unit costs 1..30", lambda: gg.with_problem(gg.grid(20, 20), 11, cost="uniform", cost_lo=1,
                                                             cost_hi=30), 4),
    ("Chung-Lu n=2000 w1..20", lambda: gg.with_problem(gg.chung_lu(2000, 3, 2.2, 10.0, 20), 3,
                                                       cost="uniform"), 32),
    ("half clients", lambda: gg.with_problem(gg.er(300, 4, 5, wmax=6), 5, cost="uniform", cost_hi=100,
                                             client_frac=0.5, fac_frac=0.5), 8),
]


@pytest.mark.parametrize("name,make,k", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_bit_exact(name, make, k):
    g = make()
    print(f"[solve] {name} n={g.n} arcs={g.n_arcs} k={k}", flush=True)
    for seed in (1, 2):
        assert_solve_equal(g, k, seed)


@pytest.mark.parametrize("eps", [0.01, 1.0])
def test_solve_other_eps(eps):
    g = gg.with_problem(gg.er(200, 5, 2, wmax=5), 2, cost="uniform", cost_hi=80)
    print(f"[solve] eps={eps}", flush=True)
    assert_solve_equal(g, 8, 3, eps=eps)


@pytest.mark.parametrize("name,make,k", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_luby_mis_bit_exact(name, make, k):
    """Luby's MIS variant (priorities redrawn every round) against the oracle's."""
    g = make()
    print(f"[solve luby] {name} k={k}", flush=True)
    assert_solve_equal(g, k, 2, flags=fl.FL_FLAG_LUBY_MIS)


def test_solve_tiny_exhaustive_graphs():
    for seed in range(8):
        n = 8 + seed % 5
        g = gg.with_problem(gg.er(n, 3, seed, wmax=6), seed, cost="uniform", cost_lo=1, cost_hi=25)
        print(f"[solve] tiny n={n} seed={seed}", flush=True)
        for k in (1, 4, n):
            assert_solve_equal(g, k, seed)


def test_solve_stall_guard():
    for seed in range(200):
        g = gg.star(5)
        g.fac_cost = np.array([3] + [gg.NOT_FACILITY] * 4, np.uint32)
        g.is_client = np.array([0, 1, 1, 1, 1], np.uint8)
        sk = O.ads_pruned(g, 1, seed=seed)
        if sk["off"][1] - sk["off"][0] == 1:
            print(f"[solve] guard seed={seed}", flush=True)
            got, want = assert_solve_equal(g, 1, seed)
            assert want["n_guard"] == 1
            return
    pytest.fail("no seed for the guard case")


END_CASES = gg.end_phase_problems()


@pytest.mark.parametrize("idx", range(len(END_CASES)), ids=[c[0] for c in END_CASES])
def test_solve_end_phase(idx):
    """Alg. 4's end phase (every facility open, clients left unfrozen): END
    rungs, open set, assignment, q and cost equal the oracle's, and the
    branch really fires on each input."""
    name, g = END_CASES[idx]
    for k, seed in ((4, 1), (16, 2)):
        print(f"[solve end] {name} k={k} seed={seed}", flush=True)
        got, want = assert_solve_equal(g, k, seed)
        assert (want["freeze_rung"] == O.RUNG_END).any(), "the end phase must fire"
        assert (got["freeze_rung"] == fl.FL_RUNG_END).sum() == (want["freeze_rung"] == O.RUNG_END).sum()


def test_solve_end_phase_batched():
    """The end-phase inputs solved together in one batch (directed and
    undirected mixed) give each element the oracle's result."""
    gs = [g for _, g in END_CASES]
    print(f"[solve end] batch of {len(gs)}", flush=True)
    outs = fl.solve_batch([fl.to_device(g) for g in gs], 8, 3, diagnostics=True)
    torch.cuda.synchronize()
    for (name, g), r in zip(END_CASES, outs):
        rc, want = O.solve(g, 8, 3, 0.1)
        assert rc == 0 and r["status"] == 0
        assert (want["freeze_rung"] == O.RUNG_END).any(), name
        for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
            got = r[key].cpu().numpy()
            got = got.view(np.uint32) if key != "open" else got
            assert np.array_equal(got, want[key]), f"{name}: {key}"
        assert r["total_cost"] == want["total_cost"], name


# Rounds run from worklists (every round of a weighted graph) cut rows of more
# than 8,192 arcs into several tasks whose kept sets a merge block prunes
# again: the inputs below have such hubs with weights 1..100.
SPLIT_ARCS_SPARSE = 8192


def _weighted_in_star(n, seed):
    """Directed star: every leaf has an arc into the hub, weights 1..100."""
    leaves = np.arange(1, n, dtype=np.uint32)
    return gg.from_arcs(n, leaves, np.zeros(n - 1, np.uint32), 100, np.random.Generator(np.random.PCG64(seed)),
                        name=f"instar_{n}")


WEIGHTED_HUB_CASES = [
    ("star 9000 w1..100", lambda: gg.star(9000, wmax=100, seed=3), 32),
    ("in-star 9000 w1..100", lambda: _weighted_in_star(9000, 4), 16),
    ("RMAT 2^14 x16 + star 9000, w1..100",
     lambda: gg.disjoint_union(gg.rmat(14, 16 << 14, 22, wmax=100), gg.star(9000, wmax=100, seed=5)), 32),
]


def _max_in_degree(g):
    return int(np.bincount(g.col, minlength=g.n).max()) if g.n_arcs else 0


@pytest.mark.parametrize("name,make,k", WEIGHTED_HUB_CASES, ids=[c[0] for c in WEIGHTED_HUB_CASES])
def test_sketches_weighted_split_hubs(name, make, k):
    """Weighted hubs above the split threshold: the split tasks, their kept
    sets and the merge that prunes them again give the oracle's sketches."""
    g = make()
    assert _max_in_degree(g) > SPLIT_ARCS_SPARSE
    print(f"[sketch] {name} n={g.n} arcs={g.n_arcs} max in-degree {_max_in_degree(g)} k={k}", flush=True)
    assert_sketch_equal(g, k, seed=5)


@pytest.mark.parametrize("name,make,k", WEIGHTED_HUB_CASES, ids=[c[0] for c in WEIGHTED_HUB_CASES])
def test_solve_weighted_split_hubs(name, make, k):
    """Full solves on the same inputs with the large weighted recipe's problem
    (10% facilities, lognormal costs, every vertex a client)."""
    g = gg.with_problem(make(), 23, cost="lognormal", fac_frac=0.1)
    assert _max_in_degree(g) > SPLIT_ARCS_SPARSE
    print(f"[solve] {name} 10% lognormal facilities k={k}", flush=True)
    assert_solve_equal(g, k, 1)


def test_solve_degenerate_inputs():
    cases = []
    nocl = gg.with_problem(gg.er(40, 4, 2, wmax=3), 2, cost="uniform", cost_hi=20)
    nocl.is_client = np.zeros(nocl.n, np.uint8)
    cases.append(("no clients", nocl))
    one = gg.empty(1)
    one.fac_cost = np.array([5], np.uint32)
    cases.append(("single vertex", one))
    iso = gg.empty(50)
    iso.fac_cost = np.arange(1, 51, dtype=np.uint32)
    cases.append(("isolated vertices", iso))
    nofac = gg.with_problem(gg.path(20), 1)
    nofac.fac_cost = np.full(20, gg.NOT_FACILITY, np.uint32)
    cases.append(("no facilities", nofac))
    comp = gg.disjoint_union(gg.path(10), gg.star(8))
    fc = np.full(comp.n, gg.NOT_FACILITY, np.uint32)
    fc[:10] = 4                                   # the star has no facility
    comp.fac_cost = fc
    cases.append(("unreachable clients", comp))
    for name, g in cases:
        print(f"[solve] {name}", flush=True)
        assert_solve_equal(g, 4, 1)


def test_error_codes():
    g = gg.with_problem(gg.er(50, 4, 1, wmax=5), 1)
    dg = fl.to_device(g)
    with pytest.raises(fl.FlError) as e:
        fl.solve(dg, 129, 1)
    assert e.value.code == fl._lib.FL_ENOTIMPL
    with pytest.raises(fl.FlError) as e:
        fl.solve(dg, 4, 1, eps=-1.0)
    assert e.value.code == fl._lib.FL_EINVAL
    bad = gg.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy(), g.fac_cost)
    bad.w[0] += 1                                 # asymmetric weight
    with pytest.raises(fl.FlError) as e:
        fl.solve(fl.to_device(bad), 4, 1)
    assert e.value.code == fl._lib.FL_EINVAL
    bad = gg.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy(), g.fac_cost)
    bad.w[3] = 0
    with pytest.raises(fl.FlError) as e:
        fl.solve(fl.to_device(bad), 4, 1)
    assert e.value.code == fl._lib.FL_EINVAL
    # a star with one arc dropped: the leaf's arc to the hub is checked only
    # through the arc counts, the hub's arc to the leaf by its lookup
    for drop_from_hub in (True, False):
        st = gg.with_problem(gg.star(20), 1)
        rows = [list(st.col[st.row_ptr[v]:st.row_ptr[v + 1]]) for v in range(st.n)]
        if drop_from_hub:
            rows[0].remove(5)
        else:
            rows[5].remove(0)
        rp = np.zeros(st.n + 1, np.uint64)
        rp[1:] = np.cumsum([len(r) for r in rows])
        cut = gg.Graph(st.n, rp, np.array([x for r in rows for x in r], np.uint32), None, st.fac_cost)
        assert O.validate(cut, 4, 0.1) == O.EINVAL
        with pytest.raises(fl.FlError) as e:
            fl.solve(fl.to_device(cut), 4, 1)
        assert e.value.code == fl._lib.FL_EINVAL
        outs = fl.solve_batch([fl.to_device(cut), dg], 4, 1, check=False)
        assert outs[0]["status"] == fl._lib.FL_EINVAL and outs[1]["status"] == 0
    big = gg.with_problem(gg.path(5, wmax=None), 1)
    big.w = np.full(big.n_arcs, 300, np.uint32)   # beyond the slot ring
    with pytest.raises(fl.FlError) as e:
        fl.solve(fl.to_device(big), 4, 1)
    assert e.value.code == fl._lib.FL_ENOTIMPL
    huge = gg.with_problem(gg.path(3), 1)
    huge.w = np.full(huge.n_arcs, 200, np.uint32)
    huge.fac_cost = np.array([0xFFFFFFF0, 1, 1], np.uint32)
    with pytest.raises(fl.FlError) as e:
        fl.solve(fl.to_device(huge), 4, 1)
    assert e.value.code == fl._lib.FL_ERANGE
    # the library keeps working after errors
    assert_solve_equal(g, 4, 1)
