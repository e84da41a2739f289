"""The seeded workload generators hold the shapes the benchmark and parity
cases state: sizes, symmetry, weight ranges, facility fractions and costs.
They contain none of the method's arithmetic."""
import numpy as np

import graphgen as gg


def _symmetric(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    dst = g.col.astype(np.int64)
    w = g.w if g.w is not None else np.ones(g.n_arcs, np.uint32)
    fwd = set(zip(src.tolist(), dst.tolist(), w.tolist()))
    return all((d, s, x) in fwd for s, d, x in fwd)


def test_rmat_weighted_fac10_shape():
    g = gg.rmat_weighted_fac10(10, 16, 3)
    assert g.n == 1 << 10
    assert g.n_arcs == int(g.row_ptr[-1]) and g.n_arcs > 0
    # weights uniform 1..100 per undirected edge, symmetric, no self loops, sorted rows
    assert g.w is not None and g.w.min() >= 1 and g.w.max() <= 100
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    assert not np.any(src == g.col)
    for v in range(g.n):
        row = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        assert np.all(np.diff(row.astype(np.int64)) > 0)
    assert _symmetric(g)
    # exactly 10% facilities (rounded), lognormal costs rounded to integers >= 1
    fac = g.fac_cost != gg.NOT_FACILITY
    assert int(fac.sum()) == round(0.1 * g.n)
    c = g.fac_cost[fac].astype(np.float64)
    assert c.min() >= 1 and np.all(c == np.rint(c))
    # log of lognormal(5, 1) costs: mean near 5, spread near 1
    lc = np.log(c)
    assert abs(lc.mean() - 5.0) < 0.3 and abs(lc.std() - 1.0) < 0.3
    assert g.is_client is None  # every vertex a client


def test_rmat_weighted_fac10_is_seeded():
    a = gg.rmat_weighted_fac10(9, 8, 5)
    b = gg.rmat_weighted_fac10(9, 8, 5)
    c = gg.rmat_weighted_fac10(9, 8, 6)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w) and np.array_equal(a.fac_cost, b.fac_cost)
    assert not (np.array_equal(a.col, c.col) and np.array_equal(a.fac_cost, c.fac_cost))
