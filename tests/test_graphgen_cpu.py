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


# ---------------------------------------------------------------- device generators (run on CPU tensors here)
def test_device_rmat_weighted_recipe():
    """The device R-MAT of the large weighted recipe is a valid symmetric CSR
    (checked by the oracle's validator), equal weights on both arcs of an edge,
    weights in 1..100, an exact 10% of facilities with lognormal costs, and the
    same arrays for the same seed."""
    import torch
    import graphgen.device as gd
    import oracle as O
    a = gd.rmat_weighted_fac10(12, 32, 3, device="cpu")
    b = gd.rmat_weighted_fac10(12, 32, 3, device="cpu")
    assert torch.equal(a.col, b.col) and torch.equal(a.w, b.w) and torch.equal(a.fac_cost, b.fac_cost)
    g = gd.to_host(a)
    assert O.validate(g, 8, 0.1) == O.OK
    assert g.w.min() >= 1 and g.w.max() <= 100
    isF = g.fac_cost != gg.NOT_FACILITY
    assert isF.sum() == round(0.1 * g.n)
    c = g.fac_cost[isF].astype(np.float64)
    assert c.min() >= 1 and 4.5 < np.log(c).mean() < 5.5
    assert g.n == 1 << 12 and 20 < g.n_arcs / g.n < 32
    c2 = gd.to_host(gd.rmat_weighted_fac10(12, 32, 4, device="cpu"))
    assert not np.array_equal(c2.col[:1000], g.col[:1000])


def test_device_directed_and_batch_generators():
    """Directed R-MAT keeps arcs (no symmetry needed, validated as directed);
    the Chung-Lu batch gives valid graphs with n in range and weights 1..20."""
    import graphgen.device as gd
    import oracle as O
    h = gd.to_host(gd.rmat_unit(10, 16, 2, directed=True, device="cpu"))
    assert h.directed and O.validate(h, 4, 0.1) == O.OK
    for dg in gd.powerlaw_batch(3, 5, n_lo=500, n_hi=5000, device="cpu"):
        x = gd.to_host(dg)
        assert 500 <= x.n <= 5000 and O.validate(x, 4, 0.1) == O.OK
        assert x.w.min() >= 1 and x.w.max() <= 20
        assert (x.fac_cost >= 1).all() and (x.fac_cost <= 1000).all()
