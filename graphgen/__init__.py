"""Seeded synthetic inputs for sketch-based facility location.

This module only builds inputs: undirected graphs as symmetric CSR arrays,
directed graphs as CSR arrays of out-arcs, edge weights, facility opening
costs and client sets.  It holds none of the
method's arithmetic, and both the HIP library's tests and the CPU oracle take
their inputs from here.

Graph families (the paper's experiments use R-MAT and Forest Fire graphs with
uniform weights in 1..100; the workloads below stand in for them):

* ``er``        Erdos-Renyi G(n, p), sampled by geometric skips over vertex pairs.
* ``rmat``      R-MAT edge sampling (Chakrabarti et al.), seeded vertex relabelling.
* ``chung_lu``  power-law expected-degree graphs (Chung-Lu), degree cap sqrt(sum w).
* ``forest_fire`` the Forest Fire growth model (Leskovec, Kleinberg, Faloutsos),
                symmetrised.
* small structured graphs (path, star, clique, grid, tree, disjoint unions).

Directed variants (``directed=True`` on ``rmat``, ``forest_fire``, ``er``,
``chung_lu``, ``path`` and ``cycle``) keep the sampled arcs as they are:
self loops and repeated arcs are dropped, and every arc draws its own weight.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` only, so
the same seed gives the same arrays on every machine.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

NOT_FACILITY = 0xFFFFFFFF


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray                 # uint64 [n+1]
    col: np.ndarray                     # uint32 [n_arcs], strictly increasing per row
    w: Optional[np.ndarray] = None      # uint32 [n_arcs] or None (unit weights)
    fac_cost: Optional[np.ndarray] = None   # uint32 [n], NOT_FACILITY marks non-facilities
    is_client: Optional[np.ndarray] = None  # uint8 [n] or None (every vertex a client)
    name: str = ""
    meta: dict = field(default_factory=dict)
    directed: bool = False              # rows are out-arcs of a directed graph

    @property
    def n_arcs(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


# --------------------------------------------------------------------------
# edge lists -> symmetric CSR
# --------------------------------------------------------------------------
def _sort_keys(keys: np.ndarray) -> np.ndarray:
    """Sorted unique uint64 keys.  Uses torch's multithreaded sort when it is
    available (same result as numpy: a sorted unique set is unique)."""
    if keys.shape[0] > (1 << 22):
        try:
            import torch
            t = torch.from_numpy(keys.view(np.int64))
            # keys < 2^63 here (vertex ids < 2^31), so signed order == unsigned order
            t = torch.unique(t, sorted=True)
            return t.numpy().view(np.uint64)
        except Exception:  # pragma: no cover - torch missing
            pass
    return np.unique(keys)


def from_edges(n: int, u: np.ndarray, v: np.ndarray, wmax: Optional[int] = None,
               rng: Optional[np.random.Generator] = None, name: str = "") -> Graph:
    """Undirected simple graph from an edge list: self loops and duplicate
    edges are dropped, then every edge gets a weight uniform in 1..wmax (None:
    unit weights), drawn in sorted edge order, and both arcs are stored."""
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    keys = _sort_keys((a << np.uint64(32)) | b)
    a = (keys >> np.uint64(32)).astype(np.uint32)
    b = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    m = a.shape[0]
    w_edge = None
    if wmax is not None:
        if rng is None:
            raise ValueError("weights need a generator")
        w_edge = rng.integers(1, wmax + 1, size=m, dtype=np.uint32)
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order_keys = (src.astype(np.uint64) << np.uint64(32)) | dst.astype(np.uint64)
    order = _argsort_u64(order_keys)
    col = dst[order]
    counts = np.bincount(src, minlength=n).astype(np.uint64)
    row_ptr = np.zeros(n + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    w = None
    if w_edge is not None:
        w = np.concatenate([w_edge, w_edge])[order]
    return Graph(n=n, row_ptr=row_ptr, col=np.ascontiguousarray(col, np.uint32),
                 w=None if w is None else np.ascontiguousarray(w, np.uint32), name=name,
                 meta={"edges": int(m)})


def from_arcs(n: int, u: np.ndarray, v: np.ndarray, wmax: Optional[int] = None,
              rng: Optional[np.random.Generator] = None, name: str = "") -> Graph:
    """Directed simple graph from an arc list u -> v: self loops and repeated
    arcs are dropped, then every arc gets a weight uniform in 1..wmax (None:
    unit weights), drawn in sorted arc order.  Rows hold out-arcs."""
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    keep = u != v
    keys = _sort_keys((u[keep] << np.uint64(32)) | v[keep])
    src = (keys >> np.uint64(32)).astype(np.uint32)
    col = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    m = src.shape[0]
    w = None
    if wmax is not None:
        if rng is None:
            raise ValueError("weights need a generator")
        w = rng.integers(1, wmax + 1, size=m, dtype=np.uint32)
    counts = np.bincount(src, minlength=n).astype(np.uint64)
    row_ptr = np.zeros(n + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=np.ascontiguousarray(col, np.uint32),
                 w=None if w is None else np.ascontiguousarray(w, np.uint32), name=name,
                 meta={"arcs": int(m)}, directed=True)


def _build(directed, n, u, v, wmax, rng, name):
    if directed:
        return from_arcs(n, u, v, wmax, rng, name="d" + name)
    return from_edges(n, u, v, wmax, rng, name=name)


def reverse(g: Graph) -> Graph:
    """The graph with every arc turned around (weights kept), rows sorted."""
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr.astype(np.int64)))
    keys = (g.col.astype(np.uint64) << np.uint64(32)) | src
    order = _argsort_u64(keys)
    col = src[order].astype(np.uint32)
    counts = np.bincount(g.col, minlength=g.n).astype(np.uint64)
    row_ptr = np.zeros(g.n + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    w = None if g.w is None else np.ascontiguousarray(g.w[order], np.uint32)
    return Graph(n=g.n, row_ptr=row_ptr, col=np.ascontiguousarray(col), w=w, fac_cost=g.fac_cost,
                 is_client=g.is_client, name="rev_" + g.name, directed=g.directed)


def _argsort_u64(keys: np.ndarray) -> np.ndarray:
    if keys.shape[0] > (1 << 22):
        try:
            import torch
            t = torch.from_numpy(keys.view(np.int64))
            return torch.argsort(t, stable=True).numpy()
        except Exception:  # pragma: no cover
            pass
    return np.argsort(keys, kind="stable")


# --------------------------------------------------------------------------
# graph families
# --------------------------------------------------------------------------
def er(n: int, avg_deg: float, seed: int, wmax: Optional[int] = None, directed: bool = False) -> Graph:
    """G(n, p) with p = avg_deg / (n - 1): geometric skips over the pairs
    i < j in row-major order.  Directed: each of the n(n-1) ordered pairs is
    an arc with probability p (avg_deg is then the mean out-degree)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = avg_deg / (n - 1)
    if directed:
        nord = n * (n - 1)
        cnt = int(rng.binomial(nord, p))
        idx = np.sort(rng.choice(nord, size=cnt, replace=False)).astype(np.int64)
        i = idx // (n - 1)
        j = idx % (n - 1)
        j = j + (j >= i)                            # skip the diagonal
        return from_arcs(n, i, j, wmax, rng, name=f"der_n{n}_d{avg_deg}")
    npairs = n * (n - 1) // 2
    pos = []
    cur = -1
    while True:
        gaps = rng.geometric(p, size=max(1024, int(npairs * p * 1.2) + 16))
        idx = cur + np.cumsum(gaps)
        pos.append(idx[idx < npairs])
        if idx[-1] >= npairs:
            break
        cur = int(idx[-1])
    idx = np.concatenate(pos).astype(np.int64)
    # pair index -> (i, j), i < j, row-major over the strict upper triangle
    # row i starts at S(i) = i*(2n - i - 1)/2
    i = np.floor(((2 * n - 1) - np.sqrt((2.0 * n - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
    start = i * (2 * n - i - 1) // 2
    fix_hi = idx < start
    i[fix_hi] -= 1
    start = i * (2 * n - i - 1) // 2
    nxt = (i + 1) * (2 * n - i - 2) // 2
    fix_lo = idx >= nxt
    i[fix_lo] += 1
    start = i * (2 * n - i - 1) // 2
    j = idx - start + i + 1
    return from_edges(n, i, j, wmax, rng, name=f"er_n{n}_d{avg_deg}")


def rmat(scale: int, n_samples: int, seed: int, abcd=(0.57, 0.19, 0.19, 0.05),
         wmax: Optional[int] = None, chunk: int = 1 << 24, directed: bool = False) -> Graph:
    """R-MAT: each sample picks one quadrant per level with probabilities
    (a, b, c, d); vertices are relabelled by a seeded permutation; self loops
    and duplicates are dropped and the graph is symmetrised (directed: each
    sample is an arc, row -> column)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b, c, _ = abcd
    n = 1 << scale
    us, vs = [], []
    left = n_samples
    while left > 0:
        m = min(chunk, left)
        u = np.zeros(m, np.uint32)
        v = np.zeros(m, np.uint32)
        for lvl in range(scale):
            r = rng.random(m)
            bit = np.uint32(1 << (scale - 1 - lvl))
            down = r >= (a + b)                      # quadrants c, d: source bit
            right = ((r >= a) & (r < a + b)) | (r >= a + b + c)   # quadrants b, d
            u |= down.astype(np.uint32) * bit
            v |= right.astype(np.uint32) * bit
        us.append(u)
        vs.append(v)
        left -= m
    u = np.concatenate(us)
    v = np.concatenate(vs)
    perm = rng.permutation(n).astype(np.uint32)
    u = perm[u]
    v = perm[v]
    return _build(directed, n, u, v, wmax, rng, f"rmat_s{scale}_m{n_samples}")


def forest_fire(n: int, seed: int, p_fwd: float = 0.3, p_bwd: float = 0.4,
                wmax: Optional[int] = None, max_burn: int = 4096, directed: bool = False) -> Graph:
    """Forest Fire (Leskovec, Kleinberg, Faloutsos, KDD 2005): vertex v links
    to a uniformly chosen earlier ambassador, then spreads from each newly
    reached vertex x to Geometric(mean p/(1-p)) of x's unvisited out-neighbours
    (forward burning p_fwd) and in-neighbours (backward burning p_bwd),
    linking to each; at most max_burn vertices per arrival.  The links point
    from the new vertex to the earlier ones; they are symmetrised unless
    directed.  Pure Python: meant for n up to about 10^5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out_adj = [[] for _ in range(n)]
    in_adj = [[] for _ in range(n)]
    us, vs = [], []

    def pick(cands, count):
        if count <= 0 or not cands:
            return []
        if count >= len(cands):
            return cands
        idx = rng.choice(len(cands), size=count, replace=False)
        return [cands[i] for i in idx]

    for v in range(1, n):
        amb = int(rng.integers(0, v))
        visited = {v, amb}
        frontier = [amb]
        linked = [amb]
        while frontier and len(linked) < max_burn:
            nxt = []
            for x in frontier:
                nf = int(rng.geometric(1.0 - p_fwd)) - 1
                nb = int(rng.geometric(1.0 - p_bwd)) - 1
                chosen = pick([y for y in out_adj[x] if y not in visited], nf)
                chosen += pick([y for y in in_adj[x] if y not in visited and y not in chosen], nb)
                for y in chosen:
                    if len(linked) >= max_burn:
                        break
                    visited.add(y)
                    linked.append(y)
                    nxt.append(y)
            frontier = nxt
        for y in linked:
            out_adj[v].append(y)
            in_adj[y].append(v)
            us.append(v)
            vs.append(y)
    u = np.asarray(us, np.uint32)
    w_ = np.asarray(vs, np.uint32)
    perm = rng.permutation(n).astype(np.uint32)
    return _build(directed, n, perm[u], perm[w_], wmax, rng, f"ff_n{n}_p{p_fwd}_{p_bwd}")


def chung_lu(n: int, seed: int, exponent: float = 2.2, avg_deg: float = 10.0,
             wmax: Optional[int] = None, directed: bool = False) -> Graph:
    """Chung-Lu power law: expected degrees w_i proportional to
    (i + 1)^(-1/(exponent-1)), scaled to the average degree and capped at
    sqrt(sum w); n*avg/2 endpoint pairs drawn proportionally to w, then
    cleaned (so the realised average degree is a little lower)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.arange(n, dtype=np.float64)
    wts = (i + 1.0) ** (-1.0 / (exponent - 1.0))
    wts *= avg_deg / wts.mean()
    cap = np.sqrt(wts.sum())
    wts = np.minimum(wts, cap)
    prob = wts / wts.sum()
    m = int(round(n * avg_deg / 2))
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    u = np.searchsorted(cdf, rng.random(m), side="right").astype(np.uint32)
    v = np.searchsorted(cdf, rng.random(m), side="right").astype(np.uint32)
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    perm = rng.permutation(n).astype(np.uint32)
    return _build(directed, n, perm[u], perm[v], wmax, rng, f"cl_n{n}_d{avg_deg}")


def path(n, wmax=None, seed=0, directed=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.arange(n - 1)
    return _build(directed, n, i, i + 1, wmax, rng, f"path{n}")


def cycle(n, wmax=None, seed=0, directed=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.arange(n)
    return _build(directed, n, i, (i + 1) % n, wmax, rng, f"cycle{n}")


def star(n, wmax=None, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.arange(1, n)
    return from_edges(n, np.zeros(n - 1, np.int64), i, wmax, rng, name=f"star{n}")


def clique(n, wmax=None, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j, wmax, rng, name=f"clique{n}")


def grid(rows, cols, wmax=None, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.arange(rows * cols).reshape(rows, cols)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(rows * cols, u, v, wmax, rng, name=f"grid{rows}x{cols}")


def random_tree(n, seed, wmax=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    return from_edges(n, np.arange(1, n), parent, wmax, rng, name=f"tree{n}")


def empty(n, directed=False):
    return Graph(n=n, row_ptr=np.zeros(n + 1, np.uint64), col=np.zeros(0, np.uint32), name=f"empty{n}",
                 directed=directed)


def disjoint_union(*gs: Graph) -> Graph:
    """Side-by-side union; the parts must be all directed or all undirected."""
    if len({bool(g.directed) for g in gs}) > 1:
        raise ValueError("mixing directed and undirected parts")
    n = sum(g.n for g in gs)
    rp = [np.zeros(1, np.uint64)]
    cols, ws = [], []
    vo = 0
    ao = 0
    weighted = any(g.w is not None for g in gs)
    for g in gs:
        rp.append(g.row_ptr[1:] + np.uint64(ao))
        cols.append(g.col + np.uint32(vo))
        if weighted:
            ws.append(g.w if g.w is not None else np.ones(g.n_arcs, np.uint32))
        vo += g.n
        ao += g.n_arcs
    return Graph(n=n, row_ptr=np.concatenate(rp), col=np.concatenate(cols).astype(np.uint32),
                 w=np.concatenate(ws).astype(np.uint32) if weighted else None,
                 name="+".join(g.name for g in gs), directed=bool(gs[0].directed) if gs else False)


# --------------------------------------------------------------------------
# facilities, costs, clients
# --------------------------------------------------------------------------
def with_problem(g: Graph, seed: int, cost: str = "uniform", cost_lo: int = 1, cost_hi: int = 1000,
                 const_cost: int = 50, fac_frac: float = 1.0, client_frac: float = 1.0,
                 lognormal=(5.0, 1.0)) -> Graph:
    """Attach facility opening costs and a client set.  fac_frac < 1 picks an
    exact, seeded fraction of the vertices as facilities; the rest get
    NOT_FACILITY.  client_frac < 1 likewise picks the clients."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    n = g.n
    if cost == "uniform":
        c = rng.integers(cost_lo, cost_hi + 1, size=n, dtype=np.uint64)
    elif cost == "const":
        c = np.full(n, const_cost, np.uint64)
    elif cost == "lognormal":
        mu, sigma = lognormal
        c = np.maximum(1, np.rint(np.exp(mu + sigma * rng.standard_normal(n)))).astype(np.uint64)
    else:
        raise ValueError(cost)
    c = np.minimum(c, NOT_FACILITY - 1).astype(np.uint32)
    if fac_frac < 1.0:
        nf = int(round(fac_frac * n))
        fac = np.zeros(n, bool)
        fac[rng.permutation(n)[:nf]] = True
        c = np.where(fac, c, np.uint32(NOT_FACILITY)).astype(np.uint32)
    g.fac_cost = c
    if client_frac < 1.0:
        ncl = int(round(client_frac * n))
        cl = np.zeros(n, np.uint8)
        cl[rng.permutation(n)[:ncl]] = 1
        g.is_client = cl
    else:
        g.is_client = None
    return g


def with_facilities(g: Graph, ids, costs, client_mask=None) -> Graph:
    """Only the listed vertices are facilities, with the given opening costs
    (a scalar or one per id); every vertex is a client unless client_mask
    (uint8 [n]) says otherwise.  Few cheap facilities far from most clients
    make every facility open while some clients are still unfrozen."""
    c = np.full(g.n, NOT_FACILITY, np.uint32)
    c[np.asarray(ids, np.int64)] = np.asarray(costs, np.uint32)
    g.fac_cost = c
    g.is_client = None if client_mask is None else np.ascontiguousarray(client_mask, np.uint8)
    return g


def end_phase_problems():
    """Small problems whose opening loop ends with every facility open and
    clients left unfrozen (each returned with a short name)."""
    return [
        ("path 30, one facility at an end", with_facilities(path(30), [0], 1)),
        ("grid 12x12 w1..9, three corner facilities",
         with_facilities(grid(12, 12, wmax=9, seed=3), [0, 11, 143], [2, 3, 2])),
        ("path 40 w1..5, facilities 0, 1, 39", with_facilities(path(40, wmax=5, seed=2), [0, 1, 39], 1)),
        ("ER 300 w1..20, five facilities, unreachable clients",
         with_facilities(er(300, 3, 4, wmax=20), [3, 50, 100, 200, 250], [1, 2, 3, 4, 5])),
        ("directed path 30, facility at the far end", with_facilities(path(30, directed=True), [29], 1)),
        ("directed cycle 40 w1..7, two facilities",
         with_facilities(cycle(40, wmax=7, seed=1, directed=True), [0, 20], 1)),
    ]


# --------------------------------------------------------------------------
# the benchmark workloads (names describe the workload and its sizes)
# --------------------------------------------------------------------------
def rmat_weighted_fac10(scale: int = 24, edge_factor: int = 16, seed: int = 1) -> Graph:
    """R-MAT 2^scale with edge_factor * 2^scale edge samples (average degree
    about 2 * edge_factor), weights uniform 1..100, 10% of the vertices
    facilities (seeded) with opening costs lognormal(5, 1) rounded to
    integers, every vertex a client."""
    g = rmat(scale, edge_factor << scale, seed, wmax=100)
    return with_problem(g, seed, cost="lognormal", fac_frac=0.1)


def tiny_er(seed: int = 1) -> Graph:
    """Erdos-Renyi n=2,000, average degree 8, weights 1..10, every vertex a
    client and a facility of cost 50."""
    g = er(2000, 8.0, seed, wmax=10)
    return with_problem(g, seed, cost="const", const_cost=50)


def rmat_unit(scale: int = 22, edge_factor: int = 16, seed: int = 1) -> Graph:
    """R-MAT (0.57, 0.19, 0.19, 0.05), 2^scale vertices, edge_factor * 2^scale
    edge samples, unit weights, all vertices clients and facilities, costs
    uniform 1..1000 (the 2^22, 64M-edge graph at the defaults)."""
    g = rmat(scale, edge_factor << scale, seed)
    return with_problem(g, seed, cost="uniform", cost_lo=1, cost_hi=1000)


def rmat_unit_directed(scale: int = 22, edge_factor: int = 16, seed: int = 1) -> Graph:
    """The same R-MAT samples kept as arcs (row -> column; self loops and
    repeats dropped), unit weights, all vertices clients and facilities,
    costs uniform 1..1000."""
    g = rmat(scale, edge_factor << scale, seed, directed=True)
    return with_problem(g, seed, cost="uniform", cost_lo=1, cost_hi=1000)


def rmat_weighted(scale: int = 24, avg_deg: int = 32, seed: int = 1) -> Graph:
    """R-MAT (0.57, 0.19, 0.19, 0.05), 2^scale vertices, avg_deg/2 * 2^scale
    edge samples, weights 1..100, 10% facilities (seeded) with lognormal(5, 1)
    costs, every vertex a client."""
    g = rmat(scale, (avg_deg // 2) << scale, seed, wmax=100)
    return with_problem(g, seed, cost="lognormal", fac_frac=0.10)


def powerlaw_batch(count: int, seed: int, n_lo: int = 500, n_hi: int = 200_000,
                   avg_deg: float = 10.0, wmax: int = 20):
    """count Chung-Lu graphs (exponent 2.2), n log-uniform in [n_lo, n_hi],
    weights 1..wmax, all vertices clients and facilities, costs 1..1000."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).astype(np.int64)
    out = []
    for i, nn in enumerate(ns):
        g = chung_lu(int(nn), seed * 1_000_003 + i, 2.2, avg_deg, wmax)
        out.append(with_problem(g, seed * 7919 + i, cost="uniform"))
    return out


def poisson_requests(count: int, seed: int, rate: float = 200.0, n_lo: int = 1000,
                     n_hi: int = 500_000, avg_deg: float = 12.0, wmax: int = 50):
    """Arrival times (seconds) of a Poisson stream and the graph of each request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    graphs = powerlaw_batch(count, seed + 17, n_lo, n_hi, avg_deg, wmax)
    return arrivals, graphs
