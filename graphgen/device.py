"""Seeded synthetic inputs built on the GPU, for the benchmark-sized workloads.

The host generators in ``graphgen`` take minutes at these sizes (R-MAT with
2^24 vertices and 268M edge samples, a thousand power-law graphs).  The same
recipes are built here with torch on the device: every random draw comes from
one ``torch.Generator`` on that device seeded with the workload's seed
(Philox), so the same seed, sizes and device type give the same arrays run
after run.  The graphs differ from the host generators' (different random
streams), not in their recipe.  Like the rest of ``graphgen`` this module
builds inputs only and holds none of the method's arithmetic.

Outputs are DeviceGraph objects of the library's binding (int64 row_ptr,
int32 columns and weights, uint32 values stored in int32) plus host copies on
demand (``to_host``), which the tests hand to the CPU oracle.
"""
import numpy as np
import torch

NOT_FACILITY = 0xFFFFFFFF


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _mix32(x):
    """A 32-bit integer mixer (xor-shift / odd multiply, the lowbias32 family)
    on int64 tensors holding values below 2^32; used to give each undirected
    edge one weight from its two end points."""
    m = 0xFFFFFFFF
    x = (x ^ (x >> 16)) & m
    x = (x * 0x21F0AAAD) & m
    x = (x ^ (x >> 15)) & m
    x = (x * 0x735A2D97) & m
    x = (x ^ (x >> 15)) & m
    return x


def _edge_weight(a, b, wmax, seed):
    """Weight 1..wmax of the edge {a, b}: a function of the unordered pair and
    the seed, so both arcs of an edge carry it."""
    lo = torch.minimum(a, b)
    hi = torch.maximum(a, b)
    s = int(seed) & 0xFFFFFFFF
    h = _mix32((lo ^ s) & 0xFFFFFFFF)
    h = _mix32((h ^ hi) & 0xFFFFFFFF)
    h = _mix32((h ^ (s * 0x9E37 & 0xFFFFFFFF)) & 0xFFFFFFFF)
    return (h % int(wmax) + 1).to(torch.int32)


def _csr(n, row, col, device):
    """CSR from arcs already sorted by (row, col)."""
    counts = torch.bincount(row, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=row_ptr[1:])
    return row_ptr


def _arcs_from_pairs(n, u, v, directed, device):
    """Drop self loops and repeats; symmetrise unless directed; sort by
    (row, col).  u, v: int64 tensors."""
    keep = u != v
    u, v = u[keep], v[keep]
    if not directed:
        u, v = torch.cat([u, v]), torch.cat([v, u])
    key = torch.unique(u * n + v)          # sorted, distinct
    del u, v
    row = key // n
    col = key - row * n
    return row, col


def rmat(scale, n_samples, seed, abcd=(0.57, 0.19, 0.19, 0.05), wmax=None, directed=False, device="cuda:0",
         chunk=1 << 26):
    """R-MAT edge sampling (one quadrant per level with probabilities a, b,
    c, d), vertices relabelled by a seeded permutation, self loops and
    repeats dropped, symmetrised unless directed.  Returns (n, row_ptr, col,
    w or None) on the device."""
    gen = _gen(seed, device)
    a, b, c, _ = abcd
    n = 1 << scale
    us, vs = [], []
    left = int(n_samples)
    while left > 0:
        m = min(chunk, left)
        u = torch.zeros(m, dtype=torch.int64, device=device)
        v = torch.zeros(m, dtype=torch.int64, device=device)
        for lvl in range(scale):
            r = torch.rand(m, generator=gen, device=device, dtype=torch.float64)
            bit = 1 << (scale - 1 - lvl)
            down = r >= (a + b)
            right = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            u |= down.to(torch.int64) * bit
            v |= right.to(torch.int64) * bit
            del r, down, right
        us.append(u)
        vs.append(v)
        left -= m
    u = torch.cat(us)
    v = torch.cat(vs)
    del us, vs
    perm = torch.randperm(n, generator=gen, device=device)
    u = perm[u]
    v = perm[v]
    row, col = _arcs_from_pairs(n, u, v, directed, device)
    del u, v
    row_ptr = _csr(n, row, col, device)
    w = None
    if wmax is not None:
        if directed:
            w = (torch.randint(1, int(wmax) + 1, (col.shape[0],), generator=gen, device=device,
                               dtype=torch.int64)).to(torch.int32)
        else:
            w = _edge_weight(row, col, wmax, seed)
    del row
    return n, row_ptr, col.to(torch.int32), w


def _u32(c):
    """int64 values in [0, 2^32) stored bit for bit in an int32 tensor."""
    return torch.where(c >= (1 << 31), c - (1 << 32), c).to(torch.int32)


def _device_graph(n, row_ptr, col, w, fac_cost, directed):
    import paper_1503_03635_amd as fl
    return fl.DeviceGraph(n=n, row_ptr=row_ptr, col=col, w=w, fac_cost=fac_cost, is_client=None,
                          directed=directed)


def rmat_weighted_fac10(scale=24, avg_deg=32, seed=1, device="cuda:0"):
    """The large weighted workload: R-MAT 2^scale with avg_deg/2 * 2^scale edge
    samples, weights 1..100, a seeded 10% of the vertices facilities with
    lognormal(5, 1) costs rounded to integers, every vertex a client."""
    n, rp, col, w = rmat(scale, (avg_deg // 2) << scale, seed, wmax=100, device=device)
    fc = _u32(problem_i64(n, seed, cost="lognormal", fac_frac=0.1, device=device))
    return _device_graph(n, rp, col, w, fc, False)


def rmat_unit(scale=22, edge_factor=16, seed=1, directed=False, device="cuda:0"):
    """R-MAT 2^scale with edge_factor * 2^scale edge samples, unit weights,
    every vertex a client and a facility with cost uniform 1..1000 (directed:
    the samples kept as arcs)."""
    n, rp, col, _ = rmat(scale, edge_factor << scale, seed, directed=directed, device=device)
    fc = _u32(problem_i64(n, seed, cost="uniform", device=device))
    return _device_graph(n, rp, col, None, fc, directed)


def problem_i64(n, seed, **kw):
    """Facility costs as int64 values: uniform integers or lognormal(mu,
    sigma) rounded (at least 1); with fac_frac < 1 an exact seeded fraction of
    the vertices are facilities and the rest get NOT_FACILITY.  Every vertex is
    a client."""
    device = kw.pop("device", "cuda:0")
    gen = _gen(int(seed) ^ 0x5EED, device)
    cost = kw.get("cost", "uniform")
    if cost == "uniform":
        c = torch.randint(kw.get("cost_lo", 1), kw.get("cost_hi", 1000) + 1, (n,), generator=gen, device=device,
                          dtype=torch.int64)
    elif cost == "lognormal":
        mu, sigma = kw.get("lognormal", (5.0, 1.0))
        z = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
        c = torch.clamp(torch.round(torch.exp(mu + sigma * z)), min=1, max=NOT_FACILITY - 1).to(torch.int64)
    else:
        raise ValueError(cost)
    ff = kw.get("fac_frac", 1.0)
    if ff < 1.0:
        nf = int(round(ff * n))
        fac = torch.zeros(n, dtype=torch.bool, device=device)
        fac[torch.randperm(n, generator=gen, device=device)[:nf]] = True
        c = torch.where(fac, c, torch.full_like(c, NOT_FACILITY))
    return c


def chung_lu(n, seed, exponent=2.2, avg_deg=10.0, wmax=None, device="cuda:0"):
    """Chung-Lu power law on the device: expected degrees proportional to
    (i + 1)^(-1/(exponent - 1)), scaled to avg_deg and capped at sqrt(sum);
    n * avg_deg / 2 end-point pairs drawn in proportion, relabelled by a
    seeded permutation, then cleaned and symmetrised.  Returns (n, row_ptr,
    col, w or None)."""
    gen = _gen(seed, device)
    i = torch.arange(n, dtype=torch.float64, device=device)
    wts = (i + 1.0) ** (-1.0 / (exponent - 1.0))
    wts = wts * (avg_deg * n / wts.sum())
    wts = torch.clamp(wts, max=float(torch.sqrt(wts.sum())))
    cdf = torch.cumsum(wts, 0)
    cdf = cdf / cdf[-1]
    m = int(n * avg_deg / 2)
    u = torch.searchsorted(cdf, torch.rand(m, generator=gen, device=device, dtype=torch.float64))
    v = torch.searchsorted(cdf, torch.rand(m, generator=gen, device=device, dtype=torch.float64))
    u = torch.clamp(u, max=n - 1)
    v = torch.clamp(v, max=n - 1)
    perm = torch.randperm(n, generator=gen, device=device)
    row, col = _arcs_from_pairs(n, perm[u], perm[v], False, device)
    rp = _csr(n, row, col, device)
    w = _edge_weight(row, col, wmax, seed) if wmax is not None else None
    return n, rp, col.to(torch.int32), w


def powerlaw_batch(count, seed, n_lo=500, n_hi=200_000, avg_deg=10.0, wmax=20, device="cuda:0"):
    """count Chung-Lu graphs (exponent 2.2), n log-uniform in [n_lo, n_hi]
    (drawn on the host from numpy's PCG64 with the seed), weights 1..wmax,
    every vertex a client and a facility with costs uniform 1..1000."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).astype(np.int64)
    out = []
    for j, nn in enumerate(ns):
        n, rp, col, w = chung_lu(int(nn), seed * 1_000_003 + j, 2.2, avg_deg, wmax, device=device)
        fc = _u32(problem_i64(n, seed * 7919 + j, cost="uniform", device=device))
        out.append(_device_graph(n, rp, col, w, fc, False))
    return out


def poisson_requests(count, seed, rate=200.0, n_lo=1000, n_hi=500_000, avg_deg=12.0, wmax=50, device="cuda:0"):
    """Arrival times (seconds, exponential gaps at `rate`) and the device
    graph of each request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    return arrivals, powerlaw_batch(count, seed + 17, n_lo, n_hi, avg_deg, wmax, device=device)


def to_host(dg):
    """Host copy of a device graph as a graphgen.Graph (for the CPU oracle)."""
    import graphgen as gg
    rp = dg.row_ptr.cpu().numpy().astype(np.uint64)
    col = dg.col.cpu().numpy().view(np.uint32).copy()
    w = None if dg.w is None else dg.w.cpu().numpy().view(np.uint32).copy()
    fc = dg.fac_cost.cpu().numpy().view(np.uint32).copy()
    return gg.Graph(int(dg.n), rp, col, w, fc, None, name="device", directed=bool(dg.directed))
