"""GPU: the HIP-estimator read off the GPU sketches (Sec. 3.3; the accuracy
experiment of Sec. 5.1 on a small graph).  Exact ball sizes come from scipy,
not from the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch
from scipy.sparse.csgraph import dijkstra

import graphgen as gg
import paper_1503_03635_amd as fl

pytestmark = pytest.mark.gpu


def _estimates(g, k, seed, vs, dists):
    s = fl.ads_build(fl.to_device(g), k, seed)
    torch.cuda.synchronize()
    off = s["off"].cpu().numpy().view(np.uint64).astype(np.int64)
    dist = s["dist"].cpu().numpy().view(np.uint32).astype(np.float64)
    thr = s["thresh"].cpu().numpy().view(np.uint32).astype(np.float64)
    a = np.where(thr == 0, 1.0, 4294967296.0 / np.maximum(thr, 1.0))
    return np.array([[a[off[v]:off[v + 1]][dist[off[v]:off[v + 1]] <= d].sum() for d in dists] for v in vs])


def _exact(g, vs, dists):
    w = g.w if g.w is not None else np.ones(g.n_arcs, np.uint32)
    A = sp.csr_matrix((w.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    D = dijkstra(A, directed=True, indices=vs)
    return np.array([[np.count_nonzero(D[i] <= d) for d in dists] for i in range(len(vs))], np.float64)


@pytest.mark.parametrize("weighted", [False, True])
def test_hip_estimate_error_below_half(weighted):
    """Mean relative error of N(v, d) stays well below the paper's 50%."""
    g = gg.rmat(11, 16 << 11, 4, wmax=100 if weighted else None)
    dists = list(range(100, 1001, 100)) if weighted else list(range(1, 8))
    vs = np.random.Generator(np.random.PCG64(1)).choice(np.nonzero(g.degrees() > 0)[0], 60, replace=False)
    est, ex = _estimates(g, 16, 3, vs, dists), _exact(g, vs, dists)
    rel = np.abs(est - ex) / ex
    print(f"[accuracy] weighted={weighted} mean relative error {rel.mean():.3f}", flush=True)
    assert rel.mean() < 0.5


def test_hip_estimate_exact_when_k_covers_graph():
    """k >= n: every weight is 1 and the estimate is the exact ball size."""
    g = gg.er(300, 5, 2, wmax=7)
    dists = [1, 3, 7, 15, 40]
    vs = np.arange(0, 300, 7)
    est, ex = _estimates(g, 64 if g.n <= 64 else 64, 5, vs, dists), _exact(g, vs, dists)
    small = ex <= 64                      # balls of at most k vertices are counted exactly
    assert np.array_equal(est[small], ex[small])
