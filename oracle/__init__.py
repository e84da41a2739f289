"""Plain CPU oracle for sketch-based facility location (arXiv 1503.03635).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the HIP
library under ``paper_1503_03635_amd``; the C source ``fl_oracle.c`` cites the
passage of the paper each function follows.

The Python layer below is argument marshalling only (ctypes), plus a few tiny
conveniences that reshape the C results into numpy arrays.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

RUNG_NONE = 0xFFFFFFFF
RUNG_GUARD = 0xFFFFFFFE
RUNG_END = 0xFFFFFFFD
NONE = 0xFFFFFFFF
NOT_FACILITY = 0xFFFFFFFF

OK, EINVAL, ERANGE, ENOMEM, EINTERNAL = 0, 1, 2, 3, 99

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = C.CDLL(path)
        _setup(_lib)
    return _lib


class _Graph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_arcs", C.c_uint64),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("w", C.c_void_p),
                ("fac_cost", C.c_void_p), ("is_client", C.c_void_p), ("directed", C.c_uint32)]


class _Sketch(C.Structure):
    _fields_ = [("off", C.POINTER(C.c_uint64)), ("rank", C.POINTER(C.c_uint32)),
                ("dist", C.POINTER(C.c_uint32)), ("id", C.POINTER(C.c_uint32))]


class _Result(C.Structure):
    _fields_ = [("open", C.c_void_p), ("assign", C.c_void_p), ("dist", C.c_void_p),
                ("open_rung", C.c_void_p), ("freeze_rung", C.c_void_p), ("q", C.c_void_p),
                ("total_cost", C.c_uint64),
                ("n_open", C.c_uint32), ("n_unreachable", C.c_uint32), ("n_rungs", C.c_uint32),
                ("mis_rounds", C.c_uint32), ("n_guard", C.c_uint32),
                ("relax_alg", C.c_uint64), ("ads_entries", C.c_uint64), ("gamma", C.c_uint64),
                ("alpha0", C.c_double), ("one_eps", C.c_double), ("n_reach_guard", C.c_uint32)]


def _setup(L):
    L.orc_splitmix64.restype = C.c_uint64
    L.orc_splitmix64.argtypes = [C.c_uint64]
    L.orc_perm.restype = C.c_uint32
    L.orc_perm.argtypes = [C.c_uint32, C.c_uint64]
    L.orc_perm_inv.restype = C.c_uint32
    L.orc_perm_inv.argtypes = [C.c_uint32, C.c_uint64]
    L.orc_rank_key.restype = C.c_uint64
    L.orc_rank_key.argtypes = [C.c_uint64]
    L.orc_prio_key.restype = C.c_uint64
    L.orc_prio_key.argtypes = [C.c_uint64]
    L.orc_ranks.argtypes = [C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p]
    L.orc_perm_check_range.restype = C.c_int
    L.orc_perm_check_range.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
    L.orc_validate.argtypes = [C.POINTER(_Graph), C.c_uint32, C.c_double]
    for name in ("orc_ads_brute", "orc_ads_pruned"):
        getattr(L, name).argtypes = [C.POINTER(_Graph), C.c_void_p, C.c_uint32, C.POINTER(_Sketch)]
    L.orc_ads_pruned_ex.argtypes = [C.POINTER(_Graph), C.c_void_p, C.c_uint32, C.POINTER(_Sketch),
                                    C.c_uint64, C.POINTER(C.c_uint64)]
    L.orc_ads_rounds.argtypes = [C.POINTER(_Graph), C.c_void_p, C.c_uint32, C.POINTER(_Sketch),
                                 C.POINTER(C.c_uint32)]
    L.orc_sketch_free.argtypes = [C.POINTER(_Sketch)]
    L.orc_prune.restype = C.c_uint32
    L.orc_prune.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32]
    L.orc_hipest.argtypes = [C.POINTER(_Sketch), C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]
    L.orc_solve.argtypes = [C.POINTER(_Graph), C.c_uint32, C.c_uint64, C.c_double, C.POINTER(_Result)]
    L.orc_ads_one.argtypes = [C.POINTER(_Graph), C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p,
                              C.c_uint32, C.POINTER(C.c_uint32)]
    L.orc_solve_luby.argtypes = [C.POINTER(_Graph), C.c_uint32, C.c_uint64, C.c_double, C.POINTER(_Result)]
    L.orc_opt_exhaustive.argtypes = [C.POINTER(_Graph), C.POINTER(C.c_uint64)]
    L.orc_sssp.argtypes = [C.POINTER(_Graph), C.c_uint32, C.c_void_p]
    L.orc_ladder.argtypes = [C.c_double, C.c_double, C.c_uint32, C.c_void_p]


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Held:
    """Keeps the numpy arrays behind a _Graph alive."""

    def __init__(self, g):
        self.row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
        self.col = np.ascontiguousarray(g.col, dtype=np.uint32)
        self.w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.uint32)
        fc = getattr(g, "fac_cost", None)
        self.fac_cost = None if fc is None else np.ascontiguousarray(fc, dtype=np.uint32)
        ic = getattr(g, "is_client", None)
        self.is_client = None if ic is None else np.ascontiguousarray(ic, dtype=np.uint8)
        self.s = _Graph(int(g.n), int(self.col.shape[0]), _ptr(self.row_ptr), _ptr(self.col),
                        _ptr(self.w), _ptr(self.fac_cost), _ptr(self.is_client),
                        1 if getattr(g, "directed", False) else 0)


def _sketch_to_numpy(sk, n):
    off = np.ctypeslib.as_array(sk.off, shape=(n + 1,)).copy()
    tot = int(off[-1])
    m = max(tot, 1)
    rank = np.ctypeslib.as_array(sk.rank, shape=(m,))[:tot].copy()
    dist = np.ctypeslib.as_array(sk.dist, shape=(m,))[:tot].copy()
    ids = np.ctypeslib.as_array(sk.id, shape=(m,))[:tot].copy()
    return {"off": off, "rank": rank, "dist": dist, "id": ids}


def splitmix64(x):
    return int(lib().orc_splitmix64(x))


def perm(v, key):
    return int(lib().orc_perm(v, key))


def perm_inv(r, key):
    return int(lib().orc_perm_inv(r, key))


def rank_key(seed):
    return int(lib().orc_rank_key(seed))


def prio_key(seed):
    return int(lib().orc_prio_key(seed))


def perm_check_range(key, lo, count):
    return bool(lib().orc_perm_check_range(key, lo, count))


def ranks(n, seed):
    r = np.empty(n, np.uint32)
    p = np.empty(n, np.uint32)
    lib().orc_ranks(n, seed, _ptr(r), _ptr(p))
    return r, p


def validate(g, k, eps):
    h = _Held(g)
    return int(lib().orc_validate(C.byref(h.s), k, eps))


def _ads(fn, g, k, seed=None, rank=None):
    if rank is None:
        rank, _ = ranks(g.n, seed)
    rank = np.ascontiguousarray(rank, dtype=np.uint32)
    h = _Held(g)
    sk = _Sketch()
    rc = fn(C.byref(h.s), _ptr(rank), k, C.byref(sk))
    if rc != OK:
        raise RuntimeError(f"oracle ADS failed: {rc}")
    out = _sketch_to_numpy(sk, g.n)
    lib().orc_sketch_free(C.byref(sk))
    return out


def ads_brute(g, k, seed=None, rank=None):
    """Alg. 1 with the (distance, id) order, one Dijkstra per vertex."""
    return _ads(lib().orc_ads_brute, g, k, seed, rank)


def ads_pruned(g, k, seed=None, rank=None):
    """Pruned Dijkstra, sources in increasing rank."""
    return _ads(lib().orc_ads_pruned, g, k, seed, rank)


def ads_pruned_timed(g, k, seed, max_sources):
    """Pruned Dijkstra over the first max_sources sources (rank order) only;
    returns the number of arc relaxations performed.  For CPU timing."""
    rank, _ = ranks(g.n, seed)
    h = _Held(g)
    cnt = C.c_uint64(0)
    rc = lib().orc_ads_pruned_ex(C.byref(h.s), _ptr(rank), k, None, max_sources, C.byref(cnt))
    if rc != OK:
        raise RuntimeError(f"oracle ADS failed: {rc}")
    return int(cnt.value)


def ads_one(g, k, seed, v, rank=None, cap=1 << 16):
    """The sketch of vertex v alone (Alg. 1 with the (distance, id) order):
    (ranks, distances) in sketch order."""
    h = _Held(g)
    if rank is None:
        rank, _ = ranks(g.n, seed)
    rank = np.ascontiguousarray(rank, np.uint32)
    out_r = np.zeros(cap, np.uint32)
    out_d = np.zeros(cap, np.uint32)
    cnt = C.c_uint32(0)
    rc = lib().orc_ads_one(C.byref(h.s), _ptr(rank), k, v, _ptr(out_r), _ptr(out_d), cap, C.byref(cnt))
    if rc != OK:
        raise RuntimeError(f"orc_ads_one failed: {rc}")
    m = int(cnt.value)
    return out_r[:m].copy(), out_d[:m].copy()


def ads_rounds(g, k, seed=None, rank=None):
    """Alg. 2 as synchronous supersteps with CleanUp every superstep."""
    if rank is None:
        rank, _ = ranks(g.n, seed)
    rank = np.ascontiguousarray(rank, dtype=np.uint32)
    h = _Held(g)
    sk = _Sketch()
    nr = C.c_uint32(0)
    rc = lib().orc_ads_rounds(C.byref(h.s), _ptr(rank), k, C.byref(sk), C.byref(nr))
    if rc != OK:
        raise RuntimeError(f"oracle ADS rounds failed: {rc}")
    out = _sketch_to_numpy(sk, g.n)
    out["rounds"] = int(nr.value)
    lib().orc_sketch_free(C.byref(sk))
    return out


def prune(d, ids, rk, k):
    d = np.array(d, dtype=np.uint64)
    ids = np.array(ids, dtype=np.uint32)
    rk = np.array(rk, dtype=np.uint32)
    m = lib().orc_prune(_ptr(d), _ptr(ids), _ptr(rk), len(d), k)
    return d[:m].copy(), ids[:m].copy(), rk[:m].copy()


def hipest(sk, k):
    """T_j (uint64, 2^32 when j < k) and a_j = 2^32 / T_j per entry."""
    n = len(sk["off"]) - 1
    off = np.ascontiguousarray(sk["off"], dtype=np.uint64)
    rank = np.ascontiguousarray(sk["rank"], dtype=np.uint32)
    tot = int(off[-1])
    T = np.empty(max(tot, 1), np.uint64)
    a = np.empty(max(tot, 1), np.float64)
    s = _Sketch(off.ctypes.data_as(C.POINTER(C.c_uint64)), rank.ctypes.data_as(C.POINTER(C.c_uint32)),
                None, None)
    lib().orc_hipest(C.byref(s), n, k, _ptr(T), _ptr(a))
    return T[:tot], a[:tot]


def solve(g, k, seed, eps=0.1, luby=False):
    """Full facility-location solve (luby=True: Luby's MIS variant with
    priorities redrawn every round).  Returns (rc, dict)."""
    n = g.n
    h = _Held(g)
    res = {
        "open": np.zeros(n, np.uint8), "assign": np.zeros(n, np.uint32),
        "dist": np.zeros(n, np.uint32), "open_rung": np.zeros(n, np.uint32),
        "freeze_rung": np.zeros(n, np.uint32), "q": np.zeros(n, np.float64),
    }
    r = _Result(_ptr(res["open"]), _ptr(res["assign"]), _ptr(res["dist"]),
                _ptr(res["open_rung"]), _ptr(res["freeze_rung"]), _ptr(res["q"]))
    fn = lib().orc_solve_luby if luby else lib().orc_solve
    rc = int(fn(C.byref(h.s), k, seed, eps, C.byref(r)))
    for name in ("total_cost", "n_open", "n_unreachable", "n_rungs", "mis_rounds", "n_guard",
                 "relax_alg", "ads_entries", "gamma", "alpha0", "one_eps", "n_reach_guard"):
        res[name] = getattr(r, name)
    return rc, res


def opt_exhaustive(g):
    h = _Held(g)
    best = C.c_uint64(0)
    rc = lib().orc_opt_exhaustive(C.byref(h.s), C.byref(best))
    if rc != OK:
        raise RuntimeError(f"exhaustive OPT failed: {rc}")
    return int(best.value)


def sssp(g, s):
    h = _Held(g)
    d = np.empty(g.n, np.uint64)
    lib().orc_sssp(C.byref(h.s), s, _ptr(d))
    return d


def ladder(alpha0, eps, count):
    out = np.empty(count, np.float64)
    lib().orc_ladder(alpha0, eps, count, _ptr(out))
    return out
