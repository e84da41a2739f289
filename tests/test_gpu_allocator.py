"""GPU: fl_set_allocator routes the library's device memory through caller
hooks (here torch's caching allocator).  Results equal those of the default
hipMalloc path; a failing hook is reported as FL_ENOMEM; hooks cannot change
while a server exists."""
import ctypes as C

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1503_03635_amd as fl

from gpu_util import gpu_sketch, gpu_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _restore_default():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    fl.use_torch_allocator(False)


def _same(a, b):
    for key in ("open", "assign", "dist", "open_rung", "freeze_rung"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["q"].view(np.uint64), b["q"].view(np.uint64))
    assert a["total_cost"] == b["total_cost"]


def test_torch_allocator_backs_the_workspace():
    g = gg.with_problem(gg.rmat(12, 16 << 12, 3, wmax=20), 3, cost="uniform")
    print("[alloc] default path", flush=True)
    want = gpu_solve(g, 16, 2)
    sk_want = gpu_sketch(g, 8, 4)
    fl.lib().fl_release_workspace()
    fl.use_torch_allocator(True)
    before = torch.cuda.memory_allocated()
    print("[alloc] torch allocator", flush=True)
    got = gpu_solve(g, 16, 2)
    held = torch.cuda.memory_allocated() - before
    assert held > 0                     # the cached workspace came from torch
    _same(got, want)
    sk = gpu_sketch(g, 8, 4)
    for key in ("off", "rank", "dist", "thresh"):
        assert np.array_equal(sk[key], sk_want[key]), key
    outs = fl.solve_batch([fl.to_device(g), fl.to_device(gg.with_problem(gg.er(300, 4, 5), 5))], 16, 2)
    torch.cuda.synchronize()
    assert outs[0]["total_cost"] == want["total_cost"]
    mid = torch.cuda.memory_allocated()
    fl.use_torch_allocator(False)       # releases the cached workspaces back to torch
    assert mid - torch.cuda.memory_allocated() >= held
    _same(gpu_solve(g, 16, 2), want)    # and the default path works again


def test_failing_hook_reports_enomem():
    L = fl.lib()
    L.fl_release_workspace()
    nothing = fl._lib.ALLOC_FN(lambda nbytes, dev, ctx: None)
    never = fl._lib.FREE_FN(lambda p, nbytes, dev, ctx: None)
    assert L.fl_set_allocator(C.cast(nothing, C.c_void_p), C.cast(never, C.c_void_p), None) == 0
    g = gg.with_problem(gg.er(200, 4, 1, wmax=5), 1)
    print("[alloc] failing hook", flush=True)
    r = fl.solve(fl.to_device(g), 8, 1, check=False)
    assert r["rc"] == fl._lib.FL_ENOMEM
    assert L.fl_set_allocator(None, None, None) == 0
    r = fl.solve(fl.to_device(g), 8, 1)
    assert r["n_open"] > 0


def test_hooks_refused_while_a_server_exists():
    srv = fl.Server(slots=1)
    try:
        f = fl._lib.ALLOC_FN(lambda nbytes, dev, ctx: None)
        fr = fl._lib.FREE_FN(lambda p, nbytes, dev, ctx: None)
        assert fl.lib().fl_set_allocator(C.cast(f, C.c_void_p), C.cast(fr, C.c_void_p), None) == fl._lib.FL_EBUSY
    finally:
        srv.close()
    assert fl.lib().fl_set_allocator(None, None, None) == 0
