"""ctypes binding of libfl.so (include/fl.h): argument marshalling only.

Every computation happens in the HIP library; this module moves pointers,
sizes and scalars across the C ABI.  PyTorch supplies device memory and the
stream.  If the library is missing the import of the binding fails loudly:
there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfl.so")

FL_OK, FL_EINVAL, FL_ERANGE, FL_ENOMEM, FL_EHIP, FL_EBUSY, FL_ENOTIMPL = range(7)
FL_NOT_FACILITY = 0xFFFFFFFF
FL_NONE = 0xFFFFFFFF
FL_RUNG_NONE = 0xFFFFFFFF
FL_RUNG_GUARD = 0xFFFFFFFE
FL_RUNG_END = 0xFFFFFFFD
FL_FLAG_NO_DENSE = 1
FL_FLAG_LUBY_MIS = 2
FL_FLAG_DIRECTED = 4


class FlProblem(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_arcs", C.c_uint64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("w", C.c_void_p), ("fac_cost", C.c_void_p),
                ("is_client", C.c_void_p)]


class FlParams(C.Structure):
    _fields_ = [("k", C.c_uint32), ("seed", C.c_uint64), ("eps", C.c_double), ("flags", C.c_uint32)]


class FlStats(C.Structure):
    _fields_ = [("ads_rounds", C.c_uint32), ("rungs", C.c_uint32), ("mis_rounds", C.c_uint32),
                ("n_guard", C.c_uint32), ("relax_alg", C.c_uint64), ("relax_exec", C.c_uint64),
                ("ads_entries", C.c_uint64), ("gamma", C.c_uint64), ("alpha0", C.c_double),
                ("ms_validate", C.c_double), ("ms_ads", C.c_double), ("ms_gamma", C.c_double),
                ("ms_open", C.c_double), ("ms_mis", C.c_double), ("ms_assign", C.c_double),
                ("ms_total", C.c_double), ("ms_ads_kernel", C.c_double), ("ms_ads_merge", C.c_double),
                ("ads_kernel_launches", C.c_uint32), ("workspace_bytes", C.c_uint64),
                ("n_reach_guard", C.c_uint32)]


class FlResult(C.Structure):
    _fields_ = [("open", C.c_void_p), ("assign", C.c_void_p), ("dist", C.c_void_p),
                ("open_rung", C.c_void_p), ("freeze_rung", C.c_void_p), ("q", C.c_void_p),
                ("total_cost", C.c_uint64), ("n_open", C.c_uint32), ("n_unreachable", C.c_uint32),
                ("status", C.c_int32), ("stats", FlStats)]


class FlSketchView(C.Structure):
    _fields_ = [("n", C.c_uint32), ("k", C.c_uint32), ("total", C.c_uint64), ("off", C.c_void_p),
                ("rank", C.c_void_p), ("dist", C.c_void_p), ("thresh", C.c_void_p)]


# every symbol include/fl.h declares, with its ctypes signature
SIGNATURES = {
    "fl_solve": (C.c_int, [C.POINTER(FlProblem), C.POINTER(FlParams), C.POINTER(FlResult), C.c_void_p]),
    "fl_solve_static": (C.c_int, [C.POINTER(FlProblem), C.POINTER(FlParams), C.POINTER(FlResult), C.c_void_p]),
    "fl_solve_batch": (C.c_int, [C.POINTER(FlProblem), C.POINTER(FlParams), C.POINTER(FlResult),
                                 C.c_uint32, C.c_void_p]),
    "fl_ads_build": (C.c_int, [C.POINTER(FlProblem), C.POINTER(FlParams), C.POINTER(C.c_void_p), C.c_void_p]),
    "fl_sketch_view": (C.c_int, [C.c_void_p, C.POINTER(FlSketchView)]),
    "fl_sketch_free": (None, [C.c_void_p]),
    "fl_rank_of": (C.c_uint32, [C.c_uint32, C.c_uint64]),
    "fl_priority_of": (C.c_uint32, [C.c_uint32, C.c_uint64]),
    "fl_strerror": (C.c_char_p, [C.c_int]),
    "fl_last_hip_error": (C.c_int, []),
    "fl_release_workspace": (None, []),
    "fl_server_create": (C.c_int, [C.c_uint64, C.c_uint32, C.POINTER(C.c_void_p)]),
    "fl_server_submit": (C.c_int, [C.c_void_p, C.POINTER(FlProblem), C.POINTER(FlParams), C.POINTER(FlResult),
                                   C.POINTER(C.c_uint64)]),
    "fl_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]),
    "fl_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]),
    "fl_server_destroy": (None, [C.c_void_p]),
    "fl_set_allocator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
}

# fl_alloc_fn / fl_free_fn of include/fl.h
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)

_lib = None


def lib():
    """Load libfl.so (built by paper_1503_03635_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FlError(RuntimeError):
    def __init__(self, code, where=""):
        msg = lib().fl_strerror(code).decode()
        if code == FL_EHIP:
            msg += f" (hip error {lib().fl_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")
        self.code = code


def strerror(code):
    return lib().fl_strerror(code).decode()
