"""ctypes binding of libmmot.so (the C ABI declared in include/mmot.h).

Argument marshalling only; every step of the solver runs in the HIP library.
Importing this module raises if the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmot.so")

MMOT_OK, MMOT_EINVAL, MMOT_ENOMEM, MMOT_EINFEASIBLE, MMOT_ENUMERIC, MMOT_EHIP, MMOT_EAGAIN, MMOT_EUNSUPPORTED = range(8)
MMOT_CSR, MMOT_DENSE = 0, 1
MMOT_FP32, MMOT_FP64, MMOT_BF16 = 0, 1, 2
MMOT_DOMAIN_AUTO, MMOT_DOMAIN_SCALED, MMOT_DOMAIN_LOG = 0, 1, 2


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("L", ctypes.c_int32), ("T", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("kind", ctypes.c_int32), ("cap_per_step", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("cost", ctypes.c_void_p),
        ("cost_dense", ctypes.c_void_p), ("state_cost", ctypes.c_void_p), ("cap", ctypes.c_void_p),
        ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
        ("cost_per_step", ctypes.c_int32),
        ("cap_comm", ctypes.c_void_p), ("cap_comm_per_step", ctypes.c_int32),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("domain", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("calib_every", ctypes.c_int32), ("polish_iters", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("tol", ctypes.c_double), ("keep_forward", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("domain", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("dual_obj", ctypes.c_double), ("src_resid", ctypes.c_double), ("cap_viol", ctypes.c_double),
        ("mass_drift", ctypes.c_double), ("dual_gap", ctypes.c_double), ("mass", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MmotError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {lib().mmot_status_str(status).decode()} (status {status})")


_LIB = None

# symbol -> (restype, argtypes)
_SIGS = {
    "mmot_default_options": (None, [ctypes.POINTER(Options)]),
    "mmot_query_workspace": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "mmot_create": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mmot_iterate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "mmot_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "mmot_stats_now": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "mmot_occupancy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mmot_occupancy_window": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_int32]),
    "mmot_edge_flows": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "mmot_get_log_duals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mmot_set_log_duals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mmot_get_comm_duals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mmot_set_comm_duals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mmot_destroy": (None, [ctypes.c_void_p]),
    "mmot_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "mmot_iterations": (ctypes.c_int64, [ctypes.c_void_p]),
    "mmot_solve_static": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.POINTER(Stats), ctypes.c_void_p]),
    "mmot_pool_query_workspace": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "mmot_pool_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mmot_pool_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "mmot_pool_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mmot_pool_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(Stats)]),
    "mmot_pool_solver": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_uint64]),
    "mmot_pool_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "mmot_pool_destroy": (None, [ctypes.c_void_p]),
    "mmot_set_precision": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mmot_time_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
}


def lib():
    """The loaded library; raises ImportError (no fallback) when it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2106_14485_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status, what):
    if status != MMOT_OK:
        raise MmotError(status, what)
