"""The C-ABI library loads on a host without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmot.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mmot_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("mmot_query_workspace", "mmot_create", "mmot_iterate", "mmot_solve", "mmot_occupancy",
                 "mmot_edge_flows", "mmot_get_log_duals", "mmot_set_log_duals", "mmot_destroy"):
        assert must in names


def test_library_exports_all_declared_symbols():
    from paper_2106_14485_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmmot.so not built (run __graft_entry__.build())")
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_host_only_entry_points():
    """Calls that touch no device memory work without a GPU."""
    from paper_2106_14485_amd import _lib, solver
    L = _lib.lib()
    o = solver.default_options()
    assert o.check_every == 10 and o.use_graph == 1 and o.tol == 1e-6
    assert L.mmot_status_str(_lib.MMOT_EINFEASIBLE).decode().startswith("infeasible")
    p = _lib.Problem()
    p.n, p.L, p.T, p.eps, p.kind, p.nnz = 2000, 256, 50, 0.05, _lib.MMOT_CSR, 18430
    nb = ctypes.c_size_t(0)
    assert o.keep_forward == 1
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_OK
    # 50 stored backward and 51 kept forward message panels of 2000 x 256 floats
    # dominate the footprint; without kept forward messages, two rolling ones
    panel = 2000 * 256 * 4
    keep = nb.value
    assert 101 * panel < keep < 2 * 101 * panel
    o.keep_forward = 0
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_OK
    assert keep - nb.value == 49 * panel
    assert 52 * panel < nb.value < 2 * 52 * panel
    o.keep_forward = 2
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_EINVAL
    o.keep_forward = 1
    # a pool request keeps no forward messages
    assert L.mmot_pool_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_EUNSUPPORTED
    o.keep_forward = 0
    assert L.mmot_pool_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_OK
    # the pool's size is the solver's, 256 bytes of alignment and the program area of
    # (check_every + 1) (2 T + 8) + 8 work items of 368 bytes
    solo = ctypes.c_size_t(0)
    for T, every in ((50, 10), (7, 1), (120, 25)):
        p.T, o.check_every = T, every
        assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(solo)) == _lib.MMOT_OK
        assert L.mmot_pool_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_OK
        assert nb.value - solo.value == 256 + ((every + 1) * (2 * T + 8) + 8) * 368
    p.T, o.check_every = 50, 10
    o.keep_forward = 1
    p.eps = -1.0
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_EINVAL
    p.eps = 0.05
    p.T = 0
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_EINVAL
    # entry points given no solver reject the call without touching the device
    assert L.mmot_occupancy(None, None, None) == _lib.MMOT_EINVAL
    assert L.mmot_occupancy_window(None, None, None, 0, 1) == _lib.MMOT_EINVAL
    assert L.mmot_edge_flows(None, None, None) == _lib.MMOT_EINVAL


def _valid_csr_problem():
    from paper_2106_14485_amd import _lib
    p = _lib.Problem()
    p.n, p.L, p.T, p.eps, p.kind, p.nnz = 500, 40, 12, 0.05, _lib.MMOT_CSR, 4000
    return p


@pytest.mark.parametrize("change,expected", [
    (dict(n=0), "EINVAL"), (dict(L=0), "EINVAL"), (dict(T=0), "EINVAL"),
    (dict(eps=0.0), "EINVAL"), (dict(eps=float("nan")), "EINVAL"), (dict(eps=float("inf")), "EINVAL"),
    (dict(kind=7), "EINVAL"), (dict(cost_per_step=2), "EINVAL"), (dict(cap_comm_per_step=2), "EINVAL"),
    (dict(nnz=0), "EINVAL"), (dict(n=1 << 24, L=1 << 10), "EINVAL"),
    (dict(precision="BF16"), "EUNSUPPORTED"), (dict(domain=3), "EINVAL"), (dict(domain=-1), "EINVAL"),
    (dict(kind="DENSE", precision="FP64"), "EUNSUPPORTED"), (dict(kind="DENSE", domain="LOG"), "EUNSUPPORTED"),
    (dict(kind="DENSE", n=46341), "EINVAL"),
    (dict(), "OK"), (dict(kind="DENSE"), "OK"), (dict(kind="DENSE", precision="BF16"), "OK"),
    (dict(precision="FP64", domain="LOG"), "OK"),
])
def test_problem_and_option_validation(change, expected):
    """Each field the library validates before touching the device, one at a
    time, through mmot_query_workspace: out-of-range sizes, eps, kinds and flags
    are EINVAL; combinations the dense or sparse path does not run (dense FP64 or
    log domain, sparse BF16) EUNSUPPORTED; the rest succeed."""
    from paper_2106_14485_amd import _lib, solver
    L = _lib.lib()
    p, o = _valid_csr_problem(), solver.default_options()
    consts = {"DENSE": _lib.MMOT_DENSE, "BF16": _lib.MMOT_BF16, "FP64": _lib.MMOT_FP64, "LOG": _lib.MMOT_DOMAIN_LOG}
    for k, v in change.items():
        v = consts.get(v, v)
        setattr(o if k in ("precision", "domain") else p, k, v)
    nb = ctypes.c_size_t(0)
    assert L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == getattr(_lib, "MMOT_" + expected)
    if expected == "OK":
        assert nb.value > 0
