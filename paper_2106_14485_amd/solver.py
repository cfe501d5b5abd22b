"""Python front end of the HIP solver: torch for device memory and streams only.

    s = Solver(instance, precision="fp32")      # uploads, validates, builds K on the GPU
    s.iterate(200)                               # Algorithm 2 iterations (async)
    st = s.stats()                               # dual objective, residuals (sync)
    occ, per_comm = s.occupancy(per_commodity=True)
    flows, cost = s.edge_flows()
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_PREC = {"fp32": _lib.MMOT_FP32, "fp64": _lib.MMOT_FP64, "bf16": _lib.MMOT_BF16}
_DOM = {"auto": _lib.MMOT_DOMAIN_AUTO, "scaled": _lib.MMOT_DOMAIN_SCALED, "log": _lib.MMOT_DOMAIN_LOG}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def default_options(**kw) -> _lib.Options:
    o = _lib.Options()
    _lib.lib().mmot_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = _PREC[v]
        if k == "domain" and isinstance(v, str):
            v = _DOM[v]
        setattr(o, k, v)
    return o


def device_problem(inst, device="cuda"):
    """Upload an Instance's arrays (float64 / int32) and fill the C problem struct.

    Returns (struct, keepalive-list)."""
    def dt(a, dtype):
        return None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)

    keep = []
    p = _lib.Problem()
    p.n, p.L, p.T, p.eps = inst.n, inst.L, inst.T, float(inst.eps)
    if inst.kind == "csr":
        p.kind = _lib.MMOT_CSR
        rp, ci, c = dt(inst.rowptr, torch.int32), dt(inst.colidx, torch.int32), dt(inst.cost, torch.float64)
        keep += [rp, ci, c]
        p.rowptr, p.colidx, p.cost = _ptr(rp), _ptr(ci), _ptr(c)
        p.nnz = int(inst.rowptr[-1])
        p.cost_per_step = 1 if np.ndim(inst.cost) == 2 else 0     # (T, nnz): time-varying network
    else:
        p.kind = _lib.MMOT_DENSE
        cd = dt(inst.cost_dense, torch.float64)
        keep.append(cd)
        p.cost_dense = _ptr(cd)
        p.nnz = int(np.isfinite(inst.cost_dense).sum())
        p.cost_per_step = 1 if np.ndim(inst.cost_dense) == 3 else 0   # (T, n, n): time-varying network
    cap = dt(inst.cap, torch.float64)
    p.cap_per_step = 1 if inst.cap.ndim == 2 else 0
    src, dst = dt(inst.src, torch.float64), dt(inst.dst, torch.float64)
    sc = dt(inst.state_cost, torch.float64)
    keep += [cap, src, dst, sc]
    p.cap, p.src, p.dst, p.state_cost = _ptr(cap), _ptr(src), _ptr(dst), _ptr(sc)
    cc = getattr(inst, "cap_comm", None)
    if cc is not None:
        ccd = dt(cc, torch.float64)
        keep.append(ccd)
        p.cap_comm = _ptr(ccd)
        p.cap_comm_per_step = 1 if np.ndim(cc) == 3 else 0     # (T-1, L, n) or (L, n)
    return p, keep


class Solver:
    def __init__(self, inst, precision="fp32", domain="auto", device="cuda", stream=None, **opts):
        L = _lib.lib()
        self.inst = inst
        self.device = torch.device(device)
        self.n, self.L, self.T = inst.n, inst.L, inst.T
        self.nnz = inst.nnz
        self.opts = default_options(precision=precision, domain=domain, **opts)
        p, keep = device_problem(inst, self.device)
        nbytes = ctypes.c_size_t(0)
        check(L.mmot_query_workspace(ctypes.byref(p), ctypes.byref(self.opts), ctypes.byref(nbytes)),
              "mmot_query_workspace")
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p(0)
        check(L.mmot_create(ctypes.byref(p), ctypes.byref(self.opts), _ptr(self.ws), self.ws_bytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "mmot_create")
        del keep
        self._h = h

    # -- iteration -------------------------------------------------------
    def iterate(self, n_iter: int, stats: bool = False):
        st = _lib.Stats() if stats else None
        check(_lib.lib().mmot_iterate(self._h, int(n_iter), ctypes.byref(st) if st is not None else None),
              "mmot_iterate")
        return st.as_dict() if st is not None else None

    def solve(self, max_iter: int):
        st = _lib.Stats()
        check(_lib.lib().mmot_solve(self._h, int(max_iter), ctypes.byref(st)), "mmot_solve")
        return st.as_dict()

    def stats(self):
        st = _lib.Stats()
        check(_lib.lib().mmot_stats_now(self._h, ctypes.byref(st)), "mmot_stats_now")
        return st.as_dict()

    @property
    def iterations(self):
        return int(_lib.lib().mmot_iterations(self._h))

    # -- outputs ---------------------------------------------------------
    def occupancy(self, per_commodity: bool = False, commodities=None):
        """Occupancy P_t, (T+1) x n; with per_commodity also P_{0,t}, (T+1) x L x n, or
        for commodities = (first, count) only that window, (T+1) x count x n."""
        occ = torch.empty((self.T + 1, self.n), dtype=torch.float64, device=self.device)
        if not per_commodity:
            check(_lib.lib().mmot_occupancy(self._h, _ptr(occ), None), "mmot_occupancy")
            return occ
        first, count = (0, self.L) if commodities is None else (int(commodities[0]), int(commodities[1]))
        # (one row at least, so that an empty window reaches the library and is rejected there)
        pc = torch.empty((self.T + 1, max(count, 1), self.n), dtype=torch.float64, device=self.device)
        check(_lib.lib().mmot_occupancy_window(self._h, _ptr(occ), _ptr(pc), first, count), "mmot_occupancy_window")
        return occ, pc

    def edge_flows(self):
        """Flows (T x nnz for a sparse network, T x n x n for a dense one) and the transport cost."""
        shape = (self.T, self.nnz) if self.inst.kind == "csr" else (self.T, self.n, self.n)
        flow = torch.empty(shape, dtype=torch.float64, device=self.device)
        cost = ctypes.c_double(0.0)
        check(_lib.lib().mmot_edge_flows(self._h, _ptr(flow), ctypes.byref(cost)), "mmot_edge_flows")
        return flow, cost.value

    def log_duals(self):
        ls = torch.empty((self.L, self.n), dtype=torch.float64, device=self.device)
        ld = torch.empty_like(ls)
        lc = torch.empty((max(self.T - 1, 1), self.n), dtype=torch.float64, device=self.device)
        check(_lib.lib().mmot_get_log_duals(self._h, _ptr(ls), _ptr(ld), _ptr(lc)), "mmot_get_log_duals")
        return ls, ld, lc[: self.T - 1]

    def set_log_duals(self, ls, ld, lc):
        ls = ls.to(self.device, torch.float64).contiguous()
        ld = ld.to(self.device, torch.float64).contiguous()
        lc = lc.to(self.device, torch.float64).contiguous()
        check(_lib.lib().mmot_set_log_duals(self._h, _ptr(ls), _ptr(ld), _ptr(lc)), "mmot_set_log_duals")
        self.stream.synchronize()

    def comm_duals(self):
        """log w_t of the commodity capacities, (T-1, L, n)."""
        lw = torch.empty((max(self.T - 1, 1), self.L, self.n), dtype=torch.float64, device=self.device)
        check(_lib.lib().mmot_get_comm_duals(self._h, _ptr(lw)), "mmot_get_comm_duals")
        return lw[: self.T - 1]

    def set_comm_duals(self, lw):
        lw = lw.to(self.device, torch.float64).contiguous()
        check(_lib.lib().mmot_set_comm_duals(self._h, _ptr(lw)), "mmot_set_comm_duals")
        self.stream.synchronize()

    def set_precision(self, precision: str):
        """Dense BF16 solvers: switch the products between 'bf16' and 'fp32' (polish)."""
        check(_lib.lib().mmot_set_precision(self._h, _PREC[precision]), "mmot_set_precision")

    def time_step(self, forward: bool = True, reps: int = 50) -> float:
        """Average device milliseconds of one sweep step (HIP events)."""
        ms = ctypes.c_double(0.0)
        check(_lib.lib().mmot_time_step(self._h, 1 if forward else 0, int(reps), ctypes.byref(ms)), "mmot_time_step")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mmot_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
