"""Continuous-batching serving loop over the library's solve pool.

Requests (problem instances) arrive over time; the loop admits them into the
pool as soon as they arrive and fit the HBM budget, advances all running
solves together in batched launches, and retires finished ones (freeing their
budget for queued requests).  Latency = completion time - arrival time.
The plain reference serves the same trace one solve at a time with the
ordinary solver (mmot_solve), in arrival order.
"""
from __future__ import annotations

import collections
import ctypes
import sys
import time

import numpy as np
import torch

from . import _lib
from ._lib import MmotError, check
from .solver import Solver, _ptr, default_options, device_problem


class Pool:
    """Thin binding of mmot_pool_*: torch provides each request's workspace."""

    def __init__(self, hbm_budget_bytes: int, device="cuda", stream=None, check_every=10, tol=1e-6):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # (the pool keeps two forward panels per request: a smaller workspace per solve)
        self.opts = default_options(precision="fp32", domain="auto", check_every=check_every, tol=tol,
                                    keep_forward=0)
        h = ctypes.c_void_p(0)
        check(_lib.lib().mmot_pool_create(int(hbm_budget_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)), "mmot_pool_create")
        self._h = h
        self._ws = {}
        self._shape = {}

    def workspace_bytes(self, inst) -> int:
        p, keep = _problem_sizes(inst)
        nb = ctypes.c_size_t(0)
        check(_lib.lib().mmot_pool_query_workspace(ctypes.byref(p), ctypes.byref(self.opts), ctypes.byref(nb)),
              "mmot_pool_query_workspace")
        return nb.value

    def submit(self, inst, max_iter=500):
        """Admit a request; returns its ticket, or None when the budget is full."""
        nbytes = self.workspace_bytes(inst)
        p, keep = device_problem(inst, self.device)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        t = ctypes.c_uint64(0)
        st = _lib.lib().mmot_pool_submit(self._h, ctypes.byref(p), ctypes.byref(self.opts), _ptr(ws), nbytes,
                                         int(max_iter), ctypes.byref(t))
        del keep
        if st == _lib.MMOT_EAGAIN:
            return None
        check(st, "mmot_pool_submit")
        self._ws[t.value] = ws
        self._shape[t.value] = (inst.T, inst.n, inst.L)
        return t.value

    def run(self, max_ticks=64) -> int:
        n = ctypes.c_int32(0)
        check(_lib.lib().mmot_pool_run(self._h, int(max_ticks), ctypes.byref(n)), "mmot_pool_run")
        return n.value

    def poll(self, ticket):
        state = ctypes.c_int32(0)
        st = _lib.Stats()
        status = _lib.lib().mmot_pool_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(state), ctypes.byref(st))
        return state.value, status, st.as_dict()

    def occupancy(self, ticket, per_commodity=False):
        T, n, L = self._shape[ticket]
        s = _lib.lib().mmot_pool_solver(self._h, ctypes.c_uint64(ticket))
        occ = torch.empty((T + 1, n), dtype=torch.float64, device=self.device)
        pc = torch.empty((T + 1, L, n), dtype=torch.float64, device=self.device) if per_commodity else None
        check(_lib.lib().mmot_occupancy(ctypes.c_void_p(s), _ptr(occ), _ptr(pc)), "mmot_occupancy")
        return (occ, pc) if per_commodity else occ

    def release(self, ticket):
        check(_lib.lib().mmot_pool_release(self._h, ctypes.c_uint64(ticket)), "mmot_pool_release")
        self._ws.pop(ticket, None)
        self._shape.pop(ticket, None)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mmot_pool_destroy(self._h)
            self._h = None
            self._ws.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_sizes(inst):
    """The problem struct as mmot_query_workspace reads it: sizes and kinds, and the
    optional arrays only as present or absent (a host placeholder, never read)."""
    p = _lib.Problem()
    p.n, p.L, p.T, p.eps = inst.n, inst.L, inst.T, float(inst.eps)
    p.kind = _lib.MMOT_CSR if inst.kind == "csr" else _lib.MMOT_DENSE
    p.nnz = inst.nnz
    p.cost_per_step = 1 if (np.ndim(inst.cost) == 2 if inst.kind == "csr" else np.ndim(inst.cost_dense) == 3) else 0
    marker = np.zeros(1)
    if inst.state_cost is not None:
        p.state_cost = marker.ctypes.data
    if getattr(inst, "cap_comm", None) is not None:
        p.cap_comm = marker.ctypes.data
        p.cap_comm_per_step = 1 if np.ndim(inst.cap_comm) == 3 else 0
    return p, marker


def _progress(tag, done, total, t0):
    print(f"[{tag}] {done}/{total} requests done after {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)


def serve(instances, arrivals, budget_bytes, max_iter=500, ticks_per_round=32, check_every=10, tol=1e-6,
          progress=0):
    """Serve a trace with the pool.  Returns per-request dicts (latency, stats).
    progress > 0: a line on stderr every `progress` finished requests."""
    order = np.argsort(arrivals, kind="stable")
    pending = collections.deque(int(i) for i in order)
    pool = Pool(budget_bytes, check_every=check_every, tol=tol)
    active = {}
    done = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while pending or active:
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            i = pending[0]
            try:
                tk = pool.submit(instances[i], max_iter=max_iter)
            except MmotError as e:          # rejected at admission (e.g. invalid data)
                pending.popleft()
                done[i] = dict(latency=time.perf_counter() - t0 - arrivals[i], stats=None, status=e.status)
                continue
            if tk is None:
                break
            active[tk] = i
            pending.popleft()
        if active:
            pool.run(ticks_per_round)
            for tk in list(active):
                state, status, st = pool.poll(tk)
                if state != 0:
                    i = active.pop(tk)
                    done[i] = dict(latency=time.perf_counter() - t0 - arrivals[i], stats=st, status=status)
                    pool.release(tk)
                    if progress and len(done) % progress == 0:
                        _progress("served", len(done), len(instances), t0)
        elif pending:
            wait = arrivals[pending[0]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    total = time.perf_counter() - t0
    pool.close()
    return [done[i] for i in range(len(instances))], total


def serve_plain(instances, arrivals, max_iter=500, check_every=10, tol=1e-6, progress=0):
    """One solve at a time, in arrival order, with the plain solver."""
    order = np.argsort(arrivals, kind="stable")
    out = [None] * len(instances)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in order:
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        st, status = None, 0
        try:
            S = Solver(instances[i], precision="fp32", domain="auto", check_every=check_every, tol=tol,
                       keep_forward=0)   # the pool's options: the same iterates and checks
            try:
                st = S.solve(max_iter)
            finally:
                S.close()
        except MmotError as e:              # the request fails; the service goes on
            status = e.status
        out[i] = dict(latency=time.perf_counter() - t0 - arrivals[i], stats=st, status=status)
        ndone = sum(1 for r in out if r is not None)
        if progress and ndone % progress == 0:
            _progress("plain", ndone, len(instances), t0)
    return out, time.perf_counter() - t0


def latency_summary(results, total_s):
    lat = np.array([r["latency"] for r in results])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "solves_per_s": len(results) / total_s, "n": len(results),
            "failed": int(sum(1 for r in results if r["status"] != 0)),
            "converged": int(sum(1 for r in results if r["stats"] and r["stats"]["converged"]))}
