"""Unregularised LP optimum and walk counts (test infrastructure only).

The dynamic multi-commodity min-cost flow problem (Section 2.1, problem
flow_dynamic_multi-commodity) is solved in node-edge form on the
time-expanded network: one variable per (commodity, transition time tau,
allowed move i -> j), flow balance per (commodity, time, state), source
distribution at time 0, sink distribution at time T, joint occupancy capacity
at the interior times, objective sum of move costs plus interior state costs.
By Theorem 2 its optimum equals that of the tensor problem "multicommodity".

For the entropy gap: if M_eps solves the regularised problem and M* the LP,
  0 <= <C, M_eps> - <C, M*> <= eps * sum_l m_l log |P_l|
where |P_l| is the number of feasible walks of commodity l (its entries are
at most m_l and its support has at most |P_l| elements).  walk_counts gives
|P_l| for point sources and sinks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

__all__ = ["lp_optimum", "walk_counts"]


def lp_optimum(C, T, src, dst, cap, state_cost=None, cap_comm=None):
    """Optimal value of the unregularised problem; C scipy sparse (allowed moves),
    or a list of T of them with one sparsity pattern (costs of the move tau ->
    tau+1; +inf closes a move at that step).  cap_comm: optional commodity
    capacities D (T-1, L, n) or (L, n): commodity l's occupancy of state i at
    interior time tau is at most D[tau-1, l, i] (+inf = none)."""
    steps = C if isinstance(C, (list, tuple)) else [C] * T
    Cc = sp.coo_matrix(steps[0])
    ei, ej = Cc.row, Cc.col
    E = len(ei)
    ecs = [sp.coo_matrix(c).data for c in steps]
    for c in steps:
        cc = sp.coo_matrix(c)
        assert np.array_equal(cc.row, ei) and np.array_equal(cc.col, ej), "one sparsity pattern for all steps"
    L, n = src.shape
    cap = np.asarray(cap, dtype=np.float64)
    if cap.ndim == 1:
        cap = np.broadcast_to(cap, (max(T - 1, 0), n))
    nv = L * T * E
    cost = np.zeros(nv)
    closed = np.zeros(nv, dtype=bool)
    for l in range(L):
        for tau in range(T):
            c = ecs[tau].copy()
            if state_cost is not None and tau + 1 < T:
                c = c + state_cost[l, ej]       # state cost at the arrival time (interior only)
            blk = slice((l * T + tau) * E, (l * T + tau + 1) * E)
            closed[blk] = ~np.isfinite(c)
            cost[blk] = np.where(np.isfinite(c), c, 0.0)
    out_of = [np.nonzero(ei == i)[0] for i in range(n)]
    into = [np.nonzero(ej == j)[0] for j in range(n)]
    R, Cl, V, b = [], [], [], []
    r = 0
    for l in range(L):
        base = l * T * E
        for i in range(n):
            es = out_of[i]
            R += [r] * len(es); Cl += list(base + es); V += [1.0] * len(es); b.append(src[l, i]); r += 1
        for j in range(n):
            es = into[j]
            R += [r] * len(es); Cl += list(base + (T - 1) * E + es); V += [1.0] * len(es); b.append(dst[l, j]); r += 1
        for tau in range(1, T):
            for i in range(n):
                a, o = into[i], out_of[i]
                R += [r] * (len(a) + len(o))
                Cl += list(base + (tau - 1) * E + a) + list(base + tau * E + o)
                V += [1.0] * len(a) + [-1.0] * len(o)
                b.append(0.0); r += 1
    Aeq = sp.csr_matrix((V, (R, Cl)), shape=(r, nv))
    beq = np.array(b)
    R, Cl, V, b = [], [], [], []
    r = 0
    for tau in range(1, T):
        for i in range(n):
            if not np.isfinite(cap[tau - 1, i]):
                continue
            a = into[i]
            for l in range(L):
                R += [r] * len(a); Cl += list(l * T * E + (tau - 1) * E + a); V += [1.0] * len(a)
            b.append(cap[tau - 1, i]); r += 1
    if cap_comm is not None:
        D = np.asarray(cap_comm, dtype=np.float64)
        if D.ndim == 2:
            D = np.broadcast_to(D, (max(T - 1, 0),) + D.shape)
        for tau in range(1, T):
            for l in range(L):
                for i in range(n):
                    if not np.isfinite(D[tau - 1, l, i]):
                        continue
                    a = into[i]
                    R += [r] * len(a); Cl += list(l * T * E + (tau - 1) * E + a); V += [1.0] * len(a)
                    b.append(D[tau - 1, l, i]); r += 1
    Aub = sp.csr_matrix((V, (R, Cl)), shape=(r, nv)) if r else None
    bub = np.array(b) if r else None
    bounds = [(0, 0) if c else (0, None) for c in closed]     # a closed move carries no flow
    res = linprog(cost, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(f"LP failed: {res.message}")
    return float(res.fun)


def walk_counts(C, T, sources, sinks):
    """Number of length-T walks along allowed moves from each source to its sink
    (exact ints); C may be a list of T per-step matrices (+inf = closed)."""
    steps = C if isinstance(C, (list, tuple)) else [C] * T
    adjs = []
    for c in steps:
        pat = sp.coo_matrix(c)
        n = pat.shape[0]
        adj = [[] for _ in range(n)]
        for i, j, v in zip(pat.row, pat.col, pat.data):
            if np.isfinite(v):
                adj[i].append(j)
        adjs.append(adj)
    counts = []
    for s, z in zip(sources, sinks):
        v = [0] * n
        v[s] = 1
        for tau in range(T):
            w = [0] * n
            for i in range(n):
                if v[i]:
                    for j in adjs[tau][i]:
                        w[j] += v[i]
            v = w
        counts.append(v[z])
    return counts
