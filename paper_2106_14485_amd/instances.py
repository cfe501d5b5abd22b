"""Seeded synthetic problem instances for the dynamic multi-commodity flow solver.

This module only *builds inputs*: graphs, transition costs, capacities and
per-commodity source/sink distributions.  It contains none of the solver's
arithmetic (no kernel K = exp(-C/eps), no scalings, no messages), so both the
FP64 oracle (through the tests) and the GPU library consume the same arrays.

Problem data follow the multi-commodity problem of Section 3.2 of the paper
(problem "multicommodity" with cost tensor "cost_multicommodity"), read with
*states = graph nodes* (transition cost matrix C on graph edges plus waiting
self-loops, capacity d on node occupancy at the interior times 1..T-1, source
distribution R^(0,1) at time 0 and sink distribution R^(0,T) at time T).
Topology is encoded by C = +inf (Section 3, hard constraints through infinite
costs), i.e. by the CSR sparsity pattern.

Every array is float64 / int32 numpy.  Node orderings are chosen for memory
locality (Morton order for point clouds, row-major for grids); a relabelling of
nodes does not change the problem.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.spatial

__all__ = [
    "Instance",
    "grid_instance",
    "rgg_instance",
    "dense_blob_instance",
    "road_grid_instance",
    "serve_trace",
    "instance_from_request",
    "lp_feasible",
    "edge_state_instance",
    "sparse_grid_edge_instance",
    "dense_random_edge_instance",
    "time_varying_instance",
    "staggered_instance",
]


@dataclasses.dataclass
class Instance:
    """One dynamic multi-commodity flow problem.

    n states, L commodities, T time steps (marginals at times 0..T), eps > 0.
    kind == "csr": transitions are the CSR entries (rowptr, colidx, cost);
    entry (i, j) with finite cost cost means moving from state i at time tau to
    state j at time tau+1 is allowed at that cost.
    kind == "dense": cost_dense (n, n) with +inf for forbidden transitions.
    cap: (n,) applied at every interior time 1..T-1, or (T-1, n); +inf means
    uncapacitated.  src / dst: (L, n) nonnegative, equal row sums (the
    commodity masses).  state_cost: optional (L, n) per-commodity state cost
    charged at interior times (None means zero).  A time-varying network
    (Section 3.3) has cost of shape (T, nnz): row tau prices the moves from
    time tau to tau+1 (same pattern; +inf closes a move at that step).
    cap_comm: optional commodity-dependent capacities D (the extension at the
    end of Section 3), (L, n) at every interior time or (T-1, L, n):
    commodity l occupies state i by at most D (+inf = no such bound).
    """

    name: str
    n: int
    L: int
    T: int
    eps: float
    kind: str
    src: np.ndarray
    dst: np.ndarray
    cap: np.ndarray
    rowptr: Optional[np.ndarray] = None
    colidx: Optional[np.ndarray] = None
    cost: Optional[np.ndarray] = None
    cost_dense: Optional[np.ndarray] = None
    state_cost: Optional[np.ndarray] = None
    cap_comm: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        if self.kind == "csr":
            return int(self.rowptr[-1])
        return int(np.isfinite(self.cost_dense).sum())

    def cap_full(self) -> np.ndarray:
        """Capacities as a (T-1, n) array (one row per interior time)."""
        if self.cap.ndim == 1:
            return np.broadcast_to(self.cap, (max(self.T - 1, 0), self.n)).copy()
        return self.cap.copy()

    def cost_csr(self):
        """The transition cost matrix as scipy CSR (the allowed moves); for a
        time-varying network (cost of shape (T, nnz)) the list of the T
        per-step matrices, +inf marking a move closed at that step."""
        if self.kind == "csr":
            if np.ndim(self.cost) == 2:
                return [sp.csr_matrix((c, self.colidx, self.rowptr), shape=(self.n, self.n)) for c in self.cost]
            return sp.csr_matrix((self.cost, self.colidx, self.rowptr), shape=(self.n, self.n))
        r, c = np.nonzero(np.isfinite(self.cost_dense))
        return sp.csr_matrix((self.cost_dense[r, c], (r, c)), shape=(self.n, self.n))

    def masses(self) -> np.ndarray:
        return self.src.sum(axis=1)


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def _morton_order(pts: np.ndarray, bits: int = 16) -> np.ndarray:
    q = np.clip((pts * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)

    def spread(v):
        v = v & 0xFFFF
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << 1)
    return np.argsort(code, kind="stable")


def _csr_from_pairs(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    m = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def _hop_dist(rowptr, colidx, n, sources):
    g = sp.csr_matrix((np.ones(len(colidx)), colidx, rowptr), shape=(n, n))
    return csgraph.shortest_path(g, directed=True, unweighted=True, indices=sources)


def lp_feasible(inst: Instance) -> bool:
    """Feasibility of the (unregularised) dynamic multi-commodity flow problem.

    Node-edge LP on the time-expanded network (Section 2.2): one flow variable
    per (commodity, transition time, allowed transition); flow balance at every
    (commodity, time, state), sources at time 0, sinks at time T, joint
    occupancy capacity at interior times.  Used only to reject seeds that make
    tiny instances infeasible.
    """
    from scipy.optimize import linprog

    Cc = inst.cost_csr().tocoo()
    src_e, dst_e = Cc.row, Cc.col
    E = len(src_e)
    n, L, T = inst.n, inst.L, inst.T
    nv = L * T * E

    def var(l, tau, e):
        return (l * T + tau) * E + e

    rows, cols, vals, rhs = [], [], [], []
    r = 0
    e_idx = np.arange(E)
    for l in range(L):
        # time 0 outflow = source
        for i in range(n):
            es = e_idx[src_e == i]
            rows += [r] * len(es); cols += [var(l, 0, e) for e in es]; vals += [1.0] * len(es)
            rhs.append(inst.src[l, i]); r += 1
        # time T inflow = sink
        for j in range(n):
            es = e_idx[dst_e == j]
            rows += [r] * len(es); cols += [var(l, T - 1, e) for e in es]; vals += [1.0] * len(es)
            rhs.append(inst.dst[l, j]); r += 1
        # balance at interior times
        for tau in range(1, T):
            for i in range(n):
                ein = e_idx[dst_e == i]
                eout = e_idx[src_e == i]
                rows += [r] * (len(ein) + len(eout))
                cols += [var(l, tau - 1, e) for e in ein] + [var(l, tau, e) for e in eout]
                vals += [1.0] * len(ein) + [-1.0] * len(eout)
                rhs.append(0.0); r += 1
    A_eq = sp.csr_matrix((vals, (rows, cols)), shape=(r, nv))
    b_eq = np.array(rhs)
    capf = inst.cap_full()
    rows, cols, vals, rhs = [], [], [], []
    r = 0
    for tau in range(1, T):
        for i in range(n):
            if not np.isfinite(capf[tau - 1, i]):
                continue
            ein = e_idx[dst_e == i]
            for l in range(L):
                rows += [r] * len(ein); cols += [var(l, tau - 1, e) for e in ein]; vals += [1.0] * len(ein)
            rhs.append(capf[tau - 1, i]); r += 1
    A_ub = sp.csr_matrix((vals, (rows, cols)), shape=(r, nv)) if r else None
    b_ub = np.array(rhs) if r else None
    res = linprog(np.zeros(nv), A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                  bounds=(0, None), method="highs")
    return res.status == 0


# ----------------------------------------------------------------------------
# configuration generators
# ----------------------------------------------------------------------------

def grid_instance(side: int = 5, T: int = 10, L: int = 3, eps: float = 0.1,
                  move_cost: float = 1.0, wait_cost: float = 0.1, cap: float = 0.5,
                  seed: int = 0, check_feasible: bool = True, max_tries: int = 200) -> Instance:
    """side x side 4-neighbour grid, unit-mass commodities, uniform node capacity.

    Node r*side + c.  Sources and sinks are drawn without replacement; a draw
    is rejected when the LP says the instance is infeasible.
    """
    n = side * side
    rows, cols, vals = [], [], []
    for r_ in range(side):
        for c_ in range(side):
            i = r_ * side + c_
            rows.append(i); cols.append(i); vals.append(wait_cost)
            for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                rr, cc = r_ + dr, c_ + dc
                if 0 <= rr < side and 0 <= cc < side:
                    rows.append(i); cols.append(rr * side + cc); vals.append(move_cost)
    rowptr, colidx, cost = _csr_from_pairs(n, np.array(rows), np.array(cols), np.array(vals))
    rng = np.random.default_rng(seed)
    for attempt in range(max_tries):
        srcs = rng.choice(n, size=L, replace=False)
        dsts = rng.choice(n, size=L, replace=False)
        src = np.zeros((L, n)); dst = np.zeros((L, n))
        src[np.arange(L), srcs] = 1.0
        dst[np.arange(L), dsts] = 1.0
        hd = _hop_dist(rowptr, colidx, n, srcs)
        if np.any(hd[np.arange(L), dsts] > T):
            continue
        inst = Instance(name=f"grid{side}x{side}", n=n, L=L, T=T, eps=eps, kind="csr",
                        src=src, dst=dst, cap=np.full(n, cap), rowptr=rowptr,
                        colidx=colidx, cost=cost,
                        meta=dict(seed=seed, attempt=attempt, sources=srcs, sinks=dsts))
        if not check_feasible or lp_feasible(inst):
            return inst
    raise RuntimeError("no feasible grid instance found")


def rgg_instance(n: int = 2000, L: int = 256, T: int = 50, eps: float = 0.05, k: int = 7,
                 wait_cost: float = 0.01, cap_lo: float = 0.2, cap_hi: float = 1.0,
                 seed: int = 0) -> Instance:
    """Random geometric graph: symmetrised k-NN over uniform points in the unit square.

    Transition cost = Euclidean edge length, self-loop = wait cost.  Commodity
    (source, sink) pairs are iid uniform nodes, rejected when the sink is more
    than T hops away; masses ~ U[0.5, 1.5]; node capacity ~ U[cap_lo, cap_hi]
    times the mean commodity mass.
    """
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    pts = pts[_morton_order(pts)]
    tree = scipy.spatial.cKDTree(pts)
    _, nb = tree.query(pts, k=k + 1)
    r0 = np.repeat(np.arange(n), k)
    c0 = nb[:, 1:].reshape(-1)
    rows = np.concatenate([r0, c0, np.arange(n)])
    cols = np.concatenate([c0, r0, np.arange(n)])
    # symmetrise (duplicates collapse), then attach costs
    pat = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    pat.sum_duplicates(); pat.sort_indices()
    coo = pat.tocoo()
    d = np.linalg.norm(pts[coo.row] - pts[coo.col], axis=1)
    d[coo.row == coo.col] = wait_cost
    rowptr, colidx, cost = _csr_from_pairs(n, coo.row, coo.col, d)
    srcs = np.empty(L, dtype=np.int64); dsts = np.empty(L, dtype=np.int64)
    filled = 0
    while filled < L:
        s = rng.integers(0, n, size=L - filled)
        z = rng.integers(0, n, size=L - filled)
        hd = _hop_dist(rowptr, colidx, n, s)
        ok = hd[np.arange(len(s)), z] <= T
        m = int(ok.sum())
        srcs[filled:filled + m] = s[ok]; dsts[filled:filled + m] = z[ok]
        filled += m
    mass = rng.uniform(0.5, 1.5, size=L)
    src = np.zeros((L, n)); dst = np.zeros((L, n))
    src[np.arange(L), srcs] = mass
    dst[np.arange(L), dsts] = mass
    capv = rng.uniform(cap_lo, cap_hi, size=n) * mass.mean()
    return Instance(name=f"rgg{n}", n=n, L=L, T=T, eps=eps, kind="csr", src=src, dst=dst,
                    cap=capv, rowptr=rowptr, colidx=colidx, cost=cost,
                    meta=dict(seed=seed, points=pts, sources=srcs, sinks=dsts, k=k))


def dense_blob_instance(n: int = 4096, L: int = 1024, T: int = 32, eps: float = 0.02,
                        trunc: float = 0.25, sigma: float = 0.05, cap_factor: float = 2.0,
                        seed: int = 0) -> Instance:
    """Complete graph on uniform points, cost = squared distance truncated at `trunc`.

    C_ij = |x_i - x_j|^2 if that is <= trunc else +inf (C_ii = 0).  Source and
    sink distributions are Gaussian blobs (std `sigma`) around uniform centres,
    each normalised to unit mass; uniform capacity cap_factor * L / n.
    """
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    pts = pts[_morton_order(pts)]
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    C = np.where(d2 <= trunc, d2, np.inf)
    np.fill_diagonal(C, 0.0)
    a = rng.random((L, 2)); b = rng.random((L, 2))

    def blobs(centres):
        e = np.exp(-((pts[None, :, :] - centres[:, None, :]) ** 2).sum(-1) / (2 * sigma ** 2))
        return e / e.sum(axis=1, keepdims=True)

    src = blobs(a); dst = blobs(b)
    capv = np.full(n, cap_factor * L / n)
    return Instance(name=f"dense{n}", n=n, L=L, T=T, eps=eps, kind="dense", src=src, dst=dst,
                    cap=capv, cost_dense=C,
                    meta=dict(seed=seed, points=pts, src_centres=a, dst_centres=b))


def road_grid_instance(side: int = 100, L: int = 2000, T: int = 120, eps: float = 0.05,
                       cost_lo: float = 1.0, cost_hi: float = 3.0, wait_cost: float = 0.1,
                       zipf_s: float = 1.1, base_cap_factor: float = 4.0,
                       weak_frac: float = 0.05, weak_factor: float = 0.1,
                       seed: int = 0) -> Instance:
    """Traffic-routing grid: side x side 4-neighbour roads with U[cost_lo, cost_hi] costs.

    Undirected edge costs (symmetric C), wait cost on self-loops.  Origins and
    destinations are Zipf(zipf_s)-weighted over a seeded node permutation; OD
    pairs further than T in Manhattan distance are redrawn.  Masses are
    lognormal(0, 0.5).  Origin/destination nodes are uncapacitated; relay nodes
    get base_cap_factor * mean mass, a seeded weak_frac of them weak_factor
    times that.  States are labelled in Morton order of their grid position
    (meta["grid_of"][k] = row-major grid id r * side + c of state k).
    """
    rng = np.random.default_rng(seed)
    n = side * side
    rows, cols, vals = [], [], []
    for r_ in range(side):
        for c_ in range(side):
            i = r_ * side + c_
            if c_ + 1 < side:
                w = rng.uniform(cost_lo, cost_hi)
                j = i + 1
                rows += [i, j]; cols += [j, i]; vals += [w, w]
            if r_ + 1 < side:
                w = rng.uniform(cost_lo, cost_hi)
                j = i + side
                rows += [i, j]; cols += [j, i]; vals += [w, w]
    rows += list(range(n)); cols += list(range(n)); vals += [wait_cost] * n
    perm = rng.permutation(n)
    w = 1.0 / np.arange(1, n + 1) ** zipf_s
    p = w / w.sum()
    o = np.empty(L, dtype=np.int64); z = np.empty(L, dtype=np.int64)
    filled = 0
    while filled < L:
        oo = perm[rng.choice(n, size=L - filled, p=p)]
        zz = perm[rng.choice(n, size=L - filled, p=p)]
        man = np.abs(oo // side - zz // side) + np.abs(oo % side - zz % side)
        ok = man <= T
        m = int(ok.sum())
        o[filled:filled + m] = oo[ok]; z[filled:filled + m] = zz[ok]
        filled += m
    mass = rng.lognormal(0.0, 0.5, size=L)
    src = np.zeros((L, n)); dst = np.zeros((L, n))
    np.add.at(src, (np.arange(L), o), mass)
    np.add.at(dst, (np.arange(L), z), mass)
    capv = np.full(n, base_cap_factor * mass.mean())
    relay = np.setdiff1d(np.arange(n), np.union1d(o, z))
    weak = rng.choice(relay, size=int(round(weak_frac * len(relay))), replace=False)
    capv[weak] *= weak_factor
    capv[np.union1d(o, z)] = np.inf
    # States relabelled in Morton (Z) order of their grid position (the draws above
    # use row-major ids): the five rows a sweep step gathers for a state then lie
    # close together in the panels.  A relabelling does not change the problem.
    grid = np.arange(n)
    order = _morton_order(np.stack([(grid % side + 0.5) / side, (grid // side + 0.5) / side], axis=1))
    lab = np.empty(n, dtype=np.int64)
    lab[order] = np.arange(n)
    rowptr, colidx, cost = _csr_from_pairs(n, lab[np.array(rows)], lab[np.array(cols)], np.array(vals))
    return Instance(name=f"road{side}x{side}", n=n, L=L, T=T, eps=eps, kind="csr",
                    src=src[:, order], dst=dst[:, order], cap=capv[order], rowptr=rowptr, colidx=colidx, cost=cost,
                    meta=dict(seed=seed, origins=lab[o], destinations=lab[z], weak=lab[weak], grid_of=order))


# ----------------------------------------------------------------------------
# edge-state lifts (the paper's own state spaces: flows on edges)
# ----------------------------------------------------------------------------
def edge_state_instance(nv: int, edges: np.ndarray, L: int, T: int, eps: float, edge_cost: np.ndarray,
                        src_vertex: np.ndarray, dst_vertex: np.ndarray, mass: np.ndarray,
                        cap_edge, terminals: str = "storage", cap_vertex=np.inf,
                        name: str = "edges") -> Instance:
    """Dynamic multi-commodity flow with flow on the edges of a directed graph.

    The state at a time is the edge (or terminal) a unit of flow is on
    (Section 3.1: the marginal P_t is the flow over the edges in one time
    interval; the transition cost C is 0 where edge i leads to edge j -- the
    head of i is the tail of j -- and +inf otherwise, eq. T_cost; the cost of
    using an edge is the per-commodity state cost c^l, charged at interior
    times).  edges: (m, 2) int array of (tail, head) vertices.  edge_cost:
    (L, m).  cap_edge: scalar or (m,) capacity of the summed flow on an edge.

    terminals = "storage" (Section 3.3, storage in the vertices): the state
    space is augmented by the vertices, n = m + nv; a vertex leads to itself
    (storage, cost 0) and to the edges leaving it, an edge leads to the edges
    leaving its head and to its head vertex; commodities start and end at
    vertices; vertex capacity cap_vertex.
    terminals = "routing" (Section 3.3, eq. cost_traffic_routing): states are
    the edges plus one source state per distinct source vertex and one sink
    state per distinct sink vertex; flow may wait only in its source and sink
    states, cannot re-enter a source and cannot leave a sink; a source state
    leads to itself and the edges leaving its vertex, an edge entering a sink
    vertex leads to that sink state.  Terminal states are uncapacitated.
    """
    edges = np.asarray(edges, dtype=np.int64)
    m = len(edges)
    tail, head = edges[:, 0], edges[:, 1]
    out_of = [[] for _ in range(nv)]
    for e in range(m):
        out_of[tail[e]].append(e)
    rows, cols = [], []
    for e in range(m):                      # line graph: e -> every edge leaving head(e)
        for f in out_of[head[e]]:
            rows.append(e); cols.append(f)
    src_vertex = np.asarray(src_vertex); dst_vertex = np.asarray(dst_vertex)
    if terminals == "storage":
        n = m + nv
        for v in range(nv):
            rows.append(m + v); cols.append(m + v)             # storage in the vertex
            for f in out_of[v]:
                rows.append(m + v); cols.append(f)             # depart along an edge
        for e in range(m):
            rows.append(e); cols.append(m + head[e])           # arrive at the head vertex
        s_state = m + src_vertex
        z_state = m + dst_vertex
        cap = np.concatenate([np.broadcast_to(np.asarray(cap_edge, dtype=np.float64), (m,)),
                              np.broadcast_to(np.asarray(cap_vertex, dtype=np.float64), (nv,))])
    elif terminals == "routing":
        srcs = np.unique(src_vertex); snks = np.unique(dst_vertex)
        sid = {int(v): m + k for k, v in enumerate(srcs)}
        zid = {int(v): m + len(srcs) + k for k, v in enumerate(snks)}
        n = m + len(srcs) + len(snks)
        for v, i in sid.items():
            rows.append(i); cols.append(i)                     # wait in the source
            for f in out_of[v]:
                rows.append(i); cols.append(f)
        for v, i in zid.items():
            rows.append(i); cols.append(i)                     # wait in the sink
        for e in range(m):
            if int(head[e]) in zid:
                rows.append(e); cols.append(zid[int(head[e])])
        s_state = np.array([sid[int(v)] for v in src_vertex])
        z_state = np.array([zid[int(v)] for v in dst_vertex])
        cap = np.concatenate([np.broadcast_to(np.asarray(cap_edge, dtype=np.float64), (m,)),
                              np.full(n - m, np.inf)])
    else:
        raise ValueError(f"unknown terminals {terminals!r}")
    rows = np.array(rows); cols = np.array(cols)
    rowptr, colidx, cost = _csr_from_pairs(n, rows, cols, np.zeros(len(rows)))
    src = np.zeros((L, n)); dst = np.zeros((L, n))
    np.add.at(src, (np.arange(L), s_state), mass)
    np.add.at(dst, (np.arange(L), z_state), mass)
    state_cost = np.zeros((L, n))
    state_cost[:, :m] = edge_cost
    return Instance(name=name, n=n, L=L, T=T, eps=eps, kind="csr", src=src, dst=dst, cap=cap,
                    rowptr=rowptr, colidx=colidx, cost=cost, state_cost=state_cost,
                    meta=dict(m=m, nv=nv, edges=edges, terminals=terminals, src_vertex=src_vertex,
                              dst_vertex=dst_vertex))


def _grid_edges(side: int) -> np.ndarray:
    e = []
    for r_ in range(side):
        for c_ in range(side):
            i = r_ * side + c_
            if c_ + 1 < side:
                e += [(i, i + 1), (i + 1, i)]
            if r_ + 1 < side:
                e += [(i, i + side), (i + side, i)]
    return np.array(e, dtype=np.int64)


def sparse_grid_edge_instance(side: int = 10, L: int = 50, T: int = 80, eps: float = 0.01,
                              seed: int = 0) -> Instance:
    """The shape of the paper's sparse-grid study (Section 5.1): a side x side grid
    of two-way streets, every commodity (unit mass) from one corner to the
    opposite corner, no storage on the streets, waiting only in the source and
    the sink (the routing lift), edge capacity 1 (the terminals take all L),
    per-commodity edge costs U[0, 1]."""
    rng = np.random.default_rng(seed)
    edges = _grid_edges(side)
    m = len(edges)
    cost = rng.uniform(0.0, 1.0, (L, m))
    return edge_state_instance(side * side, edges, L, T, eps, cost,
                               src_vertex=np.zeros(L, dtype=np.int64),
                               dst_vertex=np.full(L, side * side - 1, dtype=np.int64),
                               mass=np.ones(L), cap_edge=1.0, terminals="routing",
                               name=f"gridedges{side}")


def dense_random_edge_instance(nv: int = 40, p: float = 0.5, L: int = 100, T: int = 100,
                               eps: float = 0.0025, seed: int = 0) -> Instance:
    """The shape of the paper's dense-network study (Section 5.2): a directed edge
    between each ordered vertex pair with probability p, storage in the
    vertices (cost 0) but not on the edges, commodities of unit mass between
    random distinct vertices, capacity 1 on edges and L on vertices,
    per-commodity edge costs U[0, 1].  Draws whose sink is unreachable from
    the source within T steps are redrawn."""
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a in range(nv) for b in range(nv) if a != b]
    keep = rng.random(len(pairs)) < p
    edges = np.array([pr for pr, k in zip(pairs, keep) if k], dtype=np.int64)
    g = sp.csr_matrix((np.ones(len(edges)), (edges[:, 0], edges[:, 1])), shape=(nv, nv))
    hop = csgraph.shortest_path(g, directed=True, unweighted=True)
    s = np.empty(L, dtype=np.int64); z = np.empty(L, dtype=np.int64)
    k = 0
    while k < L:
        a, b = rng.integers(0, nv, 2)
        if a != b and 2 * hop[a, b] + 1 <= T:     # edge + vertex states alternate along a route
            s[k], z[k] = a, b
            k += 1
    cost = rng.uniform(0.0, 1.0, (L, len(edges)))
    return edge_state_instance(nv, edges, L, T, eps, cost, src_vertex=s, dst_vertex=z, mass=np.ones(L),
                               cap_edge=1.0, terminals="storage", cap_vertex=float(L),
                               name=f"denseedges{nv}")


def time_varying_instance(base: Instance, seed: int = 0, peak: float = 1.5, closed_frac: float = 0.03,
                          closed_span: float = 0.3) -> Instance:
    """A time-varying version of a CSR instance (Section 3.3: C_tau per move).

    Moves between distinct states cost base * (1 + peak * rush(tau)) with a
    smooth rush-hour profile rush(tau) = sin^2(pi tau / T) (waiting keeps its
    cost); a seeded closed_frac of the state pairs have both directions closed
    (+inf) during one window of closed_span * T consecutive steps at a seeded
    start.  The source/sink draws of the base instance are kept.  A dense
    instance gets the same profile on its finite moves, its costs of shape
    (T, n, n)."""
    if base.kind == "dense":
        return _time_varying_dense(base, seed, peak, closed_frac, closed_span)
    assert base.kind == "csr"
    rng = np.random.default_rng(seed)
    T = base.T
    rows = np.repeat(np.arange(base.n), np.diff(base.rowptr))
    move = rows != base.colidx
    tau = np.arange(T)
    rush = np.sin(np.pi * tau / max(T, 1)) ** 2
    cost = np.tile(base.cost, (T, 1))
    cost[:, move] *= (1.0 + peak * rush)[:, None]
    a = np.minimum(rows, base.colidx).astype(np.int64)
    b = np.maximum(rows, base.colidx).astype(np.int64)
    pair_id = a * base.n + b
    pairs = np.unique(pair_id[move])
    shut = rng.choice(pairs, size=int(round(closed_frac * len(pairs))), replace=False)
    span = max(1, int(round(closed_span * T)))
    for pid in shut:
        t0 = int(rng.integers(0, max(1, T - span + 1)))
        cost[t0:t0 + span, pair_id == pid] = np.inf
    return dataclasses.replace(base, name=base.name + "-tv", cost=cost, meta={**base.meta, "closed_pairs": shut})


def _time_varying_dense(base: Instance, seed, peak, closed_frac, closed_span) -> Instance:
    rng = np.random.default_rng(seed)
    T, n = base.T, base.n
    C0 = base.cost_dense
    move = np.isfinite(C0) & ~np.eye(n, dtype=bool)
    rush = np.sin(np.pi * np.arange(T) / max(T, 1)) ** 2
    cost = np.repeat(C0[None, :, :], T, axis=0)
    for t in range(T):
        cost[t][move] *= 1.0 + peak * rush[t]
    iu, ju = np.nonzero(np.triu(move, 1))
    shut = rng.choice(len(iu), size=int(round(closed_frac * len(iu))), replace=False)
    span = max(1, int(round(closed_span * T)))
    for q in shut:
        t0 = int(rng.integers(0, max(1, T - span + 1)))
        cost[t0:t0 + span, iu[q], ju[q]] = np.inf
        cost[t0:t0 + span, ju[q], iu[q]] = np.inf
    return dataclasses.replace(base, name=base.name + "-tv", cost_dense=cost,
                               meta={**base.meta, "closed_pairs": np.stack([iu[shut], ju[shut]], axis=1)})


def staggered_instance(base: Instance, enter: np.ndarray, leave: np.ndarray) -> Instance:
    """Commodities that enter and leave the network at their own times (Remark 8
    and Section 3.3), in the one-tensor form of the solver.

    base: a CSR instance with one source and one sink state per commodity
    (fixed or time-varying costs).  Commodity l is at its source s_l at time
    enter[l] and at its sink z_l at time leave[l] (0 <= enter < leave <= T) and
    counts against the capacities only in between.  Encoding, with a
    time-varying network: a holding state per distinct (enter > 0, s) where
    the commodity waits outside the network; it leads only to s, by the move
    enter-1 -> enter; an exit state per distinct (leave < T, z), reached from
    z only by the move leave -> leave+1 and kept afterwards.  Holding and exit
    states are uncapacitated and cost nothing; the source marginal sits on the
    holding state (or on s when enter = 0), the sink marginal on the exit state
    (or on z when leave = T)."""
    assert base.kind == "csr"
    L, n, T = base.L, base.n, base.T
    enter = np.asarray(enter, dtype=np.int64); leave = np.asarray(leave, dtype=np.int64)
    assert np.all(0 <= enter) and np.all(enter < leave) and np.all(leave <= T)
    assert np.all((base.src > 0).sum(axis=1) == 1) and np.all((base.dst > 0).sum(axis=1) == 1)
    s_of = base.src.argmax(axis=1); z_of = base.dst.argmax(axis=1); mass = base.src.sum(axis=1)
    hold = {}; exit_ = {}
    for l in range(L):
        if enter[l] > 0:
            hold.setdefault((int(enter[l]), int(s_of[l])), n + len(hold))
    for l in range(L):
        if leave[l] < T:
            exit_.setdefault((int(leave[l]), int(z_of[l])), n + len(hold) + len(exit_))
    n2 = n + len(hold) + len(exit_)
    base_cost = base.cost if np.ndim(base.cost) == 2 else np.tile(base.cost, (T, 1))
    rows = list(np.repeat(np.arange(n), np.diff(base.rowptr))); cols = list(base.colidx)
    steps = [list(base_cost[:, e]) for e in range(base.nnz)]
    inf = np.inf

    def add(i, j, open_at):
        rows.append(i); cols.append(j)
        steps.append([0.0 if open_at(tau) else inf for tau in range(T)])

    for (a, sn), h in hold.items():
        add(h, h, lambda tau, a=a: tau < a - 1)          # wait outside the network
        add(h, sn, lambda tau, a=a: tau == a - 1)        # enter at time a
    for (b, zn), x in exit_.items():
        add(zn, x, lambda tau, b=b: tau == b)            # leave right after time b
        add(x, x, lambda tau, b=b: tau > b)              # and stay out
    order = np.lexsort((np.array(cols), np.array(rows)))
    rows = np.array(rows)[order]; cols = np.array(cols)[order]
    cost = np.array(steps, dtype=np.float64)[order].T.copy()           # (T, nnz2)
    rowptr = np.zeros(n2 + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    src = np.zeros((L, n2)); dst = np.zeros((L, n2))
    for l in range(L):
        src[l, hold[(int(enter[l]), int(s_of[l]))] if enter[l] > 0 else s_of[l]] = mass[l]
        dst[l, exit_[(int(leave[l]), int(z_of[l]))] if leave[l] < T else z_of[l]] = mass[l]
    cap = base.cap_full()
    cap = np.concatenate([cap, np.full((cap.shape[0], n2 - n), np.inf)], axis=1)
    sc = None
    if base.state_cost is not None:
        sc = np.concatenate([base.state_cost, np.zeros((L, n2 - n))], axis=1)
    cc = None
    if base.cap_comm is not None:
        pad = np.full(base.cap_comm.shape[:-1] + (n2 - n,), np.inf)
        cc = np.concatenate([base.cap_comm, pad], axis=-1)
    return Instance(name=base.name + "-staggered", n=n2, L=L, T=T, eps=base.eps, kind="csr", src=src, dst=dst,
                    cap=cap, rowptr=rowptr, colidx=cols.astype(np.int32), cost=cost, state_cost=sc, cap_comm=cc,
                    meta={**base.meta, "enter": enter, "leave": leave, "n_network": n, "s_of": s_of, "z_of": z_of})


# ----------------------------------------------------------------------------
# serving trace
# ----------------------------------------------------------------------------

def serve_trace(num: int = 10000, rate: float = 100.0, seed: int = 0,
                n_range=(200, 10000), T_range=(10, 120), L_range=(1, 512),
                eps_choices=(0.02, 0.05, 0.1)) -> list:
    """Poisson-arriving solve requests (specs only; build with instance_from_request).

    Each request draws a generator (random geometric graph or road grid) with
    probability 1/2, n log-uniform in n_range, T uniform in T_range, L
    log-uniform in L_range and eps uniformly from eps_choices.  Arrival times
    are a Poisson process of the given rate (requests per second).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num)
    t = np.cumsum(gaps)
    reqs = []
    for r in range(num):
        gen = "rgg" if rng.random() < 0.5 else "grid"
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        L = max(1, int(round(math.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]))))))
        eps = float(rng.choice(eps_choices))
        reqs.append(dict(id=r, gen=gen, n=n, T=T, L=L, eps=eps, seed=int(rng.integers(1 << 31)),
                         arrival=float(t[r])))
    return reqs


def instance_from_request(req: dict) -> Instance:
    """Build a trace request.  Random-geometric-graph capacities are scaled by
    max(1, 8 L / n) so that many commodities on few nodes stay feasible."""
    if req["gen"] == "rgg":
        f = max(1.0, 8.0 * req["L"] / req["n"])
        return rgg_instance(n=req["n"], L=req["L"], T=req["T"], eps=req["eps"], seed=req["seed"],
                            cap_lo=0.2 * f, cap_hi=1.0 * f)
    side = max(2, int(round(math.sqrt(req["n"]))))
    return road_grid_instance(side=side, L=req["L"], T=req["T"], eps=req["eps"], seed=req["seed"])
