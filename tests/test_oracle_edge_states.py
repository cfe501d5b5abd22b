"""Pins of the edge-state lifts (CPU).

The paper's own state space is the edge a unit of flow is on (Section 3.1,
eq. T_cost: transition cost 0 where one edge leads to the next, the cost of
using an edge charged on the marginals), augmented by the vertices when flow
may be stored there, or by source and sink states for routing (Section 3.3,
eq. cost_traffic_routing).  When capacities do not bind, the unregularised
optimum of such a lift is the sum over commodities of the cheapest route in
the original graph under that commodity's edge costs -- computed here with
Dijkstra on the original graph, independently of the lift.  The Sinkhorn
oracle's plan on the lift then lies within the entropy bound above it.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

from oracle import alg2, lp_check
from paper_2106_14485_amd import instances
from tests.helpers import to_oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def cheapest_routes(inst):
    edges, nv = inst.meta["edges"], inst.meta["nv"]
    total = 0.0
    for l, (a, b) in enumerate(zip(inst.meta["src_vertex"], inst.meta["dst_vertex"])):
        g = sp.csr_matrix((inst.state_cost[l, : len(edges)], (edges[:, 0], edges[:, 1])), shape=(nv, nv))
        total += float(csgraph.dijkstra(g, directed=True, indices=int(a))[int(b)])
    return total


def _small_digraph(nv, p, seed):
    rng = np.random.default_rng(seed)
    e = [(a, b) for a in range(nv) for b in range(nv) if a != b and rng.random() < p]
    ring = [(a, (a + 1) % nv) for a in range(nv)]          # strongly connected
    return np.array(sorted(set(e) | set(ring)), dtype=np.int64)


def _lifts():
    grid = instances.sparse_grid_edge_instance(side=3, L=3, T=9, eps=0.02, seed=1)
    grid.cap = np.where(np.isfinite(grid.cap), 10.0, np.inf)          # capacities that do not bind
    edges = _small_digraph(5, 0.35, seed=2)
    rng = np.random.default_rng(3)
    st = instances.edge_state_instance(
        5, edges, L=3, T=8, eps=0.02, edge_cost=rng.uniform(0.1, 1.0, (3, len(edges))),
        src_vertex=np.array([0, 1, 4]), dst_vertex=np.array([3, 4, 2]), mass=np.array([1.0, 0.5, 2.0]),
        cap_edge=10.0, terminals="storage", cap_vertex=10.0, name="tiny-storage")
    return [grid, st]


@pytest.mark.parametrize("k", [0, 1])
def test_lift_lp_optimum_is_sum_of_cheapest_routes(k):
    inst = _lifts()[k]
    C = inst.cost_csr()
    assert C.nnz == inst.nnz and np.all(C.data == 0.0)        # explicit zero-cost moves are kept
    lp = lp_check.lp_optimum(C, inst.T, inst.src, inst.dst, inst.cap, inst.state_cost)
    masses = inst.src.sum(axis=1)
    routes = 0.0
    for l in range(inst.L):
        one = instances.Instance(**{**inst.__dict__, "L": 1, "src": inst.src[l:l + 1], "dst": inst.dst[l:l + 1],
                                    "state_cost": inst.state_cost[l:l + 1],
                                    "meta": {**inst.meta, "src_vertex": inst.meta["src_vertex"][l:l + 1],
                                             "dst_vertex": inst.meta["dst_vertex"][l:l + 1]}})
        routes += masses[l] * cheapest_routes(one)
    assert abs(lp - routes) <= 1e-7 * max(1.0, abs(routes)), (lp, routes)


@pytest.mark.parametrize("k", [0, 1])
def test_lift_sinkhorn_plan_within_entropy_bound(k):
    inst = _lifts()[k]
    p = to_oracle(inst)
    st = alg2.iterate_log(p, alg2.initial_log_state(p), 400)
    out = alg2.projections_log(p, st)
    C = inst.cost_csr()
    lp = lp_check.lp_optimum(C, inst.T, inst.src, inst.dst, inst.cap, inst.state_cost)
    s = inst.src.argmax(axis=1); z = inst.dst.argmax(axis=1)
    walks = lp_check.walk_counts(C, inst.T, s, z)
    bound = inst.eps * sum(m * np.log(w) for m, w in zip(inst.src.sum(axis=1), walks))
    gap = out["cost"] - lp
    assert -1e-6 <= gap <= bound + 1e-6, (gap, bound)
    # flow stays on the lift: each unit of a commodity occupies exactly one state per time
    assert np.allclose(out["P0t"].sum(axis=2), inst.src.sum(axis=1)[None, :], rtol=1e-9)


def test_routing_lift_forbids_storage_on_edges_and_reentry():
    inst = instances.sparse_grid_edge_instance(side=3, L=2, T=9, eps=0.1, seed=0)
    m = inst.meta["m"]
    C = inst.cost_csr().tocoo()
    pairs = set(zip(C.row.tolist(), C.col.tolist()))
    assert all((e, e) not in pairs for e in range(m))           # no waiting on a street
    src_state, sink_state = m, m + 1
    assert all(j != src_state for (i, j) in pairs if i != src_state)   # the source is never re-entered
    assert all(j == sink_state for (i, j) in pairs if i == sink_state)  # the sink is never left
