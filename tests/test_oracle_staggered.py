"""Pins of staggered entry and exit times (Remark 8, Section 3.3), CPU.

Commodity l is at its source s_l at time a_l and at its sink z_l at time b_l;
before a_l and after b_l it is outside the network and takes no capacity.  The
builder encodes this in one tensor over a time-varying network (holding and
exit states whose moves open at one step only).  Checked independently of
that encoding:

* with capacities that do not bind, the unregularised optimum is the sum over
  commodities of the cheapest time-expanded route from (a_l, s_l) to
  (b_l, z_l) under the per-step costs, by dynamic programming on the original
  network alone;
* the Sinkhorn oracle's plan puts each commodity exactly on its holding state
  before a_l, on s_l at a_l, on z_l at b_l and on its exit state after b_l,
  and is within the entropy bound of that optimum;
* a capacity of one on a corridor makes two commodities with the same
  window infeasible and lets through two whose windows are one step apart.
"""
import numpy as np
import pytest

from oracle import alg2, lp_check
from paper_2106_14485_amd import instances
from tests.helpers import to_oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _base(seed):
    g = instances.grid_instance(side=4, T=9, L=3, eps=0.05, cap=10.0, seed=seed, check_feasible=False)
    return instances.time_varying_instance(g, seed=seed, closed_frac=0.05)


def _times(seed, L, T):
    rng = np.random.default_rng(100 + seed)
    return rng.integers(0, 3, L), rng.integers(T - 1, T + 1, L)


def cheapest_timed_route(base, l, a, b):
    """min over walks i_a = s, ..., i_b = z of sum_tau C_tau[i_tau, i_tau+1]
    (plus interior state costs) on the original network, by DP over time."""
    C = base.cost_csr()
    s, z = int(base.src[l].argmax()), int(base.dst[l].argmax())
    V = np.full(base.n, np.inf); V[s] = 0.0
    if base.state_cost is not None and 0 < a < base.T:
        V[s] += base.state_cost[l, s]
    for tau in range(a, b):
        c = C[tau].tocoo()
        W = np.full(base.n, np.inf)
        np.minimum.at(W, c.col, V[c.row] + c.data)
        if base.state_cost is not None and tau + 1 < base.T:
            W = W + base.state_cost[l]
        V = W
    return float(V[z])


@pytest.mark.parametrize("seed", [0, 1])
def test_staggered_lp_is_sum_of_timed_routes(seed):
    base = _base(seed)
    a, b = _times(seed, base.L, base.T)
    st = instances.staggered_instance(base, a, b)
    lp = lp_check.lp_optimum(st.cost_csr(), st.T, st.src, st.dst, st.cap, st.state_cost)
    ref = sum(base.src[l].sum() * cheapest_timed_route(base, l, int(a[l]), int(b[l])) for l in range(base.L))
    assert np.isfinite(ref)
    assert abs(lp - ref) <= 1e-7 * max(1.0, abs(ref)), (lp, ref)


@pytest.mark.parametrize("seed", [0, 1])
def test_staggered_plan_respects_entry_and_exit(seed):
    base = _base(seed)
    a, b = _times(seed, base.L, base.T)
    st = instances.staggered_instance(base, a, b)
    p = to_oracle(st)
    s = alg2.iterate_log(p, alg2.initial_log_state(p), 300)
    out = alg2.projections_log(p, s)
    P = out["P0t"]                                         # (T+1, L, n)
    n0 = base.n
    for l in range(base.L):
        m = base.src[l].sum()
        sl, zl = int(base.src[l].argmax()), int(base.dst[l].argmax())
        assert abs(P[a[l], l, sl] - m) <= 1e-9 * m
        assert abs(P[b[l], l, zl] - m) <= 1e-9 * m
        for t in range(st.T + 1):
            inside = P[t, l, :n0].sum()
            assert abs(inside - (m if a[l] <= t <= b[l] else 0.0)) <= 1e-9 * m, (l, t)
    # within the entropy bound of the unregularised optimum
    C = st.cost_csr()
    lp = lp_check.lp_optimum(C, st.T, st.src, st.dst, st.cap, st.state_cost)
    walks = lp_check.walk_counts(C, st.T, st.src.argmax(axis=1), st.dst.argmax(axis=1))
    bound = st.eps * sum(mm * np.log(w) for mm, w in zip(st.src.sum(axis=1), walks))
    gap = out["cost"] - lp
    assert -1e-6 <= gap <= bound + 1e-6, (gap, bound)


def _corridor(T=6):
    """A path 0-1-2-3-4 with waiting everywhere and a capacity of 1 at the
    middle state 2; two unit commodities from 0 to 4."""
    n = 5
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i); cols.append(j)
    rows = np.array(rows); cols = np.array(cols)
    cost = np.where(rows == cols, 0.5, 1.0)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    src = np.zeros((2, n)); src[:, 0] = 1.0
    dst = np.zeros((2, n)); dst[:, 4] = 1.0
    cap = np.full(n, np.inf); cap[2] = 1.0
    return instances.Instance(name="corridor", n=n, L=2, T=T, eps=0.05, kind="csr", src=src, dst=dst,
                              cap=cap, rowptr=rowptr, colidx=cols.astype(np.int32), cost=cost)


def test_staggered_capacity_counts_only_commodities_inside():
    base = _corridor(T=6)
    # the cheapest route is four moves at cost 1; over the window [0, 4] it must
    # cross state 2 at time 2, so two commodities with that same window cannot
    # both fit the capacity of 1 there ...
    same = instances.staggered_instance(base, np.array([0, 0]), np.array([4, 4]))
    with pytest.raises(RuntimeError, match="infeasible"):
        lp_check.lp_optimum(same.cost_csr(), same.T, same.src, same.dst, same.cap)
    # ... while windows shifted by one step pass state 2 at times 2 and 3
    apart = instances.staggered_instance(base, np.array([0, 1]), np.array([4, 5]))
    lp_apart = lp_check.lp_optimum(apart.cost_csr(), apart.T, apart.src, apart.dst, apart.cap)
    assert lp_apart == pytest.approx(8.0, abs=1e-8)
    p = to_oracle(apart)
    out = alg2.projections_log(p, alg2.iterate_log(p, alg2.initial_log_state(p), 500))
    assert out["P0t"][1:-1, :, 2].sum(axis=1).max() <= 1.0 + 1e-3
    assert 8.0 - 1e-6 <= out["cost"] <= 8.0 + 2 * apart.eps * np.log(4.0)
