"""Pins of commodity-dependent capacities P_{0,t} <= D_t (the extension at
the end of Section 3), CPU.

* message passing with the extra scalings w_t against the explicit tensor
  whose entries carry prod_t w_t[l, i_t] (Theorem 5 / Corollary 1);
* the oracle iteration against the generic Sinkhorn updates applied to the
  explicit tensor (w_t projected right before u_t), plain and log domain,
  with binding, non-binding and zero capacities;
* one commodity: capacities on the commodity are the joint capacities, so
  the two formulations give the same plan iterate for iterate;
* the LP entropy gap with the extra constraints, and at the fixed point
  complementary slackness (w_t < 1 only where P_{0,t} = D_t);
* a zero capacity closes a state to one commodity and not to the others.
"""
import numpy as np
import pytest

from oracle import alg2, bruteforce, lp_check
from tests.helpers import dense_flow, random_tiny, rel_l1

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _with_comm(p, seed, scale=0.5, zero_frac=0.1, inf_frac=0.3):
    rng = np.random.default_rng(seed)
    shape = (p.T - 1, p.L, p.n)
    D = rng.uniform(0.3, 1.0, shape) * scale * p.src.sum(axis=1)[None, :, None]
    D[rng.random(shape) < inf_frac] = np.inf
    D[rng.random(shape) < zero_frac] = 0.0
    return alg2.make_problem(p.C, p.eps, p.T, p.src, p.dst, p.cap, p.state_cost, D)


def _dense_K(p):
    return alg2.gibbs(p).toarray()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_comm_projections_match_full_tensor(seed):
    p0, _ = random_tiny(n=4, T=4, L=3, seed=seed)
    p = _with_comm(p0, 10 + seed)
    rng = np.random.default_rng(300 + seed)
    st = alg2.initial_state(p)
    st.U01 = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.src > 0)
    st.U0T = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.dst > 0)
    st.u = rng.uniform(0.1, 1.0, st.u.shape)
    st.w = rng.uniform(0.0, 1.0, st.w.shape)
    out = alg2.projections(p, st)
    M = bruteforce.full_tensor(_dense_K(p), alg2.gibbs_state(p), st.U01, st.U0T, st.u, p.T, st.w)
    P0t, Pt, pairs = bruteforce.tensor_projections(M, p.T)
    for tau in range(p.T + 1):
        assert rel_l1(out["P0t"][tau], P0t[tau]) < 1e-13
    for tau in range(p.T):
        assert rel_l1(dense_flow(out["flows"][tau]), pairs[tau]) < 1e-13
    # w matters
    st1 = alg2.initial_state(p)
    st1.U01, st1.U0T, st1.u = st.U01, st.U0T, st.u
    assert rel_l1(alg2.projections(p, st1)["P0t"], out["P0t"]) > 1e-3


@pytest.mark.parametrize("seed,T", [(0, 3), (1, 4), (2, 4)])
def test_comm_iterates_match_tensor_sinkhorn(seed, T):
    p0, _ = random_tiny(n=4, T=T, L=2, seed=seed, cap_scale=0.5)
    p = _with_comm(p0, 20 + seed)
    st = alg2.iterate(p, alg2.initial_state(p), 6)
    U01, U0T, u, w = bruteforce.tensor_sinkhorn(_dense_K(p), alg2.gibbs_state(p), p.src, p.dst, p.cap, p.T, 6,
                                                cap_comm=p.cap_comm)
    assert rel_l1(st.U01, U01) < 1e-12
    assert rel_l1(st.U0T, U0T) < 1e-12
    assert rel_l1(st.u, u) < 1e-12
    assert rel_l1(st.w, w) < 1e-12
    assert np.array_equal(st.w == 0, w == 0) and np.all(w[p.cap_comm == 0] == 0)
    lst = alg2.iterate_log(p, alg2.initial_log_state(p), 6)
    assert rel_l1(np.exp(lst.lU0T), U0T) < 1e-12
    assert rel_l1(np.exp(lst.lu), u) < 1e-12
    assert rel_l1(np.exp(lst.lw), w) < 1e-12
    # the dual objective still increases (block coordinate ascent)
    assert np.all(np.diff(st.g) >= -1e-12 * np.abs(st.g[1:]))


def test_single_commodity_comm_caps_are_joint_caps():
    p0, _ = random_tiny(n=5, T=5, L=1, seed=7, cap_scale=0.4)
    joint = p0
    comm = alg2.make_problem(p0.C, p0.eps, p0.T, p0.src, p0.dst, np.full(p0.n, np.inf), p0.state_cost,
                             p0.cap[:, None, :])
    a = alg2.iterate(joint, alg2.initial_state(joint), 25)
    b = alg2.iterate(comm, alg2.initial_state(comm), 25)
    assert rel_l1(b.w[:, 0, :], a.u) < 1e-13
    assert np.all(b.u == 1.0)
    pa = alg2.projections(joint, a)
    pb = alg2.projections(comm, b)
    assert rel_l1(pa["P0t"], pb["P0t"]) < 1e-13
    assert abs(a.g[-1] - b.g[-1]) <= 1e-12 * abs(a.g[-1])


def test_comm_caps_lp_entropy_gap_and_slackness():
    p0, _ = random_tiny(n=4, T=4, L=2, seed=9, cap_scale=1.5, state_cost=False, point=True, eps=0.05)
    D = np.full((p0.T - 1, p0.L, p0.n), np.inf)
    # cap the first commodity below its mass on the state it uses most in the uncapacitated plan
    free = alg2.projections_log(p0, alg2.iterate_log(p0, alg2.initial_log_state(p0), 400))["P0t"]
    tau, i = np.unravel_index(np.argmax(free[1:-1, 0, :]), free[1:-1, 0, :].shape)
    D[tau, 0, i] = 0.5 * free[1 + tau, 0, i]
    p = alg2.make_problem(p0.C, p0.eps, p0.T, p0.src, p0.dst, p0.cap, None, D)
    st = alg2.iterate_log(p, alg2.initial_log_state(p), 3000)
    out = alg2.projections_log(p, st)
    lp = lp_check.lp_optimum(p.C, p.T, p.src, p.dst, p.cap, cap_comm=D)
    lp_free = lp_check.lp_optimum(p.C, p.T, p.src, p.dst, p.cap)
    assert lp >= lp_free - 1e-9
    walks = lp_check.walk_counts(p.C, p.T, p.src.argmax(axis=1), p.dst.argmax(axis=1))
    bound = p.eps * sum(m * np.log(w) for m, w in zip(p.src.sum(axis=1), walks))
    gap = out["cost"] - lp
    assert -1e-6 <= gap <= bound + 1e-6, (gap, bound)
    P = out["P0t"][1:-1]
    fin = np.isfinite(D)
    assert np.all(P[fin] <= D[fin] * (1 + 1e-6))
    active = np.exp(st.lw) < 1 - 1e-6
    assert active.any()
    assert np.allclose(P[active], D[active], rtol=1e-6)


def test_zero_comm_capacity_closes_a_state_to_one_commodity():
    p0, _ = random_tiny(n=5, T=5, L=2, seed=3, cap_scale=10.0, state_cost=False)
    D = np.full((p0.T - 1, p0.L, p0.n), np.inf)
    D[:, 0, 2] = 0.0
    p = alg2.make_problem(p0.C, p0.eps, p0.T, p0.src, p0.dst, p0.cap, None, D)
    out = alg2.projections(p, alg2.iterate(p, alg2.initial_state(p), 30))
    assert np.all(out["P0t"][1:-1, 0, 2] == 0.0)
    assert np.all(out["P0t"][1:-1, 1, 2] > 0.0)
