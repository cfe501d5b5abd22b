"""Pins of the time-varying network (CPU): C replaced by one matrix C_tau per
move tau -> tau+1 (Section 3.3), same sparsity at every step, +inf closing a
move at a step.

* message passing (Theorem 5 / Corollary 1 with K_tau) against the explicit
  tensor whose entries multiply K_tau[i_tau, i_tau+1];
* Proposition 1 updates on that tensor against the oracle iteration;
* the uncapacitated point-to-point bridge after one iteration against plain
  matrix-chain products P_t[i] = m (K_0 ... K_{t-1})[s, i] (K_t ... K_{T-1})[i, z]
  / (K_0 ... K_{T-1})[s, z];
* the LP entropy gap with per-step costs and closures;
* plain and log oracles agree.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import alg2, bruteforce, lp_check
from tests.helpers import dense_flow, random_tiny, rel_l1


def _per_step(p, seed, close_frac=0.15):
    """The same pattern at every step with costs redrawn per step; a few moves
    (never a self-loop, so every state can still wait) closed at some steps."""
    rng = np.random.default_rng(seed)
    C = p.C.tocsr() if sp.issparse(p.C) else sp.csr_matrix(np.where(np.isfinite(p.C), p.C, 0.0))
    Cs = []
    rows = np.repeat(np.arange(C.shape[0]), np.diff(C.indptr))
    for tau in range(p.T):
        c = C.copy()
        c.data = rng.uniform(0.0, 1.0, c.nnz)
        shut = (rng.random(c.nnz) < close_frac) & (rows != c.indices)
        c.data[shut] = np.inf
        Cs.append(c)
    return alg2.make_problem(Cs, p.eps, p.T, p.src, p.dst, p.cap, p.state_cost)


def _dense_Ks(p):
    return [k.toarray() for k in alg2.gibbs(p)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_time_varying_projections_match_full_tensor(seed):
    p0, _ = random_tiny(n=4, T=4, L=3, seed=seed)
    p = _per_step(p0, 50 + seed)
    rng = np.random.default_rng(200 + seed)
    st = alg2.initial_state(p)
    st.U01 = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.src > 0)
    st.U0T = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.dst > 0)
    st.u = rng.uniform(0.1, 1.0, st.u.shape)
    out = alg2.projections(p, st)
    Ks = _dense_Ks(p)
    M = bruteforce.full_tensor(Ks, alg2.gibbs_state(p), st.U01, st.U0T, st.u, p.T)
    P0t, Pt, pairs = bruteforce.tensor_projections(M, p.T)
    for tau in range(p.T + 1):
        assert rel_l1(out["P0t"][tau], P0t[tau]) < 1e-13
    for tau in range(p.T):
        assert rel_l1(dense_flow(out["flows"][tau]), pairs[tau]) < 1e-13
        closed = ~np.isfinite(p.C[tau].toarray()) & (p.C[tau].toarray() != 0)
        assert np.all(dense_flow(out["flows"][tau])[closed] == 0.0)
    Cf = [np.where(K > 0, c.toarray(), 0.0) for K, c in zip(Ks, p.C)]
    brute = sum((Cf[tau] * pairs[tau]).sum() for tau in range(p.T))
    brute += sum((p.state_cost * P0t[tau]).sum() for tau in range(1, p.T))
    assert abs(out["cost"] - brute) <= 1e-12 * abs(brute)
    # the time-varying kernels matter: the fixed first-step network gives other marginals
    fixed = alg2.make_problem(p.C[0], p.eps, p.T, p.src, p.dst, p.cap, p.state_cost)
    assert rel_l1(alg2.projections(fixed, st)["P0t"], out["P0t"]) > 1e-3


@pytest.mark.parametrize("seed", [0, 1])
def test_time_varying_dense_projections_match_full_tensor(seed):
    """The same pin with dense per-step cost matrices (+inf closing a move at a
    step): message passing, per-commodity marginals, flows (dense K_tau times a
    matrix product) and the transport cost against the explicit tensor."""
    p0, C0 = random_tiny(n=4, T=4, L=3, seed=seed, kind="dense")
    rng = np.random.default_rng(300 + seed)
    Cs = []
    for tau in range(p0.T):
        c = np.where(np.isfinite(C0), rng.uniform(0.0, 1.0, C0.shape), np.inf)
        shut = (rng.random(C0.shape) < 0.15) & ~np.eye(p0.n, dtype=bool)
        c[shut] = np.inf
        Cs.append(c)
    p = alg2.make_problem(Cs, p0.eps, p0.T, p0.src, p0.dst, p0.cap, p0.state_cost)
    st = alg2.initial_state(p)
    st.U01 = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.src > 0)
    st.U0T = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.dst > 0)
    st.u = rng.uniform(0.1, 1.0, st.u.shape)
    out = alg2.projections(p, st)
    Ks = alg2.gibbs(p)
    M = bruteforce.full_tensor(Ks, alg2.gibbs_state(p), st.U01, st.U0T, st.u, p.T)
    P0t, Pt, pairs = bruteforce.tensor_projections(M, p.T)
    for tau in range(p.T + 1):
        assert rel_l1(out["P0t"][tau], P0t[tau]) < 1e-13
    for tau in range(p.T):
        assert rel_l1(dense_flow(out["flows"][tau]), pairs[tau]) < 1e-13
        assert np.all(dense_flow(out["flows"][tau])[~np.isfinite(Cs[tau])] == 0.0)
    brute = sum((np.where(Ks[tau] > 0, Cs[tau], 0.0) * pairs[tau]).sum() for tau in range(p.T))
    brute += sum((p.state_cost * P0t[tau]).sum() for tau in range(1, p.T))
    assert abs(out["cost"] - brute) <= 1e-12 * abs(brute)


@pytest.mark.parametrize("seed,T", [(0, 3), (3, 4)])
def test_time_varying_iterates_match_tensor_sinkhorn(seed, T):
    p0, _ = random_tiny(n=4, T=T, L=2, seed=seed, cap_scale=0.35, state_cost=False)
    p = _per_step(p0, 70 + seed, close_frac=0.1)
    st = alg2.iterate(p, alg2.initial_state(p), 6)
    U01, U0T, u = bruteforce.tensor_sinkhorn(_dense_Ks(p), alg2.gibbs_state(p), p.src, p.dst, p.cap, p.T, 6)
    assert rel_l1(st.U01, U01) < 1e-12
    assert rel_l1(st.U0T, U0T) < 1e-12
    assert rel_l1(st.u, u) < 1e-12
    lst = alg2.iterate_log(p, alg2.initial_log_state(p), 6)
    assert rel_l1(np.exp(lst.lU0T), U0T) < 1e-12
    assert rel_l1(np.exp(lst.lu), u) < 1e-12


def test_time_varying_bridge_is_a_matrix_chain():
    rng = np.random.default_rng(4)
    n, T = 6, 5
    pat = rng.random((n, n)) < 0.5
    np.fill_diagonal(pat, True)
    r, c = np.nonzero(pat)
    Cs = []
    for tau in range(T):
        vals = rng.uniform(0.0, 2.0, len(r))
        vals[(rng.random(len(r)) < 0.2) & (r != c)] = np.inf
        Cs.append(sp.csr_matrix((vals, (r, c)), shape=(n, n)))
    s, z, m = 1, 4, 1.7
    src = np.zeros((1, n)); src[0, s] = m
    dst = np.zeros((1, n)); dst[0, z] = m
    p = alg2.make_problem(Cs, 0.3, T, src, dst, np.full(n, np.inf))
    st = alg2.iterate(p, alg2.initial_state(p), 1)
    out = alg2.projections(p, st)
    Ks = [np.where(np.isfinite(cc.toarray()) & pat, np.exp(-cc.toarray() / 0.3), 0.0) for cc in Cs]
    eye = np.eye(n)
    for t in range(T + 1):
        head = eye.copy()
        for k in Ks[:t]:
            head = head @ k
        tail = eye.copy()
        for k in Ks[t:]:
            tail = tail @ k
        ref = m * head[s, :] * tail[:, z] / (head @ tail)[s, z]
        assert rel_l1(out["Pt"][t], ref) < 1e-12


def test_time_varying_lp_entropy_gap():
    p0, _ = random_tiny(n=4, T=4, L=2, seed=9, cap_scale=0.8, state_cost=False, point=True)
    p = _per_step(p0, 91, close_frac=0.1)
    st = alg2.iterate_log(p, alg2.initial_log_state(p), 2000)
    out = alg2.projections_log(p, st)
    lp = lp_check.lp_optimum(p.C, p.T, p.src, p.dst, p.cap)
    walks = lp_check.walk_counts(p.C, p.T, p.src.argmax(axis=1), p.dst.argmax(axis=1))
    bound = p.eps * sum(mm * np.log(w) for mm, w in zip(p.src.sum(axis=1), walks))
    gap = out["cost"] - lp
    assert -1e-6 <= gap <= bound + 1e-6, (gap, bound)


def test_time_varying_plain_and_log_oracles_agree():
    p0, _ = random_tiny(n=5, T=5, L=3, seed=12, cap_scale=0.4)
    p = _per_step(p0, 120)
    a = alg2.projections(p, alg2.iterate(p, alg2.initial_state(p), 40))
    b = alg2.projections_log(p, alg2.iterate_log(p, alg2.initial_log_state(p), 40))
    assert rel_l1(a["P0t"], b["P0t"]) < 1e-12
    assert abs(a["cost"] - b["cost"]) < 1e-12 * abs(a["cost"])
