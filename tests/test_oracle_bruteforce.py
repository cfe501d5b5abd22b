"""Oracle message passing vs the explicit tensor (Theorem 5, Corollary 1, Proposition 1)."""
import numpy as np
import pytest

from oracle import alg2, bruteforce
from tests.helpers import dense_flow, random_tiny, rel_l1


def _dense_K(p):
    K = alg2.gibbs(p)
    return K.toarray() if hasattr(K, "toarray") else K


@pytest.mark.parametrize("seed,kind", [(0, "csr"), (1, "csr"), (2, "dense"), (3, "csr")])
def test_projections_match_full_tensor(seed, kind):
    p, _ = random_tiny(n=4, T=4, L=3, seed=seed, kind=kind)
    rng = np.random.default_rng(100 + seed)
    st = alg2.initial_state(p)
    st.U01 = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.src > 0)
    st.U0T = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.dst > 0)
    st.u = rng.uniform(0.1, 1.0, st.u.shape)
    out = alg2.projections(p, st)
    K = _dense_K(p)
    KL = alg2.gibbs_state(p)
    M = bruteforce.full_tensor(K, KL, st.U01, st.U0T, st.u, p.T)
    P0t, Pt, pairs = bruteforce.tensor_projections(M, p.T)
    for tau in range(p.T + 1):
        assert rel_l1(out["P0t"][tau], P0t[tau]) < 1e-13
        assert rel_l1(out["Pt"][tau], Pt[tau]) < 1e-13
    for tau in range(p.T):
        assert rel_l1(dense_flow(out["flows"][tau]), pairs[tau]) < 1e-13
    # transport cost <C, M> from the tensor
    Cfull = np.where(K > 0, p.C.toarray() if hasattr(p.C, "toarray") else p.C, 0.0)
    brute_cost = sum((Cfull * pairs[tau]).sum() for tau in range(p.T))
    brute_cost += sum((p.state_cost * P0t[tau]).sum() for tau in range(1, p.T))
    assert abs(out["cost"] - brute_cost) <= 1e-12 * abs(brute_cost)


@pytest.mark.parametrize("seed,T", [(0, 3), (1, 4), (2, 5), (4, 1), (5, 2)])
def test_iterates_match_tensor_sinkhorn(seed, T):
    p, _ = random_tiny(n=4, T=T, L=2, seed=seed, cap_scale=0.35)
    st = alg2.iterate(p, alg2.initial_state(p), 6)
    K = _dense_K(p)
    KL = alg2.gibbs_state(p)
    U01, U0T, u = bruteforce.tensor_sinkhorn(K, KL, p.src, p.dst, p.cap, p.T, 6)
    assert rel_l1(st.U01, U01) < 1e-12
    assert rel_l1(st.U0T, U0T) < 1e-12
    if T > 1:
        assert rel_l1(st.u, u) < 1e-12
        assert np.any(st.u < 1.0), "instance should have active capacities"


def test_log_oracle_matches_tensor():
    p, _ = random_tiny(n=4, T=4, L=2, seed=7, cap_scale=0.35)
    lst = alg2.iterate_log(p, alg2.initial_log_state(p), 6)
    K = _dense_K(p)
    U01, U0T, u = bruteforce.tensor_sinkhorn(K, alg2.gibbs_state(p), p.src, p.dst, p.cap, p.T, 6)
    assert rel_l1(np.exp(lst.lU01), U01) < 1e-12
    assert rel_l1(np.exp(lst.lU0T), U0T) < 1e-12
    assert rel_l1(np.exp(lst.lu), u) < 1e-12


def test_planted_mistake_is_caught():
    """A transposed operand in the forward product must break the brute-force pin."""
    p, _ = random_tiny(n=4, T=3, L=2, seed=11, density=0.5)
    K = _dense_K(p)
    assert np.abs(K - K.T).max() > 1e-3
    st = alg2.initial_state(p)
    rng = np.random.default_rng(5)
    st.U01 = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.src > 0)
    st.U0T = rng.uniform(0.2, 2.0, (p.L, p.n)) * (p.dst > 0)
    st.u = rng.uniform(0.1, 1.0, st.u.shape)
    good = alg2.projections(p, st)
    orig = alg2._right
    try:
        alg2._right = alg2._right_t          # planted: X K^T instead of X K
        bad = alg2.projections(p, st)
    finally:
        alg2._right = orig
    M = bruteforce.full_tensor(K, alg2.gibbs_state(p), st.U01, st.U0T, st.u, p.T)
    P0t, _, _ = bruteforce.tensor_projections(M, p.T)
    assert rel_l1(good["P0t"][1], P0t[1]) < 1e-13
    assert rel_l1(bad["P0t"][1], P0t[1]) > 1e-3
