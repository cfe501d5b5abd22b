"""Pins of two oracle helpers that the other pins build on.

* lp_check.walk_counts (the walk counts |P_l| in the entropy-gap bound of
  Theorem 2's regularised problem) against integer matrix powers of the move
  adjacency (a length-T walk count is an entry of A^T, or of A_0 A_1 ... A_{T-1}
  for a time-varying network).
* alg2._dual_log, the log-domain dual objective of Theorem 3 (eq.
  omt_multi_graph_dual): equal to the plain-domain dual iterate by iterate,
  non-decreasing (block coordinate ascent, Proposition 1), and at convergence
  equal to the primal objective <C, M> + eps sum M (log M - 1) evaluated on the
  explicit tensor M = K (.) U (strong duality), which involves no scaling
  formula at all.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import alg2, bruteforce, lp_check
from paper_2106_14485_amd import instances
from tests.helpers import random_tiny, to_oracle


def _adjacency(C):
    A = sp.coo_matrix(C)
    n = A.shape[0]
    out = np.zeros((n, n), dtype=object)        # exact integers, no overflow
    for i, j, v in zip(A.row, A.col, A.data):
        if np.isfinite(v):
            out[i, j] = 1
    return out


def _matpow(A, T):
    n = A.shape[0]
    R = np.eye(n, dtype=np.int64).astype(object)
    for _ in range(T):
        R = R.dot(A)
    return R


def test_walk_counts_are_matrix_power_entries():
    inst = instances.grid_instance(side=4, T=9, L=3, check_feasible=False, seed=2)
    C = inst.cost_csr()
    src, snk = inst.src.argmax(axis=1), inst.dst.argmax(axis=1)
    got = lp_check.walk_counts(C, inst.T, src, snk)
    AT = _matpow(_adjacency(C), inst.T)
    assert got == [AT[s, z] for s, z in zip(src, snk)]
    assert all(g > 1 for g in got)
    # every ordered pair, on a small random digraph with some one-way moves
    rng = np.random.default_rng(5)
    n = 7
    pat = rng.random((n, n)) < 0.35
    np.fill_diagonal(pat, True)
    Cr = sp.csr_matrix(np.where(pat, 1.0, 0.0))
    Cr.data[:] = rng.uniform(0.5, 1.5, Cr.nnz)
    AT = _matpow(_adjacency(Cr), 6)
    ss, zz = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = lp_check.walk_counts(Cr, 6, ss.ravel(), zz.ravel())
    assert got == [AT[s, z] for s, z in zip(ss.ravel(), zz.ravel())]


def test_walk_counts_time_varying_is_a_matrix_chain():
    base = instances.rgg_instance(n=40, L=4, T=6, seed=2)
    inst = instances.time_varying_instance(base, seed=1, closed_frac=0.2)
    steps = inst.cost_csr()
    assert isinstance(steps, list) and len(steps) == inst.T
    src, snk = inst.src.argmax(axis=1), inst.dst.argmax(axis=1)
    got = lp_check.walk_counts(steps, inst.T, src, snk)
    R = _matpow(_adjacency(steps[0]), 0)
    for c in steps:
        R = R.dot(_adjacency(c))
    assert got == [R[s, z] for s, z in zip(src, snk)]
    # closing moves removes walks: fewer than on the base network
    full = lp_check.walk_counts(base.cost_csr(), base.T, src, snk)
    assert all(a <= b for a, b in zip(got, full)) and sum(got) < sum(full)


@pytest.mark.parametrize("which", ["grid", "rgg"])
def test_log_dual_equals_plain_dual(which):
    if which == "grid":
        inst = instances.grid_instance()
    else:
        inst = instances.rgg_instance(n=300, L=16, T=12, seed=1)
    p = to_oracle(inst)
    st = alg2.iterate(p, alg2.initial_state(p), 25)
    lst = alg2.iterate_log(p, alg2.initial_log_state(p), 25)
    g, lg = np.array(st.g), np.array(lst.g)
    assert np.abs(lg - g).max() <= 1e-12 * np.abs(g).max()
    assert np.all(np.diff(lg) >= -1e-12 * np.abs(lg).max())


def _primal_on_tensor(p, K, KL, lst):
    """<C, M> + eps sum M (log M - 1) on the explicit tensor of the log state."""
    with np.errstate(divide="ignore"):
        M = bruteforce.full_tensor(K, KL, np.exp(lst.lU01), np.exp(lst.lU0T), np.exp(lst.lu), p.T)
        Kfull = bruteforce.full_tensor(K, KL, np.ones((p.L, p.n)), np.ones((p.L, p.n)),
                                       np.ones((p.T - 1, p.n)), p.T)
    pos = M > 0
    Cfull = -p.eps * np.log(Kfull[pos])           # path cost incl. state costs
    return float((M[pos] * Cfull).sum() + p.eps * (M[pos] * (np.log(M[pos]) - 1.0)).sum())


@pytest.mark.parametrize("seed", [0, 5])
def test_log_dual_meets_primal_on_the_tensor(seed):
    """Strong duality (Theorem 3): at the converged iterate of the log oracle
    the dual it reports equals the primal value of the plan on the explicit
    tensor.  The capacities bind (u < 1 somewhere), so the capacity term of the
    dual is exercised; dropping it, or flipping a sign, breaks the equality."""
    p, _ = random_tiny(n=4, T=4, L=2, seed=seed, cap_scale=0.5, eps=0.5)
    lst = alg2.iterate_log(p, alg2.initial_log_state(p), 3000)
    assert (lst.lu < -1e-3).any()
    K = alg2.gibbs(p).toarray()
    KL = alg2.gibbs_state(p)
    prim = _primal_on_tensor(p, K, KL, lst)
    g = lst.g[-1]
    assert abs(prim - g) <= 1e-9 * abs(g), (prim, g)
    # the capacity term is not negligible here: without it the dual would be off
    fin = np.isfinite(p.cap)
    cap_term = p.eps * (p.cap[fin] * lst.lu[fin]).sum()
    assert abs(cap_term) > 1e3 * abs(prim - g)
