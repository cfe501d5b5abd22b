"""Oracle vs closed forms: Schroedinger bridge, two-route capacity split, two-marginal structure."""
import json
import os

import numpy as np
import scipy.sparse as sp

from oracle import alg2, closed_forms
from paper_2106_14485_amd import instances
from tests.helpers import dense_flow, rel_l1, to_oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_markov_bridge_after_one_iteration():
    inst = instances.grid_instance(side=4, T=7, L=1, check_feasible=False, seed=3)
    inst.cap = np.full(inst.n, np.inf)
    p = to_oracle(inst)
    st = alg2.iterate(p, alg2.initial_state(p), 1)
    out = alg2.projections(p, st)
    K = alg2.gibbs(p).toarray()
    s = int(inst.meta["sources"][0]); z = int(inst.meta["sinks"][0])
    ref = closed_forms.bridge_marginals(K, s, z, p.T, mass=1.0)
    for tau in range(p.T + 1):
        assert rel_l1(out["Pt"][tau], ref[tau]) < 1e-12
    # a second iteration does not move anything (fixed point reached)
    st2 = alg2.iterate(p, st, 1)
    out2 = alg2.projections(p, st2)
    assert rel_l1(out2["Pt"], out["Pt"]) < 1e-13


def test_two_route_capacity_split_golden():
    with open(os.path.join(GOLDEN, "two_route.json")) as f:
        g = json.load(f)
    ca, cb, eps, da = g["ca"], g["cb"], g["eps"], g["d_a"]
    # states s=0, a=1, b=2, z=3
    C = sp.csr_matrix((np.array([ca, cb, 0.0, 0.0]), (np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3]))), shape=(4, 4))
    src = np.array([[1.0, 0, 0, 0]]); dst = np.array([[0, 0, 0, 1.0]])
    cap = np.array([[np.inf, da, np.inf, np.inf]])
    p = alg2.make_problem(C, eps, 2, src, dst, cap)
    st = alg2.iterate(p, alg2.initial_state(p), 400)
    out = alg2.projections(p, st)
    expect = np.array(g["expected_occupancy_a_b"])
    assert np.allclose(out["Pt"][1][1:3], expect, atol=1e-12, rtol=0)
    assert np.allclose(closed_forms.two_route_split(ca, cb, eps, da), expect, atol=1e-15)
    # without the cap the split is the Gibbs split
    p2 = alg2.make_problem(C, eps, 2, src, dst, np.full((1, 4), np.inf))
    out2 = alg2.projections(p2, alg2.iterate(p2, alg2.initial_state(p2), 5))
    free = 1.0 / (1.0 + np.exp((ca - cb) / eps))
    assert abs(out2["Pt"][1][1] - free) < 1e-14


def test_two_marginal_limit_is_diagonal_scaling():
    rng = np.random.default_rng(0)
    n = 6
    C = rng.uniform(0, 1, (n, n))
    C[rng.random((n, n)) < 0.3] = np.inf
    np.fill_diagonal(C, 0.1)
    a = rng.uniform(0.5, 1.5, (1, n)); b = rng.uniform(0.5, 1.5, (1, n)); b *= a.sum() / b.sum()
    p = alg2.make_problem(C, 0.3, 1, a, b, np.zeros((0, n)))
    st = alg2.iterate(p, alg2.initial_state(p), 3000)
    out = alg2.projections(p, st)
    M = dense_flow(out["flows"][0])
    assert np.allclose(M.sum(1), a[0], rtol=1e-9, atol=0)
    assert np.allclose(M.sum(0), b[0], rtol=1e-12, atol=0)
    assert closed_forms.rank_one_residual(M, alg2.gibbs(p), None, None) < 1e-10


def test_rank_one_residual_rejects_a_non_scaling():
    """The residual is not blind: a matrix that is not diag(a) K diag(b) -- one
    entry of a scaled kernel moved by a factor 1.5, or the kernel of another
    cost -- leaves a misfit the row and column terms cannot absorb."""
    rng = np.random.default_rng(3)
    n = 6
    C = rng.uniform(0, 1, (n, n))
    C[rng.random((n, n)) < 0.3] = np.inf
    np.fill_diagonal(C, 0.1)
    K = np.exp(-C / 0.3)
    a = rng.uniform(0.5, 2.0, n); b = rng.uniform(0.5, 2.0, n)
    M = a[:, None] * K * b[None, :]
    assert closed_forms.rank_one_residual(M, K, None, None) < 1e-12
    bad = M.copy()
    i, j = 2, 2                                   # a diagonal entry: its row and column hold others
    bad[i, j] *= 1.5
    assert closed_forms.rank_one_residual(bad, K, None, None) > 1e-3
    other = a[:, None] * np.exp(-np.where(np.isfinite(C), C ** 2, np.inf) / 0.3) * b[None, :]
    assert closed_forms.rank_one_residual(other, K, None, None) > 1e-3
