"""Oracle invariants (mass identity, marginal equalities, dual ascent, convergence) and LP bound."""
import numpy as np
import pytest

from oracle import alg2, lp_check
from paper_2106_14485_amd import instances
from tests.helpers import dense_flow, rel_l1, to_oracle


@pytest.fixture(scope="module")
def grid_run():
    inst = instances.grid_instance()          # 5x5 grid, T=10, L=3, eps=0.1, cap 0.5
    p = to_oracle(inst)
    st = alg2.initial_state(p)
    outs = []
    for _ in range(4):
        alg2.iterate(p, st, 50)
        outs.append(alg2.projections(p, st))
    return inst, p, st, outs


def test_per_iterate_invariants(grid_run):
    inst, p, st, outs = grid_run
    for out in outs:
        # Corollary 1: per-commodity mass is the same at every time
        m = out["mass"]
        assert np.abs(m - m[0][None, :]).max() <= 1e-12 * m.max()
        # after the sink update the sink marginal is met exactly
        assert np.abs(out["P0t"][-1] - p.dst).max() <= 1e-13
        assert (out["P0t"] >= 0).all()
    assert (st.u > 0).all() and (st.u <= 1).all()


def test_dual_objective_nondecreasing(grid_run):
    _, _, st, _ = grid_run
    g = np.array(st.g)
    assert np.all(np.diff(g) >= -1e-12 * np.abs(g).max())
    assert g[-1] > g[0]


def test_convergence_and_complementary_slackness(grid_run):
    inst, p, st, outs = grid_run
    out = outs[-1]
    Pt = out["Pt"][1:-1]
    viol = np.maximum(Pt - p.cap, 0).max()
    assert viol < 1e-6
    assert rel_l1(out["P0t"][0], p.src) < 1e-6
    active = st.u < 1 - 1e-6
    assert active.any()
    assert np.abs(Pt[active] - p.cap[active]).max() < 1e-5
    # the duality gap closes
    g = st.g[-1]
    prim = p.eps * (np.sum(np.where(p.src > 0, out["P0t"][0] * np.log(np.where(st.U01 > 0, st.U01, 1)), 0))
                    + np.sum(np.where(p.dst > 0, out["P0t"][-1] * np.log(np.where(st.U0T > 0, st.U0T, 1)), 0))
                    + np.sum(Pt * np.log(st.u))) - p.eps * out["mass"][0].sum()
    assert abs(prim - g) < 1e-5 * abs(g)


def test_plain_and_log_oracles_agree():
    for inst in (instances.grid_instance(), instances.rgg_instance(n=300, L=16, T=12, seed=1)):
        p = to_oracle(inst)
        st = alg2.iterate(p, alg2.initial_state(p), 15)
        lst = alg2.iterate_log(p, alg2.initial_log_state(p), 15)
        assert rel_l1(np.exp(lst.lU01), st.U01) < 1e-12
        assert rel_l1(np.exp(lst.lU0T), st.U0T) < 1e-12
        assert rel_l1(np.exp(lst.lu), st.u) < 1e-12
        a = alg2.projections(p, st)
        b = alg2.projections_log(p, lst)
        assert rel_l1(b["Pt"], a["Pt"]) < 1e-12
        fa = np.concatenate([dense_flow(f).ravel() for f in a["flows"]])
        fb = np.concatenate([dense_flow(f).ravel() for f in b["flows"]])
        assert rel_l1(fb, fa) < 1e-12
        assert abs(a["cost"] - b["cost"]) < 1e-11 * abs(a["cost"])


def test_commodity_split_invariance():
    inst = instances.rgg_instance(n=200, L=6, T=8, seed=2)
    p = to_oracle(inst)
    st = alg2.iterate(p, alg2.initial_state(p), 10)
    a = alg2.projections(p, st)
    src2 = np.concatenate([p.src, p.src[:1] * 0.5]); src2[0] *= 0.5
    dst2 = np.concatenate([p.dst, p.dst[:1] * 0.5]); dst2[0] *= 0.5
    p2 = alg2.make_problem(p.C, p.eps, p.T, src2, dst2, p.cap)
    st2 = alg2.iterate(p2, alg2.initial_state(p2), 10)
    b = alg2.projections(p2, st2)
    assert rel_l1(b["Pt"], a["Pt"]) < 1e-13
    assert rel_l1(b["P0t"][:, 0], 0.5 * a["P0t"][:, 0]) < 1e-13
    assert rel_l1(b["P0t"][:, -1], 0.5 * a["P0t"][:, 0]) < 1e-13


def test_time_reversal_at_convergence():
    inst = instances.grid_instance(side=4, T=6, L=2, cap=0.6, eps=0.3, seed=5)
    p = to_oracle(inst)          # grid costs are symmetric
    st = alg2.iterate(p, alg2.initial_state(p), 600)
    assert (st.u < 1 - 1e-6).any(), "capacities must be active for the check to mean anything"
    a = alg2.projections(p, st)
    pr = alg2.make_problem(p.C, p.eps, p.T, p.dst, p.src, p.cap[::-1])
    sr = alg2.iterate(pr, alg2.initial_state(pr), 600)
    b = alg2.projections(pr, sr)
    assert rel_l1(b["Pt"][::-1], a["Pt"]) < 1e-8


@pytest.mark.parametrize("eps", [0.2, 0.1])
def test_lp_entropy_gap_bound(eps):
    inst = instances.grid_instance(side=3, T=5, L=2, cap=0.6, eps=eps, seed=4)
    p = to_oracle(inst)
    st = alg2.iterate(p, alg2.initial_state(p), 3000)
    out = alg2.projections(p, st)
    lp = lp_check.lp_optimum(inst.cost_csr(), p.T, p.src, p.dst, p.cap)
    walks = lp_check.walk_counts(inst.cost_csr(), p.T, inst.meta["sources"], inst.meta["sinks"])
    bound = eps * sum(m * np.log(w) for m, w in zip(inst.masses(), walks))
    gap = out["cost"] - lp
    assert -1e-6 <= gap <= bound + 1e-6, (gap, bound)
