"""FP64 CPU oracle for the multi-commodity graph-structured Sinkhorn scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls, links or executes anything in this package; it
is used by the tests, by the smoke check and by the benchmark's CPU-baseline
leg.  It shares no code with the GPU path.

Contents (paper: Haasler, Ringh, Chen, Karlsson, "Scalable computation of
dynamic flow problems via multi-marginal graph-structured optimal
transport"):

  alg2          Algorithm 2 (Section 4.3) in FP64, plain scaling domain and
                log domain, with the projections of Theorem 5 / Corollary 1,
                the bi-marginal (edge-flow) projections of eq. proj_discrete_bi
                and the dual objective of Theorem 3 (eq. omt_multi_graph_dual).
  bruteforce    the full tensor K (.) U of eqs. K_multicommodity /
                U_multicommodity for tiny instances, its projections
                (eqs. proj_discrete, proj_discrete_bi) and the generic Sinkhorn
                updates of Proposition 1 applied to it.
  closed_forms  cases with a closed-form answer: Schroedinger-bridge marginals
                (uncapacitated, point source and sink; remark in Section 4.2),
                the two-route capacity split, the rank-one structure of the
                two-marginal (T = 1) limit.
  lp_check      the unregularised dynamic multi-commodity flow LP in node-edge
                form on the time-expanded network (Section 2.1, Theorem 2) and
                walk counts for the entropy gap bound.

Pins (tests/test_oracle_*.py): every function above is checked against
something other than itself -- brute-force tensors, closed forms, LP optima,
invariants.  Parity with numbers printed in the paper is unpinned: the paper
prints no worked-example values (its result figures are not recoverable).
"""
