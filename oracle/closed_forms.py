"""Closed-form answers for special cases of the regularised problem (test infrastructure only).

* Schroedinger bridge (remark in Section 4.2): without capacity constraints
  and without state costs, a single commodity of mass m from a point source s
  to a point sink z has the Markov-bridge marginals
      P_tau[i] = m (K^tau)[s, i] (K^(T-tau))[i, z] / (K^T)[s, z].
  (The tensor is a product of K factors; fixing i at time tau splits the walk
  sum into the walks s -> i of length tau and i -> z of length T-tau.)
* Two routes with a binding capacity: states {s, a, b, z}, T = 2, moves
  s->a (cost ca), s->b (cost cb), a->z, b->z (cost 0).  Without the cap the
  entropic split puts 1/(1 + exp((ca - cb)/eps)) on a; if that exceeds the
  capacity d_a the regularised optimum puts exactly d_a on a (the capacity
  dual is active, so complementary slackness makes the constraint tight).
* Two marginals (T = 1): the regularised optimum is diag(a) K diag(b) for
  some positive a, b; i.e. log M - log K is a sum of a row term and a
  column term on the support, and M has the prescribed row/column sums.
"""
from __future__ import annotations

import numpy as np

__all__ = ["bridge_marginals", "two_route_split", "rank_one_residual"]


def bridge_marginals(K, s, z, T, mass=1.0):
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    P = np.zeros((T + 1, n))
    denom = np.linalg.matrix_power(K, T)[s, z]
    for tau in range(T + 1):
        left = np.linalg.matrix_power(K, tau)[s, :]
        right = np.linalg.matrix_power(K, T - tau)[:, z]
        P[tau] = mass * left * right / denom
    return P


def two_route_split(ca, cb, eps, d_a):
    free = 1.0 / (1.0 + np.exp((ca - cb) / eps))
    pa = min(free, d_a)
    return np.array([pa, 1.0 - pa])


def rank_one_residual(M, K, rows, cols):
    """Least-squares misfit of log M - log K = alpha_i + beta_j on the support.

    Returns the max absolute residual; zero (to rounding) iff M = diag(a) K diag(b).
    """
    sup = (M > 0) & (K > 0)
    r, c = np.nonzero(sup)
    y = np.log(M[r, c]) - np.log(K[r, c])
    n1, n2 = M.shape
    A = np.zeros((len(r), n1 + n2))
    A[np.arange(len(r)), r] = 1.0
    A[np.arange(len(r)), n1 + c] = 1.0
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(np.abs(A @ coef - y).max())
