"""Explicit-tensor computations for tiny instances (test infrastructure only).

The multi-commodity tensor has one commodity mode and T+1 state modes
(times 0..T).  Its entries are (eqs. K_multicommodity and U_multicommodity)

  (K (.) U)[l, i_0, ..., i_T] = U01[l, i_0] * prod_{tau=0}^{T-1} K_tau[i_tau, i_tau+1]
                                * prod_{tau=1}^{T-1} KL[l, i_tau] u_tau[i_tau] w_tau[l, i_tau]
                                * U0T[l, i_T]

(K_tau = K for a fixed network, one kernel per move for a time-varying one;
w_tau = 1 unless commodity-dependent capacities are present.)
Projections are plain sums over the other modes (eqs. proj_discrete and
proj_discrete_bi).  The generic Sinkhorn updates of Proposition 1 are applied
to the explicit tensor, in the block order of Algorithm 2.  Everything here
costs L * n^(T+1) and is meant for n^(T+1) up to ~1e5.
"""
from __future__ import annotations

import numpy as np

__all__ = ["full_tensor", "tensor_projections", "tensor_sinkhorn"]


def full_tensor(K, KL, U01, U0T, u, T, w=None):
    """Dense K (.) U of shape (L, n, ..., n) (T+1 state axes); w (T-1, L, n) or None."""
    L, n = U01.shape
    M = U01.reshape((L, n) + (1,) * T).astype(np.float64).copy()
    for tau in range(1, T + 1):
        # factor K[i_{tau-1}, i_tau] spans state axes tau-1 and tau (array axes tau, tau+1);
        # a list holds one kernel per move (time-varying network)
        shapeK = [1] * (T + 2)
        shapeK[tau] = n
        shapeK[tau + 1] = n
        Kt = K[tau - 1] if isinstance(K, (list, tuple)) else K
        M = M * Kt.reshape(shapeK)
        if tau < T:
            shapeS = [1] * (T + 2)
            shapeS[0] = L
            shapeS[tau + 1] = n
            f = KL * u[tau - 1][None, :]
            if w is not None:
                f = f * w[tau - 1]
            M = M * f.reshape(shapeS)
    shapeE = [1] * (T + 2)
    shapeE[0] = L
    shapeE[T + 1] = n
    return M * U0T.reshape(shapeE)


def tensor_projections(M, T):
    """P0t (T+1, L, n), occupancy Pt (T+1, n) and pair projections summed over commodities.

    pairs[tau] (n x n) = sum over l and all other states of M with state i at
    tau and state j at tau+1 (eq. proj_discrete_bi).
    """
    L = M.shape[0]
    n = M.shape[1]
    axes_all = tuple(range(1, T + 2))
    P0t = np.zeros((T + 1, L, n))
    for tau in range(T + 1):
        P0t[tau] = M.sum(axis=tuple(a for a in axes_all if a != tau + 1))
    pairs = []
    for tau in range(T):
        keep = (tau + 1, tau + 2)
        pairs.append(M.sum(axis=(0,) + tuple(a for a in axes_all if a not in keep)))
    return P0t, P0t.sum(axis=1), pairs


def tensor_sinkhorn(K, KL, src, dst, cap, T, n_iter, cap_comm=None):
    """Proposition 1 updates on the explicit tensor, Algorithm 2 block order.

    U01 <- U01 (.) R01 ./ P_{0,1}; for tau = 1..T-1: u_tau <- min(u_tau (.) d ./ P_tau, 1);
    U0T <- U0T (.) R0T ./ P_{0,T}.  With commodity capacities D (T-1, L, n)
    the update w_tau <- min(w_tau (.) D_tau ./ P_{0,tau}, 1) (0 where D = 0)
    comes right before u_tau's.  Each projection is recomputed from the full
    tensor right before its update.  Start: U01 = 1 on supp(R01), u = 1, w = 1,
    U0T = 1 on supp(R0T).  Returns the scalings after n_iter rounds (and w).
    """
    L, n = src.shape
    U01 = (src > 0).astype(np.float64)
    U0T = (dst > 0).astype(np.float64)
    u = np.ones((max(T - 1, 0), n))
    w = None if cap_comm is None else np.ones((max(T - 1, 0), L, n))

    def proj(tau):
        M = full_tensor(K, KL, U01, U0T, u, T, w)
        return M.sum(axis=tuple(a for a in range(1, T + 2) if a != tau + 1))

    for _ in range(n_iter):
        P = proj(0)
        m = src > 0
        U01 = np.where(m, U01 * src / np.where(m, P, 1.0), 0.0)
        for tau in range(1, T):
            if w is not None:
                P0 = proj(tau)
                D = cap_comm[tau - 1]
                ratio = np.where(P0 > 0, w[tau - 1] * D / np.where(P0 > 0, P0, 1.0), np.inf)
                w[tau - 1] = np.where(D == 0, 0.0, np.minimum(ratio, 1.0))
            Pt = proj(tau).sum(axis=0)
            ratio = np.where(Pt > 0, u[tau - 1] * cap[tau - 1] / np.where(Pt > 0, Pt, 1.0), np.inf)
            u[tau - 1] = np.minimum(ratio, 1.0)
        P = proj(T)
        m = dst > 0
        U0T = np.where(m, U0T * dst / np.where(m, P, 1.0), 0.0)
    if w is not None:
        return U01, U0T, u, w
    return U01, U0T, u
