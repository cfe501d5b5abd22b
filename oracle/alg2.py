"""Algorithm 2 of the paper in plain FP64 (test infrastructure only).

Notation.  The paper indexes marginals t = 1..TT (TT = number of time
marginals) plus the commodity mode 0.  Here time is tau = t - 1 = 0..T with
T = TT - 1 transitions:
  tau = 0      source marginal, scaling U01 = U^(0,1)          (L x n)
  tau = 1..T-1 interior marginals with capacity d_tau, scaling u_tau (n)
  tau = T      sink marginal, scaling U0T = U^(0,TT)            (L x n)
K = exp(-C/eps) (n x n), KL = exp(-C_L/eps) (L x n), charged at interior
times only (eq. cost_multicommodity).  A time-varying network (Section 3.3:
C replaced by one matrix C_tau per transition) is a list of T matrices; the
move from time tau to tau+1 then uses K_tau = exp(-C_tau/eps).

Messages (Theorem 5, eqs. psi_hat and psi):
  psi[tau]    = Psi_{tau+1}:  psi[T-1] = U0T K^T,
                psi[tau-1] = (psi[tau] (.) KL) diag(u_tau) K^T
  psihat[tau] = hatPsi_{tau+1}: psihat[1] = U01 K,
                psihat[tau+1] = (psihat[tau] (.) KL) diag(u_tau) K
Bi-marginal projections (eq. proj_0t) and marginals (Corollary 1):
  P_{0,0} = U01 (.) psi[0],  P_{0,T} = U0T (.) psihat[T],
  P_{0,tau} = psihat[tau] (.) psi[tau] (.) KL diag(u_tau),
  P_tau = u_tau (.) (psihat[tau] (.) psi[tau] (.) KL)^T 1.

Sinkhorn updates (eq. sinkhorn_multicommodity, Proposition 1):
  U01 <- R01 ./ psi[0]; u_tau <- min(d ./ P_tau-without-u_tau, 1);
  U0T <- R0T ./ psihat[T].

Readings where the paper is silent or inconsistent:
  * The u-update of Algorithm 2 writes the column sum with K; Corollary 1
    (and the brute-force tensor) have K_L there.  K_L is used.
  * Initial values are not given: u = 1, U0T = indicator of supp(R0T)
    (U01 is overwritten before it is first read).
  * One iteration = backward sweep, source update, forward sweep with the
    capacity updates, sink update (Algorithm 2's loop body, rotated so the
    initial message computation is the first backward sweep).
  * Zero marginals (Theorem 4): U = 0 where R = 0; a positive R facing a zero
    message is infeasible (error).  min(d/s, 1) is evaluated as 1 when s <= d
    (no division; covers s = 0 and d = +inf).
  * Commodity-dependent capacities (the extension closing Section 3:
    P_{0,tau} <= D_tau, (T-1) x L x n, +inf = none) get one more dual
    scaling w_tau (L x n, in (0, 1]) per interior time, multiplying K_L at
    that time in every message and projection.  In the forward sweep, at
    time tau, w_tau is projected first with the current u_tau,
        w_tau = min(D_tau ./ (hatPsi (.) Psi (.) KL (.) u_tau), 1),
    then u_tau with the new w_tau (both are exact Bregman projections, so
    any fixed order is a valid block-coordinate ascent step).  Where
    D_tau = 0 the scaling is 0 (the state is closed to that commodity;
    where it already carries no mass any value would do, 0 is chosen).
  * Dual objective (Theorem 3, with u = exp(-lambda/eps)):
      g = eps * (<log U01, R01> + <log U0T, R0T> + sum_tau <log u_tau, d_tau>
                 + sum_tau <log w_tau, D_tau>) - eps * <K, U>,
      with 0 log 0 = 0 and d, D = +inf contributing 0.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem", "make_problem", "State", "initial_state", "iterate",
    "backward_sweep", "source_update", "forward_sweep", "sink_update",
    "dual_objective", "projections", "LogState", "initial_log_state",
    "iterate_log", "projections_log", "lse_matmul", "InfeasibleError",
]


class InfeasibleError(RuntimeError):
    """A positive source/sink entry faces a zero message (Theorem 4 support)."""


@dataclasses.dataclass
class Problem:
    C: object                 # scipy.sparse (finite entries = allowed moves) or dense ndarray (+inf = forbidden),
                              # or a list of T of them (C_tau for the move tau -> tau+1)
    eps: float
    T: int
    src: np.ndarray           # R^(0,1), (L, n)
    dst: np.ndarray           # R^(0,TT), (L, n)
    cap: np.ndarray           # (T-1, n), +inf = uncapacitated
    state_cost: Optional[np.ndarray] = None   # C_L, (L, n)
    cap_comm: Optional[np.ndarray] = None     # D, (T-1, L, n), +inf = none; None = no such constraints

    @property
    def L(self):
        return self.src.shape[0]

    @property
    def n(self):
        return self.src.shape[1]


def make_problem(C, eps, T, src, dst, cap, state_cost=None, cap_comm=None) -> Problem:
    src = np.asarray(src, dtype=np.float64)
    n = src.shape[1]
    cap = np.asarray(cap, dtype=np.float64)
    if cap.ndim == 1:
        cap = np.broadcast_to(cap, (max(T - 1, 0), n)).copy()
    def one(c):
        return sp.csr_matrix(c, dtype=np.float64) if sp.issparse(c) else np.asarray(c, dtype=np.float64)
    if isinstance(C, (list, tuple)):
        assert len(C) == T, "a time-varying network needs one cost matrix per transition"
        C = [one(c) for c in C]
    else:
        C = one(C)
    sc = None if state_cost is None else np.asarray(state_cost, dtype=np.float64)
    cc = None
    if cap_comm is not None:
        cc = np.asarray(cap_comm, dtype=np.float64)
        if cc.ndim == 2:
            cc = np.broadcast_to(cc, (max(T - 1, 0),) + cc.shape).copy()
        assert cc.shape == (max(T - 1, 0),) + src.shape
    return Problem(C=C, eps=float(eps), T=int(T), src=src,
                   dst=np.asarray(dst, dtype=np.float64), cap=cap, state_cost=sc, cap_comm=cc)


def _gibbs_one(C, eps):
    if sp.issparse(C):
        K = C.copy()
        with np.errstate(over="ignore"):
            K.data = np.exp(-K.data / eps)
        return K
    with np.errstate(over="ignore"):
        return np.exp(-C / eps)


def gibbs(p: Problem):
    """K = exp(-C/eps) (eq. K_multicommodity); a forbidden move gives K = 0.
    A list of K_tau for a time-varying network."""
    if isinstance(p.C, list):
        return [_gibbs_one(c, p.eps) for c in p.C]
    return _gibbs_one(p.C, p.eps)


def _kat(K, tau):
    """The kernel of the move tau -> tau+1."""
    return K[tau] if isinstance(K, list) else K


def gibbs_state(p: Problem):
    if p.state_cost is None:
        return np.ones((p.L, p.n))
    return np.exp(-p.state_cost / p.eps)


def _right(X, K):
    """X K for a dense panel X (L x n) and K sparse or dense (n x n)."""
    if sp.issparse(K):
        return np.asarray((K.T @ X.T).T)
    return X @ K


def _right_t(X, K):
    """X K^T."""
    if sp.issparse(K):
        return np.asarray((K @ X.T).T)
    return X @ K.T


@dataclasses.dataclass
class State:
    U01: np.ndarray
    U0T: np.ndarray
    u: np.ndarray             # (T-1, n): u[tau-1] is the scaling at interior time tau
    psi: np.ndarray           # (T, L, n): psi[tau] = Psi_{tau+1}
    g: list
    w: Optional[np.ndarray] = None   # (T-1, L, n) commodity-capacity scalings (None: no such constraints)


def initial_state(p: Problem) -> State:
    w = None if p.cap_comm is None else np.ones((max(p.T - 1, 0), p.L, p.n))
    return State(U01=np.zeros((p.L, p.n)), U0T=(p.dst > 0).astype(np.float64),
                 u=np.ones((max(p.T - 1, 0), p.n)), psi=np.zeros((p.T, p.L, p.n)), g=[], w=w)


def _klw(KL, w, tau):
    """K_L at interior time tau, times the commodity-capacity scaling w_tau."""
    return KL if w is None else KL * w[tau - 1]


def backward_sweep(p: Problem, st: State, K=None, KL=None) -> None:
    """Theorem 5, eq. psi: Psi_{TT-1} = U0T K^T, then (Psi_t (.) KL) diag(u_t) K^T."""
    K = gibbs(p) if K is None else K
    KL = gibbs_state(p) if KL is None else KL
    st.psi[p.T - 1] = _right_t(st.U0T, _kat(K, p.T - 1))
    for tau in range(p.T - 1, 0, -1):
        st.psi[tau - 1] = _right_t(st.psi[tau] * _klw(KL, st.w, tau) * st.u[tau - 1][None, :], _kat(K, tau - 1))


def _divide_support(R, msg, what):
    bad = (R > 0) & (msg <= 0)
    if np.any(bad):
        raise InfeasibleError(f"{what}: positive marginal on a state with zero message")
    out = np.zeros_like(R)
    m = R > 0
    out[m] = R[m] / msg[m]
    return out


def source_update(p: Problem, st: State) -> None:
    """Algorithm 2: U01 <- R01 ./ Psi_1 (zero off the support of R01, Theorem 4)."""
    st.U01 = _divide_support(p.src, st.psi[0], "source")


def forward_sweep(p: Problem, st: State, K=None, KL=None, update: bool = True,
                  keep: bool = False):
    """Theorem 5 eq. psi_hat with the capacity updates of Algorithm 2.

    At each interior time tau the column sum s = (hatPsi (.) Psi (.) KL)^T 1
    gives u_tau = min(d_tau ./ s, 1) (Corollary 1, eq. sinkhorn_multicommodity);
    then hatPsi <- (hatPsi (.) KL) diag(u_tau) K.  Returns hatPsi at time T
    (and the list of all hatPsi when keep=True).
    """
    K = gibbs(p) if K is None else K
    KL = gibbs_state(p) if KL is None else KL
    ph = _right(st.U01, _kat(K, 0))
    kept = [None, ph] if keep else None
    for tau in range(1, p.T):
        if update:
            q = ph * st.psi[tau] * KL                  # P_{0,tau} without u_tau and w_tau
            if st.w is not None:
                st.w[tau - 1] = _comm_update(q * st.u[tau - 1][None, :], p.cap_comm[tau - 1])
                q = q * st.w[tau - 1]
            s = q.sum(axis=0)
            d = p.cap[tau - 1]
            u = np.ones(p.n)
            over = s > d
            u[over] = d[over] / s[over]
            st.u[tau - 1] = u
        ph = _right(ph * _klw(KL, st.w, tau) * st.u[tau - 1][None, :], _kat(K, tau))
        if keep:
            kept.append(ph)
    return (ph, kept) if keep else ph


def _comm_update(q, D):
    """w = min(D ./ q, 1), evaluated as 1 where q <= D and as 0 where D = 0."""
    w = np.ones_like(q)
    over = q > D
    w[over] = D[over] / q[over]
    w[D == 0] = 0.0
    return w


def sink_update(p: Problem, st: State, ph) -> None:
    """Algorithm 2: U0T <- R0T ./ hatPsi_TT."""
    st.U0T = _divide_support(p.dst, ph, "sink")


def _xlogy_masked(x, y):
    out = np.zeros_like(x, dtype=np.float64)
    m = x > 0
    out[m] = x[m] * np.log(y[m])
    return out


def dual_objective(p: Problem, st: State, mass: float) -> float:
    """Dual objective of Theorem 3 at the current scalings (see module doc)."""
    val = _xlogy_masked(p.src, st.U01).sum() + _xlogy_masked(p.dst, st.U0T).sum()
    fin = np.isfinite(p.cap)
    if p.T > 1:
        val += (p.cap[fin] * np.log(st.u[fin])).sum()
    if st.w is not None:
        m = np.isfinite(p.cap_comm) & (p.cap_comm > 0)
        val += (p.cap_comm[m] * np.log(st.w[m])).sum()
    return p.eps * val - p.eps * mass


def iterate(p: Problem, st: State, n_iter: int) -> State:
    """n_iter iterations of (backward sweep, source update, forward sweep, sink update).

    After each sink update the tensor mass <K, U> equals sum(R0T); the dual
    objective at that point is appended to st.g.
    """
    K = gibbs(p)
    KL = gibbs_state(p)
    for _ in range(n_iter):
        backward_sweep(p, st, K, KL)
        source_update(p, st)
        ph = forward_sweep(p, st, K, KL, update=True)
        sink_update(p, st, ph)
        st.g.append(dual_objective(p, st, float((st.U0T * ph).sum())))
    return st


def projections(p: Problem, st: State, want_flows: bool = True):
    """Exact projections of K (.) U at the current scalings.

    Runs a fresh backward sweep and an update-free forward sweep (Theorem 5),
    then forms (Corollary 1, eq. proj_0t, eq. proj_discrete_bi):
      P0t  (T+1, L, n)  bi-marginal projections on (commodity, time tau)
      Pt   (T+1, n)     occupancy marginals
      flows list of T (n x n) matrices (sparse for a sparse K, dense for a dense K),
            flows[tau][i, j] = total mass
            moving i -> j between tau and tau+1:
            K_ij * sum_l A_tau[l, i] B_{tau+1}[l, j], with A_0 = U01,
            A_tau = hatPsi_tau (.) KL (.) u_tau, B_T = U0T,
            B_tau = Psi_tau (.) KL (.) u_tau (KL times w_tau with
            commodity capacities).
      cost  transport cost <C, M> = sum_tau <C, flows[tau]> + sum_interior <C_L, P0t>
      mass  (T+1, L) per-commodity mass at every time (all equal)
    """
    K = gibbs(p)
    KL = gibbs_state(p)
    tmp = State(U01=st.U01.copy(), U0T=st.U0T.copy(), u=st.u.copy(), psi=np.zeros_like(st.psi), g=[],
                w=None if st.w is None else st.w.copy())
    backward_sweep(p, tmp, K, KL)
    ph_T, hats = forward_sweep(p, tmp, K, KL, update=False, keep=True)
    T, L, n = p.T, p.L, p.n
    P0t = np.zeros((T + 1, L, n))
    P0t[0] = tmp.U01 * tmp.psi[0]
    for tau in range(1, T):
        P0t[tau] = hats[tau] * tmp.psi[tau] * _klw(KL, tmp.w, tau) * tmp.u[tau - 1][None, :]
    P0t[T] = tmp.U0T * ph_T
    if not want_flows:
        return dict(P0t=P0t, Pt=P0t.sum(axis=1), mass=P0t.sum(axis=2), psi=tmp.psi, psihat=hats)
    A = [tmp.U01] + [hats[tau] * _klw(KL, tmp.w, tau) * tmp.u[tau - 1][None, :] for tau in range(1, T)]
    B = [None] + [tmp.psi[tau] * _klw(KL, tmp.w, tau) * tmp.u[tau - 1][None, :] for tau in range(1, T)] + [tmp.U0T]
    flows = []
    for tau in range(T):
        Kt = _kat(K, tau)
        if sp.issparse(Kt):
            Kc = Kt.tocoo()
            vals = Kc.data * np.einsum("li,li->i", A[tau][:, Kc.row], B[tau + 1][:, Kc.col])
            flows.append(sp.csr_matrix((vals, (Kc.row, Kc.col)), shape=(n, n)))
        else:
            # dense K: the same entries, K_ij sum_l A[l, i] B[l, j], as one matrix product
            flows.append(Kt * (A[tau].T @ B[tau + 1]))
    cost = 0.0
    for tau in range(T):
        Ct = _kat(p.C, tau)
        if sp.issparse(flows[tau]):
            F = flows[tau].tocoo()
            cvals = np.asarray(Ct[F.row, F.col]).ravel() if sp.issparse(Ct) else Ct[F.row, F.col]
            fv = F.data
        else:
            cvals, fv = Ct.ravel(), flows[tau].ravel()
        m = fv > 0                           # a closed move (+inf cost) carries no mass
        cost += float((cvals[m] * fv[m]).sum())
    if p.state_cost is not None:
        for tau in range(1, T):
            cost += float((p.state_cost * P0t[tau]).sum())
    return dict(P0t=P0t, Pt=P0t.sum(axis=1), flows=flows, cost=cost,
                mass=P0t.sum(axis=2), psi=tmp.psi, psihat=hats)


# ----------------------------------------------------------------------------
# log domain
# ----------------------------------------------------------------------------

def _log_kernel_csc_one(C, eps, transpose: bool):
    if sp.issparse(C):
        Cm = C.tocsr()
    else:
        fin = np.isfinite(C)
        r, c = np.nonzero(fin)
        Cm = sp.csr_matrix((C[r, c], (r, c)), shape=C.shape)
    M = Cm.T.tocsr() if not transpose else Cm.tocsr()
    M.sort_indices()
    return M.indptr, M.indices, -M.data / eps


def _log_kernel_csc(p: Problem, transpose: bool):
    """log K as (indptr, row-of-entry, value) grouped by output column.

    For out = LSE-product X K (transpose=False), out[:, j] gathers column j
    of K; for X K^T it gathers row j of K.  A list of them (one per
    transition) for a time-varying network.
    """
    if isinstance(p.C, list):
        return [_log_kernel_csc_one(c, p.eps, transpose) for c in p.C]
    return _log_kernel_csc_one(p.C, p.eps, transpose)


def lse_matmul(logX, kern, chunk=128):
    """out[l, j] = log sum_i exp(logX[l, i] + logK_(i -> j)) over the listed entries."""
    indptr, src_idx, logk = kern
    L, n = logX.shape
    out = np.full((L, n), -np.inf)
    nonempty = np.nonzero(np.diff(indptr) > 0)[0]
    starts = indptr[nonempty]
    seg = np.repeat(np.arange(len(nonempty)), np.diff(indptr)[nonempty])
    for l0 in range(0, L, chunk):
        Z = logX[l0:l0 + chunk][:, src_idx] + logk[None, :]
        m = np.maximum.reduceat(Z, starts, axis=1)
        safe_m = np.where(np.isfinite(m), m, 0.0)
        with np.errstate(invalid="ignore"):
            e = np.exp(Z - safe_m[:, seg])
        s = np.add.reduceat(e, starts, axis=1)
        with np.errstate(divide="ignore"):
            res = safe_m + np.log(s)
        res[~np.isfinite(m)] = -np.inf
        out[l0:l0 + chunk, nonempty] = res
    return out


def _lse_rows(Z):
    """log sum over axis 0 with -inf handling."""
    m = Z.max(axis=0)
    safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        r = safe + np.log(np.exp(Z - safe[None, :]).sum(axis=0))
    r[~np.isfinite(m)] = -np.inf
    return r


@dataclasses.dataclass
class LogState:
    lU01: np.ndarray
    lU0T: np.ndarray
    lu: np.ndarray
    lpsi: np.ndarray
    g: list
    lw: Optional[np.ndarray] = None


def initial_log_state(p: Problem) -> LogState:
    lw = None if p.cap_comm is None else np.zeros((max(p.T - 1, 0), p.L, p.n))
    return LogState(lU01=np.full((p.L, p.n), -np.inf),
                    lU0T=np.where(p.dst > 0, 0.0, -np.inf),
                    lu=np.zeros((max(p.T - 1, 0), p.n)),
                    lpsi=np.full((p.T, p.L, p.n), -np.inf), g=[], lw=lw)


def _lklw(lKL, lw, tau):
    return lKL if lw is None else lKL + lw[tau - 1]


def _log_divide_support(R, lmsg, what):
    bad = (R > 0) & ~np.isfinite(lmsg)
    if np.any(bad):
        raise InfeasibleError(f"{what}: positive marginal on a state with zero message")
    out = np.full_like(R, -np.inf)
    m = R > 0
    out[m] = np.log(R[m]) - lmsg[m]
    return out


def _log_cap(p):
    with np.errstate(divide="ignore"):
        return np.log(p.cap)


def iterate_log(p: Problem, st: LogState, n_iter: int) -> LogState:
    """Algorithm 2 with every quantity kept as its natural logarithm.

    Products X K become log-sum-exp over the allowed moves; the capacity
    update is log u = min(log d - log s, 0).  Same schedule and readings as
    iterate(); this form does not underflow when route costs / eps are large.
    """
    kf = _log_kernel_csc(p, transpose=False)
    kb = _log_kernel_csc(p, transpose=True)
    lKL = np.zeros((p.L, p.n)) if p.state_cost is None else -p.state_cost / p.eps
    lcap = _log_cap(p)
    with np.errstate(divide="ignore"):
        lD = None if p.cap_comm is None else np.log(p.cap_comm)
    for _ in range(n_iter):
        st.lpsi[p.T - 1] = lse_matmul(st.lU0T, _kat(kb, p.T - 1))
        for tau in range(p.T - 1, 0, -1):
            st.lpsi[tau - 1] = lse_matmul(st.lpsi[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :],
                                          _kat(kb, tau - 1))
        st.lU01 = _log_divide_support(p.src, st.lpsi[0], "source")
        lph = lse_matmul(st.lU01, _kat(kf, 0))
        for tau in range(1, p.T):
            lq = lph + st.lpsi[tau] + lKL
            if st.lw is not None:
                with np.errstate(invalid="ignore"):
                    lw = np.minimum(lD[tau - 1] - (lq + st.lu[tau - 1][None, :]), 0.0)
                lw[~np.isfinite(lq)] = 0.0
                lw[p.cap_comm[tau - 1] == 0] = -np.inf
                st.lw[tau - 1] = lw
                lq = lq + lw
            ls = _lse_rows(lq)
            st.lu[tau - 1] = np.minimum(lcap[tau - 1] - ls, 0.0)
            lph = lse_matmul(lph + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :], _kat(kf, tau))
        st.lU0T = _log_divide_support(p.dst, lph, "sink")
        mass = float(np.exp(_lse_rows((st.lU0T + lph).reshape(-1, 1))[0]))
        st.g.append(_dual_log(p, st, mass))
    return st


def _dual_log(p, st, mass):
    val = 0.0
    m = p.src > 0
    val += (p.src[m] * st.lU01[m]).sum()
    m = p.dst > 0
    val += (p.dst[m] * st.lU0T[m]).sum()
    if p.T > 1:
        fin = np.isfinite(p.cap)
        val += (p.cap[fin] * st.lu[fin]).sum()
    if st.lw is not None:
        m = np.isfinite(p.cap_comm) & (p.cap_comm > 0)
        val += (p.cap_comm[m] * st.lw[m]).sum()
    return p.eps * val - p.eps * mass


def projections_log(p: Problem, st: LogState, want_flows: bool = True):
    """projections() for a log-domain state (values returned in linear scale)."""
    kf = _log_kernel_csc(p, transpose=False)
    kb = _log_kernel_csc(p, transpose=True)
    lKL = np.zeros((p.L, p.n)) if p.state_cost is None else -p.state_cost / p.eps
    T, L, n = p.T, p.L, p.n
    lpsi = np.full((T, L, n), -np.inf)
    lpsi[T - 1] = lse_matmul(st.lU0T, _kat(kb, T - 1))
    for tau in range(T - 1, 0, -1):
        lpsi[tau - 1] = lse_matmul(lpsi[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :], _kat(kb, tau - 1))
    lhats = [None, lse_matmul(st.lU01, _kat(kf, 0))]
    for tau in range(1, T):
        lhats.append(lse_matmul(lhats[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :], _kat(kf, tau)))
    P0t = np.zeros((T + 1, L, n))
    P0t[0] = np.exp(st.lU01 + lpsi[0])
    for tau in range(1, T):
        P0t[tau] = np.exp(lhats[tau] + lpsi[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :])
    P0t[T] = np.exp(st.lU0T + lhats[T])
    out = dict(P0t=P0t, Pt=P0t.sum(axis=1), mass=P0t.sum(axis=2), lpsi=lpsi, lpsihat=lhats)
    if want_flows:
        lA = [st.lU01] + [lhats[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :] for tau in range(1, T)]
        lB = [None] + [lpsi[tau] + _lklw(lKL, st.lw, tau) + st.lu[tau - 1][None, :] for tau in range(1, T)] + [st.lU0T]
        flows = []
        cost = 0.0
        for tau in range(T):
            Ct = _kat(p.C, tau)
            Cm = Ct.tocoo() if sp.issparse(Ct) else sp.coo_matrix(np.where(np.isfinite(Ct), 1.0, 0.0))
            rows, cols = Cm.row, Cm.col
            cvals = Cm.data if sp.issparse(Ct) else Ct[rows, cols]
            lk = -cvals / p.eps
            Z = lA[tau][:, rows] + lB[tau + 1][:, cols] + lk[None, :]
            vals = np.exp(_lse_rows(Z))
            flows.append(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)))
            m = vals > 0                     # a closed move (+inf cost) carries no mass
            cost += float((cvals[m] * vals[m]).sum())
        if p.state_cost is not None:
            for tau in range(1, T):
                cost += float((p.state_cost * P0t[tau]).sum())
        out["flows"] = flows
        out["cost"] = cost
    return out
