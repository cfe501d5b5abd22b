"""Shared test helpers: random tiny instances and Instance -> oracle.Problem conversion."""
import numpy as np
import scipy.sparse as sp

from oracle import alg2
from paper_2106_14485_amd.instances import Instance


def to_oracle(inst: Instance) -> alg2.Problem:
    if inst.kind == "csr":
        C = inst.cost_csr()
    else:   # a time-varying dense network: one cost matrix per move
        C = list(inst.cost_dense) if np.ndim(inst.cost_dense) == 3 else inst.cost_dense
    return alg2.make_problem(C, inst.eps, inst.T, inst.src, inst.dst, inst.cap, inst.state_cost, inst.cap_comm)


def random_tiny(n=4, T=4, L=2, seed=0, density=0.6, state_cost=True, cap_scale=0.6,
                point=False, kind="csr", eps=0.5):
    """A tiny random instance with self-loops (every state can wait)."""
    rng = np.random.default_rng(seed)
    pat = rng.random((n, n)) < density
    np.fill_diagonal(pat, True)
    ring = np.arange(n)
    pat[ring, (ring + 1) % n] = True         # a two-way ring keeps every state reachable
    pat[(ring + 1) % n, ring] = True
    if T < 2:
        pat[:] = True
    C = np.where(pat, rng.uniform(0.0, 1.0, (n, n)), np.inf)
    if point:
        src = np.zeros((L, n)); dst = np.zeros((L, n))
        m = rng.uniform(0.5, 1.5, L)
        src[np.arange(L), rng.integers(0, n, L)] = m
        dst[np.arange(L), rng.integers(0, n, L)] = m
    else:
        src = rng.uniform(0.1, 1.0, (L, n)) * (rng.random((L, n)) < 0.7)
        src[:, 0] += 0.5
        dst = rng.uniform(0.1, 1.0, (L, n)) * (rng.random((L, n)) < 0.7)
        dst[:, -1] += 0.5
        dst *= (src.sum(1) / dst.sum(1))[:, None]
    cap = rng.uniform(cap_scale, 1.5 * cap_scale, (max(T - 1, 0), n)) * src.sum() / n * 2
    sc = rng.uniform(0.0, 0.5, (L, n)) if state_cost else None
    if kind == "csr":
        r, c = np.nonzero(pat)
        Cm = sp.csr_matrix((C[r, c], (r, c)), shape=(n, n))
    else:
        Cm = C
    return alg2.make_problem(Cm, eps, T, src, dst, cap, sc), C


def dense_flow(f):
    """An oracle flow matrix as a dense array (sparse for a sparse K, dense for a dense K)."""
    return f.toarray() if sp.issparse(f) else np.asarray(f)


def rel_l1(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / (den if den > 0 else 1.0))


def fp32_log_floor(proj, T, per_commodity=False):
    """Precision floor of an FP32 log-domain solve, from the oracle's log messages.

    The GPU log domain stores log2-messages relative to per-commodity offsets
    centred on the state where the plan peaks, so an entry whose log-message is
    a distance g (nats) from its value there is held with an absolute rounding
    error up to u g, u = 2^-24, i.e. a relative error u g in the linear value.
    A plan entry carries that error from its backward and its forward message:
    relative error u (g_b + g_f).  The plan-weighted mean of g_b + g_f over the
    interior times gives the first-order relative-L1 error of the marginals;
    the floor is four times it, covering the re-rounding along the T-step
    recursions and the exp2 / log2 instruction errors.  per_commodity=True
    returns the same figure for each commodity's own marginals (length L).
    """
    P, lpsi, lh = proj["P0t"], proj["lpsi"], proj["lpsihat"]
    L = P.shape[1]
    num = np.zeros(L); den = np.zeros(L)
    for t in range(1, T):
        b, f = lpsi[t], lh[t]
        plan = np.where(np.isfinite(b) & np.isfinite(f), b + f, -np.inf)
        peak = plan.argmax(axis=1)
        rows = np.arange(b.shape[0])
        gaps = 0.0
        for m in (b, f):
            ref = m[rows, peak][:, None]
            gaps = gaps + np.where(np.isfinite(m) & np.isfinite(ref), np.abs(m - ref), 0.0)
        num += (P[t] * gaps).sum(axis=1)
        den += P[t].sum(axis=1)
    if per_commodity:
        return 4.0 * 2.0 ** -24 * np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return 4.0 * 2.0 ** -24 * (num.sum() / den.sum() if den.sum() > 0 else 0.0)
