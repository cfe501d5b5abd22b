"""The seeded input generators against the recipes they implement (CPU only).

The generators hold no solver arithmetic; these tests pin what every parity
test and the benchmark take as given: the structure of each workload's
network, the marginals' masses and placement, the capacities, the state
labelling, and that a seed fixes an instance.
"""
import math

import numpy as np
import pytest

from paper_2106_14485_amd import instances


def _csr_dict(inst):
    d = {}
    for i in range(inst.n):
        for e in range(inst.rowptr[i], inst.rowptr[i + 1]):
            d[(i, int(inst.colidx[e]))] = float(inst.cost[e])
    return d


def test_road_grid_structure_at_full_size():
    """100 x 100 four-neighbour roads plus waiting: 10^4 states and
    10^4 + 4 * 100 * 99 = 49,600 moves; symmetric U[1, 3] street costs, wait 0.1;
    under the Morton labelling a state's moves go exactly to itself and its grid
    neighbours; rows of at most five entries (the ELL width of the sweep steps)."""
    side = 100
    inst = instances.road_grid_instance(side=side, L=2000, T=120)
    n = side * side
    assert (inst.n, inst.L, inst.T, inst.kind) == (n, 2000, 120, "csr")
    assert inst.nnz == n + 4 * side * (side - 1) == 49_600
    assert np.diff(inst.rowptr).max() == 5 and np.diff(inst.rowptr).min() == 3
    grid_of = inst.meta["grid_of"]
    assert np.array_equal(np.sort(grid_of), np.arange(n))
    lab = np.empty(n, dtype=np.int64)
    lab[grid_of] = np.arange(n)
    moves = _csr_dict(inst)
    for k in range(n):
        g = int(grid_of[k])
        r, c = divmod(g, side)
        want = {k}
        for rr, cc in ((r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)):
            if 0 <= rr < side and 0 <= cc < side:
                want.add(int(lab[rr * side + cc]))
        got = set(inst.colidx[inst.rowptr[k]:inst.rowptr[k + 1]].tolist())
        assert got == want, k
    for (i, j), w in moves.items():
        if i == j:
            assert w == pytest.approx(0.1)
        else:
            assert 1.0 <= w <= 3.0
            assert moves[(j, i)] == w


def test_road_grid_marginals_and_capacities():
    """One origin and one destination per commodity, Manhattan distance <= T,
    lognormal masses equal at both ends; origins and destinations uncapacitated,
    relays at 4 x mean mass, a seeded 5% of them at a tenth of that."""
    side, L, T = 30, 400, 25
    inst = instances.road_grid_instance(side=side, L=L, T=T, seed=3)
    assert np.all((inst.src > 0).sum(axis=1) == 1) and np.all((inst.dst > 0).sum(axis=1) == 1)
    assert np.allclose(inst.src.sum(axis=1), inst.dst.sum(axis=1))
    mass = inst.src.sum(axis=1)
    assert np.all(mass > 0)
    # lognormal(0, 0.5): the log-masses have mean ~0 and spread ~0.5
    assert abs(np.log(mass).mean()) < 0.1 and abs(np.log(mass).std() - 0.5) < 0.08
    grid_of = inst.meta["grid_of"]
    o = grid_of[inst.src.argmax(axis=1)]
    z = grid_of[inst.dst.argmax(axis=1)]
    man = np.abs(o // side - z // side) + np.abs(o % side - z % side)
    assert man.max() <= T
    ends = np.union1d(inst.src.argmax(axis=1), inst.dst.argmax(axis=1))
    assert np.all(np.isinf(inst.cap[ends]))
    relay = np.setdiff1d(np.arange(inst.n), ends)
    base = 4.0 * mass.mean()
    weak = np.isclose(inst.cap[relay], 0.1 * base)
    assert np.all(weak | np.isclose(inst.cap[relay], base))
    assert weak.sum() == int(round(0.05 * len(relay)))
    assert np.array_equal(np.sort(relay[weak]), np.sort(inst.meta["weak"]))


def test_rgg_structure_and_marginals():
    """Symmetrised 7-NN over uniform points with a waiting self-loop per state:
    a symmetric move pattern, Euclidean lengths for moves and 0.01 for waiting,
    rows of at most 16 entries (one ELL batch) averaging about 9.2; each sink
    within T hops of its source; masses U[0.5, 1.5]; capacities
    U[0.2, 1.0] x mean mass."""
    inst = instances.rgg_instance(n=2000, L=256, T=50, seed=0)
    moves = _csr_dict(inst)
    pts = inst.meta["points"]
    for (i, j), w in moves.items():
        assert (j, i) in moves
        if i == j:
            assert w == pytest.approx(0.01)
        else:
            assert w == pytest.approx(float(np.linalg.norm(pts[i] - pts[j])))
    assert all((i, i) in moves for i in range(inst.n))
    deg = np.diff(inst.rowptr)
    assert deg.max() <= 16 and deg.min() >= 8
    assert 8.7 <= deg.mean() <= 9.7
    hd = instances._hop_dist(inst.rowptr, inst.colidx, inst.n, inst.meta["sources"])
    assert np.all(hd[np.arange(inst.L), inst.meta["sinks"]] <= inst.T)
    mass = inst.src.sum(axis=1)
    assert np.allclose(mass, inst.dst.sum(axis=1)) and mass.min() >= 0.5 and mass.max() <= 1.5
    assert inst.cap.min() >= 0.2 * mass.mean() - 1e-12 and inst.cap.max() <= 1.0 * mass.mean() + 1e-12


def test_dense_blobs():
    """Complete graph on uniform points, cost = squared distance truncated at
    0.25 (+inf beyond), zero on the diagonal, symmetric; Gaussian-blob source and
    sink distributions of unit mass; uniform capacity 2 L / n."""
    n, L = 512, 64
    inst = instances.dense_blob_instance(n=n, L=L, T=8, seed=1)
    C = inst.cost_dense
    pts = inst.meta["points"]
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    fin = np.isfinite(C)
    assert np.array_equal(fin, d2 <= 0.25)
    assert np.allclose(C[fin], d2[fin]) and np.all(np.diag(C) == 0.0)
    assert np.array_equal(fin, fin.T)
    assert np.allclose(inst.src.sum(axis=1), 1.0) and np.allclose(inst.dst.sum(axis=1), 1.0)
    assert np.all(inst.src >= 0) and np.all(inst.dst >= 0)
    assert np.allclose(inst.cap, 2.0 * L / n)


@pytest.mark.parametrize("make", [
    lambda s: instances.road_grid_instance(side=12, L=30, T=20, seed=s),
    lambda s: instances.rgg_instance(n=300, L=20, T=15, seed=s),
    lambda s: instances.dense_blob_instance(n=128, L=8, T=4, seed=s),
])
def test_a_seed_fixes_the_instance(make):
    a, b, c = make(5), make(5), make(6)
    for f in ("src", "dst", "cap", "rowptr", "colidx", "cost", "cost_dense"):
        x, y = getattr(a, f), getattr(b, f)
        if x is None:
            assert y is None
            continue
        assert np.array_equal(x, y, equal_nan=True), f
    assert not (np.array_equal(a.src, c.src) and np.array_equal(a.dst, c.dst))


def test_serving_trace():
    """Poisson arrivals at the stated rate; per request n log-uniform in
    [200, 10000], T uniform in {10..120}, L log-uniform in [1, 512], eps from
    {0.02, 0.05, 0.1}, the generator either graph family with probability 1/2."""
    rate = 100.0
    reqs = instances.serve_trace(num=10000, rate=rate, seed=0)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() * rate - 1.0) < 0.03
    assert abs(gaps.std() * rate - 1.0) < 0.05          # exponential: std = mean
    n = np.array([r["n"] for r in reqs])
    T = np.array([r["T"] for r in reqs])
    L = np.array([r["L"] for r in reqs])
    assert n.min() >= 200 and n.max() <= 10000
    assert T.min() == 10 and T.max() == 120
    assert L.min() >= 1 and L.max() <= 512
    # log-uniform: the median of log n sits at the middle of the log range
    assert abs(np.median(np.log(n)) - 0.5 * (math.log(200) + math.log(10000))) < 0.1
    assert {r["eps"] for r in reqs} == {0.02, 0.05, 0.1}
    share = np.mean([r["gen"] == "rgg" for r in reqs])
    assert abs(share - 0.5) < 0.02
    assert instances.serve_trace(num=50, seed=4) == instances.serve_trace(num=50, seed=4)
