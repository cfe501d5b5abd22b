"""Serving pool: continuous batching of uneven solves; each result equals the plain solve."""
import numpy as np
import pytest

from paper_2106_14485_amd import instances

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _mix():
    return [
        instances.rgg_instance(n=400, L=24, T=12, seed=11, cap_lo=1.0, cap_hi=2.0),
        instances.road_grid_instance(side=14, L=9, T=30, eps=0.1, seed=12),
        instances.rgg_instance(n=900, L=70, T=20, seed=13, cap_lo=1.0, cap_hi=2.0),
        instances.road_grid_instance(side=20, L=3, T=45, eps=0.05, seed=14),
        instances.rgg_instance(n=250, L=1, T=10, seed=15),
        # steps of 300 blocks: runs in a dedicated lane next to the batched ones
        instances.rgg_instance(n=1200, L=256, T=14, seed=16, cap_lo=1.0, cap_hi=2.0),
    ]


def _plain(inst, max_iter):
    from paper_2106_14485_amd.solver import Solver
    # (the pool's options: two forward panels, checks by an update-free forward pass)
    S = Solver(inst, precision="fp32", domain="auto", check_every=10, tol=1e-6, keep_forward=0)
    st = S.solve(max_iter)
    occ = S.occupancy().cpu().numpy()
    S.close()
    return st, occ


def _pooled(insts, max_iter, budget=1 << 36):
    from paper_2106_14485_amd.serve import Pool
    pool = Pool(budget, check_every=10, tol=1e-6)
    tickets = [pool.submit(x, max_iter=max_iter) for x in insts]
    assert all(t is not None for t in tickets)
    while pool.run(64) > 0:
        pass
    out = []
    for t in tickets:
        state, status, st = pool.poll(t)
        assert state == 1 and status == 0
        out.append((st, pool.occupancy(t).cpu().numpy()))
        pool.release(t)
    pool.close()
    return out


def test_each_result_same_alone_in_mix_and_plain():
    insts = _mix()
    mixed = _pooled(insts, 60)
    for k, inst in enumerate(insts):
        alone = _pooled([inst], 60)[0]
        plain = _plain(inst, 60)
        assert np.array_equal(mixed[k][1], alone[1]), f"request {k}: mix differs from alone"
        assert np.array_equal(alone[1], plain[1]), f"request {k}: pool differs from plain solver"
        assert mixed[k][0]["iters"] == plain[0]["iters"]
        assert mixed[k][0]["dual_obj"] == plain[0]["dual_obj"]


def test_budget_admission_and_release():
    from paper_2106_14485_amd.serve import Pool
    m = _mix()
    insts = [m[2], m[0], m[4]]                    # large, medium, small workspace
    probe = Pool(1 << 40)
    sizes = [probe.workspace_bytes(x) for x in insts]
    probe.close()
    pool = Pool(sizes[0] + sizes[1])            # room for the first two only
    t0 = pool.submit(insts[0], max_iter=20)
    t1 = pool.submit(insts[1], max_iter=20)
    assert t0 is not None and t1 is not None
    assert pool.submit(insts[2], max_iter=20) is None        # over budget -> queued by the caller
    while pool.run(64) > 0:
        pass
    pool.release(t0)
    t2 = pool.submit(insts[2], max_iter=20)                   # admitted once budget frees up
    assert t2 is not None
    while pool.run(64) > 0:
        pass
    assert pool.poll(t2)[0] == 1
    pool.close()


def test_serve_loop_latency_report():
    from paper_2106_14485_amd.serve import latency_summary, serve
    insts = _mix()
    arrivals = np.array([0.0, 0.01, 0.02, 0.05, 0.06, 0.03])
    res, total = serve(insts, arrivals, budget_bytes=1 << 36, max_iter=40)
    s = latency_summary(res, total)
    assert s["n"] == len(insts) and s["p99_s"] >= s["p50_s"] > 0
    assert all(r["status"] == 0 for r in res)


def _extensions():
    """Requests using the extensions: a time-varying network, commodity-dependent
    capacities (both on the CSR operators), staggered entry/exit windows and
    per-commodity state costs."""
    import dataclasses
    tv = instances.time_varying_instance(instances.rgg_instance(n=300, L=12, T=10, seed=21, cap_lo=1.0, cap_hi=2.0),
                                         seed=3, closed_frac=0.02)
    base = instances.rgg_instance(n=350, L=20, T=12, seed=22, cap_lo=1.0, cap_hi=2.0)
    rng = np.random.default_rng(5)
    shape = (base.T - 1, base.L, base.n)
    D = np.where(rng.random(shape) < 0.2, 0.3 * base.src.sum(axis=1)[None, :, None], np.inf)
    comm = dataclasses.replace(base, cap_comm=D)
    g = instances.grid_instance(side=5, T=12, L=3, eps=0.1, cap=2.0, seed=4, check_feasible=False)
    stag = instances.staggered_instance(instances.time_varying_instance(g, seed=1, closed_frac=0.0),
                                        np.array([0, 1, 2]), np.array([12, 11, 12]))
    sc = dataclasses.replace(instances.rgg_instance(n=320, L=10, T=10, seed=23, cap_lo=1.0, cap_hi=2.0),
                             state_cost=rng.uniform(0.0, 0.5, (10, 320)))
    return [tv, comm, stag, sc]


def test_extension_requests_same_in_pool_and_plain():
    insts = _extensions() + [_mix()[0]]
    mixed = _pooled(insts, 40)
    for k, inst in enumerate(insts):
        plain = _plain(inst, 40)
        assert np.array_equal(mixed[k][1], plain[1]), f"request {k}: pool differs from plain solver"
        assert mixed[k][0]["iters"] == plain[0]["iters"]
        assert mixed[k][0]["dual_obj"] == plain[0]["dual_obj"]


def test_more_requests_than_tick_slots():
    """80 small requests at once: a tick runs at most 64 requests' items, so the
    others wait for later ticks; every request still runs its whole recorded
    schedule in order, and its result is bitwise the plain solver's."""
    insts = [instances.rgg_instance(n=200 + 10 * (k % 7), L=1 + k % 5, T=6 + k % 4, seed=100 + k,
                                    cap_lo=1.0, cap_hi=2.0) for k in range(80)]
    mixed = _pooled(insts, 30)
    for k in (0, 1, 13, 63, 64, 65, 79):
        plain = _plain(insts[k], 30)
        assert np.array_equal(mixed[k][1], plain[1]), f"request {k}: pool differs from plain solver"
        assert mixed[k][0]["iters"] == plain[0]["iters"]
        assert mixed[k][0]["dual_obj"] == plain[0]["dual_obj"]


def test_workspace_exactly_the_queried_size():
    """The pool carves each request's program area from the caller's workspace:
    the queried size is enough, one byte less is ENOMEM."""
    import ctypes
    from paper_2106_14485_amd import _lib
    from paper_2106_14485_amd.serve import Pool
    from paper_2106_14485_amd.solver import _ptr, device_problem
    inst = _mix()[1]
    pool = Pool(1 << 34)
    nbytes = pool.workspace_bytes(inst)
    p, keep = device_problem(inst, pool.device)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=pool.device)
    t = ctypes.c_uint64(0)
    L = _lib.lib()
    assert L.mmot_pool_submit(pool._h, ctypes.byref(p), ctypes.byref(pool.opts), _ptr(ws), nbytes - 1, 20,
                              ctypes.byref(t)) == _lib.MMOT_ENOMEM
    assert L.mmot_pool_submit(pool._h, ctypes.byref(p), ctypes.byref(pool.opts), _ptr(ws), nbytes, 20,
                              ctypes.byref(t)) == _lib.MMOT_OK
    while pool.run(64) > 0:
        pass
    # (a request asking for kept forward messages is refused before anything is done)
    o1 = _lib.Options.from_buffer_copy(pool.opts)
    o1.keep_forward = 1
    t1 = ctypes.c_uint64(0)
    assert L.mmot_pool_submit(pool._h, ctypes.byref(p), ctypes.byref(o1), _ptr(ws), nbytes, 20,
                              ctypes.byref(t1)) == _lib.MMOT_EUNSUPPORTED
    state, status, st = pool.poll(t.value)
    assert state == 1 and status == 0
    s = L.mmot_pool_solver(pool._h, ctypes.c_uint64(t.value))
    occ_d = torch.empty((inst.T + 1, inst.n), dtype=torch.float64, device=pool.device)
    assert L.mmot_occupancy(ctypes.c_void_p(s), _ptr(occ_d), None) == _lib.MMOT_OK
    occ = occ_d.cpu().numpy()
    pool.release(t.value)
    pool.close()
    plain = _plain(inst, 20)
    assert np.array_equal(occ, plain[1])
    del keep


def test_served_result_matches_the_oracle():
    """A served request against the FP64 oracle directly (not only against the
    plain solver): the same schedule -- chunks of ten iterations, each ended by
    the check pass -- to a fixed iteration count, occupancy and per-commodity
    marginals to 1e-5."""
    from oracle import alg2
    from paper_2106_14485_amd.serve import Pool
    from tests.helpers import rel_l1, to_oracle
    inst = _mix()[0]
    pool = Pool(1 << 34, check_every=10, tol=1e-30)         # runs to max_iter
    t = pool.submit(inst, max_iter=30)
    while pool.run(64) > 0:
        pass
    state, status, st = pool.poll(t)
    assert state == 1 and status == 0 and st["iters"] == 30 and st["domain"] == 1
    occ, pc = pool.occupancy(t, per_commodity=True)
    occ, pc = occ.cpu().numpy(), pc.cpu().numpy()
    pool.release(t)
    pool.close()
    p = to_oracle(inst)
    ost = alg2.iterate(p, alg2.initial_state(p), 30)
    ref = alg2.projections(p, ost, want_flows=False)
    assert rel_l1(occ, ref["Pt"]) <= 1e-5
    assert rel_l1(pc, ref["P0t"]) <= 1e-5
    assert abs(st["dual_obj"] - ost.g[-1]) <= 1e-5 * abs(ost.g[-1])
