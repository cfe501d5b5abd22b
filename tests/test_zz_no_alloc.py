"""mmot_solve_static, the solve that allocates nothing (its workspace is a static
device array of the library), against mmot_create + mmot_solve + mmot_occupancy
with a workspace from the caller: the same kernels, so bitwise the same plan and
statistics, on two calls in a row (the second smaller, reusing the array), and
ENOMEM for a problem whose workspace exceeds the array."""
import ctypes

import numpy as np
import pytest

from paper_2106_14485_amd import _lib, instances

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _static(inst, max_iter):
    from paper_2106_14485_amd.solver import _ptr, default_options, device_problem
    p, keep = device_problem(inst, "cuda")
    o = default_options(precision="fp32", domain="auto", check_every=10, tol=1e-6)
    occ = torch.full((inst.T + 1, inst.n), -1.0, dtype=torch.float64, device="cuda")
    st = _lib.Stats()
    stream = torch.cuda.current_stream()
    status = _lib.lib().mmot_solve_static(ctypes.byref(p), ctypes.byref(o), int(max_iter), _ptr(occ),
                                          ctypes.byref(st), ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    del keep
    return status, st.as_dict(), occ.cpu().numpy()


def _regular(inst, max_iter):
    from paper_2106_14485_amd.solver import Solver
    S = Solver(inst, precision="fp32", domain="auto", check_every=10, tol=1e-6)
    st = S.solve(max_iter)
    occ = S.occupancy().cpu().numpy()
    S.close()
    return st, occ


def test_static_solve_matches_the_regular_entry_points():
    big = instances.rgg_instance(n=1500, L=96, T=30, seed=31, cap_lo=1.0, cap_hi=2.0)     # scaled domain
    small = instances.road_grid_instance(side=12, L=20, T=24, eps=0.05, seed=32)          # log domain
    for inst, max_iter in ((big, 60), (small, 40)):
        status, st, occ = _static(inst, max_iter)
        assert status == _lib.MMOT_OK
        ref_st, ref_occ = _regular(inst, max_iter)
        assert np.array_equal(occ, ref_occ)
        for k in ("iters", "converged", "domain", "dual_obj", "src_resid", "cap_viol", "mass_drift"):
            assert st[k] == ref_st[k], (k, st[k], ref_st[k])
    assert st["domain"] == 2


def test_static_solve_rejects_a_workspace_beyond_the_array():
    from paper_2106_14485_amd.serve import _problem_sizes
    from paper_2106_14485_amd.solver import default_options
    inst = instances.rgg_instance(n=2000, L=512, T=120, seed=33)
    p, keep = _problem_sizes(inst)
    o = default_options(precision="fp32", domain="auto")
    nb = ctypes.c_size_t(0)
    assert _lib.lib().mmot_query_workspace(ctypes.byref(p), ctypes.byref(o), ctypes.byref(nb)) == _lib.MMOT_OK
    assert nb.value > 256 << 20
    status, _, _ = _static(inst, 5)
    assert status == _lib.MMOT_ENOMEM
