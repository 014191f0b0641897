"""The library's HIP-event profile (rsilu_set_profiling, rsilu_set_profiling_mask) on the
grid recipe at 30000 x 20000 with the correction by Jacobi CG steps through the explicit Y~:
timing changes no result, and a class mask times exactly the launches of its classes.
"""

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def test_profile_mask(gpu_lib):
    R = gpu_lib
    import torch

    prob = gen.by_name("c2-small")
    S = R.Solver.from_problem(prob, p=20, mu=1.0, form=R.FORM_ALG2, smode=R.S_CG, cg_steps=8, ystore=R.Y_EXPLICIT,
                              ytau=5e-2, cg_precond=R.CG_JACOBI, maxit=2000).upload()
    b = torch.from_numpy(prob.b).cuda()
    x0, code, it0, _, _ = S.solve(b, tol=1e-8)
    x0 = x0.cpu().numpy().copy()
    assert code == R.OK
    runs = {}
    for what in ("all", "sweep", "sweep+y"):
        if what == "all":
            assert R.rsilu_set_profiling(S.h, 1) == R.OK
        else:
            names = ["k_trsv_sweep"] + (["k_spmv_y"] if what == "sweep+y" else [])
            assert R.rsilu_set_profiling_mask(S.h, names) == R.OK
        x, code, it, _, _ = S.solve(b, tol=1e-8)
        runs[what] = R.rsilu_get_profile(S.h)
        assert code == R.OK and it == it0
        assert np.array_equal(x.cpu().numpy(), x0), what  # timing changes no result
    assert R.rsilu_set_profiling(S.h, 0) == R.OK
    S.close()
    full = runs["all"]
    assert full["k_trsv_sweep"][0] > 0 and full["k_spmv_y"][0] > 0
    for what, names in (("sweep", {"k_trsv_sweep"}), ("sweep+y", {"k_trsv_sweep", "k_spmv_y"})):
        for name in R.PROF_NAMES:
            launches, ms, nbytes = runs[what][name]
            if name in names:
                # the same launches, bytes, and a time
                assert launches == full[name][0] and nbytes == full[name][2] and ms > 0, (what, name)
            else:
                assert launches == 0 and ms == 0 and nbytes == 0, (what, name)
