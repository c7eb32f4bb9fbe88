"""The allocation-free solve (sgf_shifted_solve_static, workspace in the
library's static device scratch) against the workspace entry point
(sgf_shifted_solve) on the same prepared columns: both run the same
kernels, and batching does not change a bit, so G, rho, iterations, status,
residuals and step counts must be bitwise equal.  Two calls in a row, the
second with fewer columns and shifts, so that the scratch holds the first
call's contents when the second starts; the first call is large enough to
take several batches of the scratch."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sgf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_09616_amd as sgf
    sgf.lib()
    return sgf


def _equal(a, b):
    np.testing.assert_array_equal(a.status, b.status)
    np.testing.assert_array_equal(a.iters, b.iters)
    np.testing.assert_array_equal(a.G, b.G)
    np.testing.assert_array_equal(a.rho, b.rho)
    np.testing.assert_array_equal(a.resid, b.resid)
    np.testing.assert_array_equal(a.shift_iters, b.shift_iters)


def test_static_scratch_solve_equals_workspace_solve(sgf):
    import torch
    wl = W.bundle_workload(4, 4, 60, n_shifts=128, config_no=131)
    s = sgf.system_for(wl)
    # first call: every column (3,840), more than one batch of the scratch
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    in_scratch = sgf.batch_limit(prep, wl.z.size, sgf.STATIC_SCRATCH_BYTES)
    assert in_scratch < wl.columns.size
    ref = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, shift_iters=True).numpy()
    got = sgf.shifted_solve_static(prep, wl.z, wl.w, tol=wl.tol, shift_iters=True)
    torch.cuda.synchronize()
    got = got.numpy()
    print(f"  call 1: {wl.columns.size} columns x {wl.z.size} shifts ({in_scratch} columns per batch of "
          f"the scratch; the workspace solve in one batch)", flush=True)
    assert np.all(ref.status == sgf.CONVERGED)
    _equal(got, ref)
    # second call: fewer columns and shifts, other energies, on the scratch the
    # first call left behind
    z2, w2 = wl.z[::2][:50], wl.w[::2][:50]
    cols2 = wl.columns[5:400:3]
    prep2 = sgf.prepare(s, cols2, radius=wl.radius, prune=True)
    ref2 = sgf.solve_prepared(prep2, z2, w2, tol=wl.tol, shift_iters=True).numpy()
    got2 = sgf.shifted_solve_static(prep2, z2, w2, tol=wl.tol, shift_iters=True)
    torch.cuda.synchronize()
    got2 = got2.numpy()
    print(f"  call 2: {cols2.size} columns x {z2.size} shifts", flush=True)
    assert np.all(ref2.status == sgf.CONVERGED)
    _equal(got2, ref2)


def test_static_scratch_limits(sgf):
    """A column whose history cannot fit the scratch is refused with
    SGF_EUNSUPPORTED, and profiling (HIP events) with SGF_EINVAL; nothing is
    launched in either case."""
    wl = W.bundle_workload(1, 1, 20, n_shifts=16, config_no=132)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns[:4], radius=wl.radius, prune=True)
    with pytest.raises(sgf.SgfError) as e:
        sgf.shifted_solve_static(prep, wl.z, wl.w, tol=wl.tol, max_iter=2_000_000)
    assert e.value.code == sgf.SGF_EUNSUPPORTED and "static scratch" in str(e.value)
    import ctypes
    import torch
    opts = sgf.SolveOptsC(0, 1e-10, 0, -1, 0, -1, 0, 1, 0, 0, 0, 0.0, 0.0, 0)
    zh = np.ascontiguousarray(wl.z).view(np.float64)
    rho = torch.zeros(prep.n_rows, dtype=torch.float64, device="cuda")
    iters = torch.zeros(4, dtype=torch.int32, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    rc = sgf.lib().sgf_shifted_solve_static(
        ctypes.byref(s.c()), ctypes.byref(prep.plan.c()), ctypes.byref(prep.plan.totals), 4, prep.cols.data_ptr(),
        prep.col_plan.data_ptr(), None, wl.z.size, zh.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(opts),
        prep.proj_off.data_ptr(), None, rho.data_ptr(), iters.data_ptr(), status.data_ptr(), None, None, None)
    assert rc == sgf.SGF_EINVAL and b"profile" in sgf.lib().sgf_last_error()
