"""GPU tests of the boundary calls around the solve: the block count of a
Hamiltonian before it is built, a system around a caller's matrix, the
diagonal-only Green's-function output, the learned schedule option of the
binding, and the status of mixed-precision columns as the traces and forces
see it."""
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


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.mark.parametrize("overlap", [False, True])
def test_hamiltonian_size_matches_build_and_oracle(sgf, O, overlap):
    wl = W.bundle_workload(5, 4, 90, overlap=overlap, config_no=140)
    n = sgf.hamiltonian_size(wl.xyz, wl.tb)
    s = sgf.system_for(wl)
    assert n == s.nnzb == O.tb_build(wl.xyz, wl.tb).nnzb


def test_system_from_bsr_solves_like_the_built_system(sgf):
    wl = W.bundle_workload(2, 2, 40, n_shifts=64, config_no=141)
    built = sgf.system_for(wl)
    wrapped = sgf.system_from_bsr(built.row_ptr, built.col, built.h, xyz=built.xyz)
    a = sgf.shifted_solve(built, wl.columns[::5], wl.z, wl.w, tol=wl.tol, radius=wl.radius).numpy()
    b = sgf.shifted_solve(wrapped, wl.columns[::5], wl.z, wl.w, tol=wl.tol, radius=wl.radius).numpy()
    np.testing.assert_array_equal(a.G, b.G)
    np.testing.assert_array_equal(a.rho, b.rho)


def _diag_rows(res, cols):
    out = []
    for c, j in enumerate(cols):
        a, b = res.proj_off[c], res.proj_off[c + 1]
        out.append(a + int(np.nonzero(res.proj_row[a:b] == j)[0][0]))
    return np.array(out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_diagonal_only_output(sgf, O, precision):
    """g_out='diag' writes G_jj(z_k) of every column, the same bits as the
    diagonal rows of the full projected output, with the same rho; the FP64
    values match the oracle's diagonal within the FP64 bar."""
    wl = W.bundle_workload(3, 2, 50, n_shifts=128, config_no=142)
    cols = wl.columns[::2]
    tol = wl.tol if precision == "fp64" else 1e-5
    full = sgf.solve_workload(wl, cols=cols, precision=precision, tol=tol).numpy()
    diag = sgf.solve_workload(wl, cols=cols, precision=precision, tol=tol, g_out="diag").numpy()
    assert diag.G is None and diag.G_diag.shape == (cols.size, wl.z.size)
    np.testing.assert_array_equal(diag.G_diag, full.G[_diag_rows(full, cols)])
    np.testing.assert_array_equal(diag.rho, full.rho)
    np.testing.assert_array_equal(diag.status, full.status)
    if precision == "fp64":
        ref = O.solve_workload(wl, cols=cols, threads=8)
        gj = ref.g_diag(cols)
        err = (np.abs(diag.G_diag - gj).max(axis=1) / np.abs(gj).max(axis=1)).max()
        print(f"  G_jj vs oracle: {err:.2e}", flush=True)
        assert err < 1e-10


def test_learned_schedule_option_keeps_results(sgf):
    """schedule='learned' queues the columns by the network's prediction
    (features, forward pass and counting sort on the device); the results are
    bitwise those of the natural order."""
    import torch
    wl = W.bundle_workload(3, 3, 50, n_shifts=64, config_no=143)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius)
    model = sgf.IterationModel(W.mlp_init(7))
    nat = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol)
    feat = sgf.features(prep)
    model.fit(feat, torch.log(nat.iters.to(torch.float32)), epochs=2, seed=3)
    order = sgf.learned_order(prep, model).cpu().numpy()
    assert sorted(order.tolist()) == list(range(wl.columns.size))
    a = sgf.shifted_solve(s, wl.columns, wl.z, wl.w, tol=wl.tol, radius=wl.radius).numpy()
    b = sgf.shifted_solve(s, wl.columns, wl.z, wl.w, tol=wl.tol, radius=wl.radius, schedule="learned",
                          model=model).numpy()
    np.testing.assert_array_equal(a.G, b.G)
    np.testing.assert_array_equal(a.rho, b.rho)
    np.testing.assert_array_equal(a.iters, b.iters)


def test_mixed_columns_are_left_out_of_traces_and_forces(sgf):
    """An accepted mixed-precision column ends with SGF_DIAG_ONLY: its
    off-diagonal rows are not certified, so the status-filtered traces and
    forces count it no more than a rejected one; after the FP64 re-solve of
    those columns they count again."""
    wl = W.bundle_workload(2, 1, 24, n_shifts=64, config_no=144)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius)
    raw = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-5, precision="mixed", fallback=False)
    st = raw.status.cpu().numpy()
    assert np.any(st == sgf.DIAG_ONLY) and not np.any(st == sgf.CONVERGED)
    F = sgf.band_forces(prep, raw, wl.tb).cpu().numpy()
    T, U, (ts, th) = sgf.traces(prep, raw)
    assert np.all(F == 0.0) and np.all(T == 0) and np.all(U == 0) and ts == 0.0 and th == 0.0
    fp64 = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    F64 = sgf.band_forces(prep, fp64, wl.tb).cpu().numpy()
    assert np.abs(F64).max() > 0
