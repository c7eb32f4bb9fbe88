"""GPU tests of the traces after rho (T_k = sum_j (G S)_jj, U_k = sum_j (G H)_jj,
tr(rho S), tr(rho H)) and the Fermi level computed from them.

Bar: each trace within 1e-10 of the oracle's relative to its largest entry
(the traces sum G entries that each meet the 1e-10 parity bar); on the full
bundle, the identity z_k T_k - U_k = n_cols (row j of the restricted
equations, each column converged to tol) within n_cols * 10 * tol.
"""
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


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("overlap,prune", [(False, True), (False, False), (True, True)])
def test_traces_vs_oracle(sgf, O, overlap, prune):
    wl = W.bundle_workload(3, 2, 40, overlap=overlap, n_shifts=64, config_no=150)
    cols = wl.columns[::3]
    print(f"  {cols.size} columns, overlap {overlap}, prune {prune}", flush=True)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, cols, radius=1.0, prune=prune)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    T, U, (ts, th) = sgf.traces(prep, res)
    b = O.system_for(wl)
    ref = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=prune, threads=8)
    Tr, Ur = O.traces(b, ref, cols)
    tsr, thr = O.rho_traces(b, ref, cols)
    print(f"  T {rel(T, Tr):.2e}  U {rel(U, Ur):.2e}  tr(rho S) {abs(ts - tsr):.2e}  tr(rho H) {abs(th - thr):.2e}")
    assert rel(T, Tr) < 1e-10 and rel(U, Ur) < 1e-10
    assert abs(ts - tsr) <= 1e-10 * max(1.0, abs(tsr)) and abs(th - thr) <= 1e-10 * max(1.0, abs(thr))
    # the library's electron count at the solve's own weights is the rho trace
    ne, eb = sgf.occupation(T, U, wl.w)
    assert abs(ne - ts) <= 1e-11 * max(1.0, abs(ts)) and abs(eb - th) <= 1e-11 * max(1.0, abs(th))
    # repeatable bit for bit
    T2, U2, r2 = sgf.traces(prep, res)
    np.testing.assert_array_equal(T, T2)
    np.testing.assert_array_equal(U, U2)
    assert r2 == (ts, th)


def test_traces_chain_vs_oracle(sgf, O):
    wl = W.config_chain()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=0.0, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol)
    T, U, _ = sgf.traces(prep, res)
    b = O.system_for(wl)
    ref = O.solve_workload(wl, threads=8)
    Tr, Ur = O.traces(b, ref, wl.columns)
    print(f"  chain: T {rel(T, Tr):.2e}  U {rel(U, Ur):.2e}")
    assert rel(T, Tr) < 1e-9 and rel(U, Ur) < 1e-9


def test_trace_identity_and_fermi_level_full_bundle(sgf, O):
    """All 473,200 columns of the bundle: z_k T_k - U_k = n_cols for every
    shift, and the Fermi level of half filling (two electrons per atom and
    spin over the solved columns) from the library equals the oracle's scan
    on the same traces."""
    import torch
    wl = W.config_bundle()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, batch_cols=sgf.batch_limit(prep, wl.z.size, 112 << 30))
    assert int((res.status != 0).sum()) == 0
    T, U, (ts, th) = sgf.traces(prep, res)
    n = wl.columns.size
    gap = np.abs(wl.z * T - U - n).max()
    print(f"  {n} columns: max |z T - U - n| = {gap:.2e} (bound {10 * wl.tol * n:.2e})", flush=True)
    assert gap <= 10 * wl.tol * n
    target = 0.5 * n
    mu, ne, eb = sgf.fermi_level(wl.z, T, U, target)
    rmu, rne, reb = O.fermi_level(wl.z, T, U, target)
    print(f"  half filling: mu {mu:.4f} eV, N_e {ne:.2f}, E_band {eb:.2f} eV")
    assert mu == rmu and abs(ne - rne) <= 1e-9 * n and abs(eb - reb) <= 1e-9 * max(1.0, abs(reb))
    del res
    torch.cuda.empty_cache()


def test_traces_leave_out_columns_that_did_not_converge(sgf, O):
    """A NaN block poisons the columns whose subspace holds it: with the
    status filter they contribute nothing and the traces equal those of the
    clean columns alone."""
    wl = W.bundle_workload(2, 1, 30, n_shifts=32, config_no=151)
    s = sgf.system_for(wl)
    s.h[int(s.row_ptr[1])] = float("nan")
    cols = np.array([0, 4, 100, 150, 180])
    prep = sgf.prepare(s, cols, radius=0.6)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    st = res.status.cpu().numpy()
    assert list(st[:2]) == [sgf.NONFINITE, sgf.NONFINITE] and np.all(st[2:] == sgf.CONVERGED)
    T, U, _ = sgf.traces(prep, res)
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(U))
    prep2 = sgf.prepare(s, cols[2:], radius=0.6)
    res2 = sgf.solve_prepared(prep2, wl.z, wl.w, tol=1e-12)
    T2, U2, _ = sgf.traces(prep2, res2)
    assert rel(T, T2) < 1e-13 and rel(U, U2) < 1e-13
