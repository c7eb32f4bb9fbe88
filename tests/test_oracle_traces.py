"""Pins for the oracle's traces, electron count, band energy and Fermi level
(the quantities formed from G and rho after the shifted solves), each
checked against something other than the oracle's own trace code:

* row j of the restricted equations: z_k (G S)_jj - (G H)_jj = 1 for every
  converged column, so z_k T_k - U_k = n_cols up to the residuals;
* closed forms: an isolated atom and the clean chain's eigen-expansion;
* the Fermi-level scan against the weights of the input generator.
"""
import numpy as np
import pytest

import workloads as W


def identity_gap(z, T, U, n_cols):
    return np.abs(z * T - U - n_cols).max()


@pytest.mark.parametrize("overlap,prune", [(False, True), (False, False), (True, True)])
def test_trace_identity(oracle_lib, overlap, prune):
    """z_k T_k - U_k = n_cols: row j of (z S - H) x = e_j, summed over the
    solved columns; each converged column's residual is <= tol (||b|| = 1)."""
    O = oracle_lib
    wl = W.bundle_workload(2, 1, 24, overlap=overlap, n_shifts=16, config_no=93)
    b = O.system_for(wl)
    cols = wl.columns[::3]
    tol = 1e-12
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=tol, radius=0.8, prune=prune, threads=4)
    assert np.all(res.status == O.CONVERGED)
    T, U = O.traces(b, res, cols)
    gap = identity_gap(wl.z, T, U, cols.size)
    print(f"  max |z T - U - n| = {gap:.2e} over {cols.size} columns")
    assert gap <= 10 * tol * cols.size


def test_trace_identity_catches_a_transposed_block(oracle_lib):
    """The identity is sensitive to the orientation of the off-diagonal
    blocks (the s-p entries change sign under transposition)."""
    O = oracle_lib
    wl = W.bundle_workload(2, 1, 24, n_shifts=8, config_no=94)
    b = O.system_for(wl)
    cols = wl.columns[:20]
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, None, tol=1e-12, radius=0.8, prune=True)
    bt = O.BSR(b.row_ptr, b.col, np.ascontiguousarray(np.transpose(b.h, (0, 2, 1))), b.s)
    T, U = O.traces(bt, res, cols)
    assert identity_gap(wl.z, T, U, cols.size) > 1e-3


def test_traces_isolated_atom(oracle_lib):
    """One atom with no bond, its four columns: T_k = 1/(z - E_s) + 3/(z - E_p)
    and U_k = E_s/(z - E_s) + 3 E_p/(z - E_p)."""
    O = oracle_lib
    p = W.BUNDLE_TB
    xyz = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    b = O.tb_build(xyz, p)
    z = W.shift_grid(-10, 10, 9, 0.05)
    res = O.shifted_solve(b, xyz, np.arange(4), z, None, tol=1e-13, radius=1.0)
    T, U = O.traces(b, res, np.arange(4))
    np.testing.assert_allclose(T, 1 / (z - p.e_s) + 3 / (z - p.e_p), rtol=1e-12)
    np.testing.assert_allclose(U, p.e_s / (z - p.e_s) + 3 * p.e_p / (z - p.e_p), rtol=1e-12)


def test_traces_clean_chain(oracle_lib):
    """Uniform chain, whole system: T_k = sum_j sum_m v_m(j)^2 / (z - lambda_m),
    U_k = sum_j sum_m v_m(j)^2 lambda_m / (z - lambda_m)."""
    O = oracle_lib
    N, t = 96, -1.0
    wl = W.chain_workload(N, 7, 20, disorder=0.0, config_no=95)
    b = O.chain_build(np.zeros(N), t)
    res = O.shifted_solve(b, None, wl.columns, wl.z, wl.w, tol=1e-13)
    m = np.arange(1, N + 1)
    lam = 2 * t * np.cos(m * np.pi / (N + 1))
    V = np.sqrt(2 / (N + 1)) * np.sin(np.outer(np.arange(1, N + 1), m) * np.pi / (N + 1))
    wt = (V[wl.columns] ** 2).sum(0)  # sum over the solved columns of v_m(j)^2
    T_ref = (wt[None, :] / (wl.z[:, None] - lam[None, :])).sum(1)
    U_ref = (wt[None, :] * lam[None, :] / (wl.z[:, None] - lam[None, :])).sum(1)
    T, U = O.traces(b, res, wl.columns)
    assert np.abs(T - T_ref).max() / np.abs(T_ref).max() < 1e-10
    assert np.abs(U - U_ref).max() / np.abs(U_ref).max() < 1e-10


def test_rho_traces_match_the_trace_route(oracle_lib):
    """tr(rho S) and tr(rho H) from the projected rho equal the trace route
    with the solve's own weights."""
    O = oracle_lib
    wl = W.bundle_workload(2, 1, 24, overlap=True, n_shifts=16, config_no=96)
    b = O.system_for(wl)
    cols = wl.columns[::4]
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=0.8, prune=True, threads=4)
    T, U = O.traces(b, res, cols)
    ne, eb = O.occupation(T, U, wl.w)
    ts, th = O.rho_traces(b, res, cols)
    assert abs(ts - ne) <= 1e-12 * max(1.0, abs(ne))
    assert abs(th - eb) <= 1e-12 * max(1.0, abs(eb))


def test_fermi_level_scan_brackets_the_target(oracle_lib):
    """The returned mu is a grid energy whose trapezoid occupation (the input
    generator's weights) reaches the target while the grid point below does
    not; n_e and e_band equal the occupation at mu."""
    O = oracle_lib
    g = np.random.default_rng(3)
    z = W.shift_grid(-8.0, 8.0, 41, 0.05)
    T = -(np.abs(g.standard_normal(41)) + 0.1) * 1j + g.standard_normal(41)   # Im T < 0, as for (G S)_jj
    U = g.standard_normal(41) + 1j * g.standard_normal(41)
    top = O.occupation(T, U, W.occupied_weights(z, 9.0))[0]
    for frac in (0.1, 0.37, 0.5, 0.93):
        target = frac * top
        mu, ne, eb = O.fermi_level(z, T, U, target)
        k = int(np.argmin(np.abs(z.real - mu)))
        assert z[k].real == mu
        n_at, e_at = O.occupation(T, U, W.occupied_weights(z, mu))
        assert n_at >= target and abs(n_at - ne) < 1e-12 * top and abs(e_at - eb) < 1e-12 * max(1, abs(eb))
        if k > 0:
            assert O.occupation(T, U, W.occupied_weights(z, z[k - 1].real))[0] < target
    with pytest.raises(ValueError):
        O.fermi_level(z, T, U, 2 * top)
