"""GPU tests of the Fermi-Dirac density matrix from the pole expansion
(sgf_fermi_shifts): parity with the oracle on the same shifts, accuracy
against the plain definition rho = f(H_L) from the dense eigen-decomposition
of each local subspace, independence of the seed, and the comparison with
the real-axis grid.

Bars: parity 1e-10 (both sides run the same FP64 shifted COCG on the same
shifts); against f(H_L) 1e-9 relative to a column's largest entry (the
expansion's own error is below 1e-12 over the local spectra at 48 poles
with S = I (|e - mu| <= 60 eV) and at 64 with the overlap (<= 97 eV); the
rest is the solve's tolerance)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KT, MU, NPOLE = 0.1, 0.0, 48
NPOLE_OVERLAP = 64   # the overlap stretches the local spectra to ~|97| eV, |y| ~ 970


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
    from oracle import contour
    return oracle, contour


def _rho_err(off, rho, ref_rho):
    worst = 0.0
    for c in range(off.size - 1):
        a, b = off[c], off[c + 1]
        worst = max(worst, np.abs(rho[a:b] - ref_rho[a:b]).max() / np.abs(ref_rho[a:b]).max())
    return worst


@pytest.mark.parametrize("overlap", [False, True])
def test_fermi_rho_vs_oracle_and_definition(sgf, O, overlap):
    oracle, C = O
    wl = W.bundle_workload(3, 2, 50, overlap=overlap, config_no=160)
    cols = wl.columns[::5]
    z, w = sgf.fermi_shifts(NPOLE_OVERLAP if overlap else NPOLE, KT, MU)
    got = sgf.shifted_solve(sgf.system_for(wl), cols, z, w, tol=1e-12, radius=1.0, seed_index=-2).numpy()
    b = oracle.system_for(wl)
    ref = oracle.shifted_solve(b, wl.xyz, cols, z, w, tol=1e-12, radius=1.0, prune=True, seed_index=0, threads=8)
    np.testing.assert_array_equal(got.proj_off, ref.proj_ptr)
    np.testing.assert_array_equal(got.proj_row, ref.proj_row)
    assert np.all(got.status == 0) and np.all(ref.status == 0)
    e_par = _rho_err(ref.proj_ptr, got.rho, ref.rho)
    g_par = max(np.abs(got.G[a:bb] - ref.G[a:bb]).max() / np.abs(ref.G[a:bb]).max()
                for a, bb in zip(ref.proj_ptr[:-1], ref.proj_ptr[1:]))
    off, rows, exact = C.fermi_rho_columns(b, wl.xyz, cols, KT, MU, radius=1.0, prune=True)
    np.testing.assert_array_equal(rows, got.proj_row)
    e_def = _rho_err(off, got.rho, exact)
    print(f"  {z.size} shifts, iterations {got.iters.mean():.1f}: vs oracle rho {e_par:.2e} G {g_par:.2e}; "
          f"vs f(H_L) {e_def:.2e}", flush=True)
    assert e_par < 1e-10 and g_par < 1e-10
    assert e_def < 1e-9


def test_seed_choice_changes_results_within_the_tolerance_bound(sgf):
    """Any seed gives the same shifted iterates in exact arithmetic; in FP64
    each frozen shift is within tol/Im z of its exact solve, so two seeds
    differ by at most 2 tol / min Im z per entry of G."""
    wl = W.bundle_workload(2, 2, 40, config_no=161)
    z, w = sgf.fermi_shifts(NPOLE, KT, MU)
    s = sgf.system_for(wl)
    runs = [sgf.shifted_solve(s, wl.columns[::3], z, w, tol=1e-12, radius=1.0, seed_index=k).numpy()
            for k in (-2, 0, 5, 20)]
    np.testing.assert_array_equal(runs[0].G, runs[1].G)   # -2 picks the pole nearest the axis, index 0
    bound = 2e-12 / z.imag.min()
    for r in runs[2:]:
        assert np.all(r.status == 0)
        d = np.abs(r.G - runs[0].G).max()
        print(f"  seed change: max |dG| {d:.2e} (bound {bound:.2e})", flush=True)
        assert d <= bound


def test_fewer_shifts_than_the_real_axis_grid(sgf, O):
    """The real-axis grid (128 shifts at eta = 0.01 eV, trapezoid weights up
    to mu) and the 49 Fermi shifts, both against f(H_L) at kT = 0.1 eV: the
    grid is far from converged (the spacing is 47 eta), the poles meet 1e-9,
    and the poles' distance from the real axis cuts the iteration count."""
    oracle, C = O
    wl = W.bundle_workload(3, 2, 50, config_no=162)
    cols = wl.columns[::7]
    s = sgf.system_for(wl)
    z, w = sgf.fermi_shifts(NPOLE, KT, MU)
    pole = sgf.shifted_solve(s, cols, z, w, tol=1e-12, radius=1.0, seed_index=-2).numpy()
    grid = sgf.shifted_solve(s, cols, wl.z, W.occupied_weights(wl.z, MU), tol=1e-12, radius=1.0).numpy()
    off, _, exact = C.fermi_rho_columns(oracle.system_for(wl), wl.xyz, cols, KT, MU, radius=1.0, prune=True)
    e_pole, e_grid = _rho_err(off, pole.rho, exact), _rho_err(off, grid.rho, exact)
    print(f"  poles: {z.size} shifts, {pole.iters.mean():.1f} iterations, error {e_pole:.2e}; real axis: "
          f"{wl.z.size} shifts, {grid.iters.mean():.1f} iterations, error {e_grid:.2e}", flush=True)
    assert e_pole < 1e-9 and e_grid > 1e-3
    assert pole.iters.mean() < grid.iters.mean()
