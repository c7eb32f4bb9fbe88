"""Pins for the band-force oracle (oracle/forces.py):

* the analytic block gradient against central differences of the C
  builder's blocks (a separate implementation of the Slater-Koster rules);
* the force against a central difference of E = sum_j sum_{i in P(j)}
  rho_ij H_ij(R) at fixed rho, with H rebuilt by the C builder at displaced
  positions;
* translation invariance: the forces sum to zero.
"""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def fo(oracle_lib):
    from oracle import forces
    return forces


def test_block_gradient_vs_builder(fo, oracle_lib):
    O = oracle_lib
    tb = W.BUNDLE_TB
    g = np.random.default_rng(5)
    for _ in range(12):
        u = g.normal(size=3)
        d = u / np.linalg.norm(u) * g.uniform(0.1, 0.29)
        grad = fo.sk_grad(d, tb)
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            hp = O.tb_build(np.array([[0.0, 0.0, 0.0], d + e]), tb)
            hm = O.tb_build(np.array([[0.0, 0.0, 0.0], d - e]), tb)
            # block (atom 0 row, atom 1 column) is the second block of row 0
            fd = (hp.h[1] - hm.h[1]) / 2e-6
            assert np.abs(fd - grad[k]).max() <= 1e-6 * np.abs(grad).max() + 1e-9
        assert np.abs(fo.sk_block(d, tb) - O.tb_build(np.array([[0.0, 0.0, 0.0], d]), tb).h[1]).max() < 1e-13


def small_solve(O):
    wl = W.bundle_workload(2, 1, 14, config_no=120)
    b = O.system_for(wl)
    cols = np.arange(wl.n_orb)
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    return wl, b, cols, res


def dense_rho(res, cols, n):
    R = np.zeros((n, n))
    for c, j in enumerate(cols):
        for t in range(res.proj_ptr[c], res.proj_ptr[c + 1]):
            R[res.proj_row[t], j] = res.rho[t]
    return R


def test_force_is_the_fixed_rho_gradient(fo, oracle_lib):
    O = oracle_lib
    wl, b, cols, res = small_solve(O)
    F = fo.band_forces(wl.xyz, wl.tb, res, cols, wl.n_atoms)
    R = dense_rho(res, cols, wl.n_orb)  # R[i, j] = rho_ij of column j (not symmetric)
    step = 1e-6
    for A in (0, 5, 13, 20, 27):
        for k in range(3):
            xp, xm = wl.xyz.copy(), wl.xyz.copy()
            xp[A, k] += step
            xm[A, k] -= step
            ep = np.sum(R * O.tb_build(xp, wl.tb).dense("h"))
            em = np.sum(R * O.tb_build(xm, wl.tb).dense("h"))
            fd = -(ep - em) / (2 * step)
            assert abs(fd - F[A, k]) <= 1e-6 * np.abs(F).max(), (A, k, fd, F[A, k])


def test_forces_sum_to_zero(fo, oracle_lib):
    O = oracle_lib
    wl, b, cols, res = small_solve(O)
    F = fo.band_forces(wl.xyz, wl.tb, res, cols, wl.n_atoms)
    assert np.all(np.isfinite(F)) and np.abs(F).max() > 1.0
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()


def test_forces_of_a_column_subset(fo, oracle_lib):
    """The force of a subset of columns is the gradient of that subset's band
    energy: the forces of two complementary subsets add up to the whole."""
    O = oracle_lib
    wl, b, cols, res = small_solve(O)
    F = fo.band_forces(wl.xyz, wl.tb, res, cols, wl.n_atoms)
    sel = np.arange(cols.size) % 3 == 0
    resa = O.shifted_solve(b, wl.xyz, cols[sel], wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    resb = O.shifted_solve(b, wl.xyz, cols[~sel], wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    Fa = fo.band_forces(wl.xyz, wl.tb, resa, cols[sel], wl.n_atoms)
    Fb = fo.band_forces(wl.xyz, wl.tb, resb, cols[~sel], wl.n_atoms)
    assert np.abs(Fa + Fb - F).max() <= 1e-12 * np.abs(F).max()
