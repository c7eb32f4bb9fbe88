"""Pins for the band-force oracle (oracle/forces.py):

* the analytic block gradient against central differences of the C
  builder's blocks (a separate implementation of the Slater-Koster rules);
* the force against a central difference of E = sum_j sum_{i in P(j)}
  rho_ij H_ij(R) at fixed rho, with H rebuilt by the C builder at displaced
  positions;
* translation invariance: the forces sum to zero;
* with an overlap: the overlap-block gradient against the C builder; the
  Hellmann-Feynman theorem of the generalized eigenproblem (the force from
  the exact rho and energy-density matrix of the lowest states equals a
  central difference of the sum of their eigenvalues); the force against a
  central difference of sum rho H - sum eps S at fixed rho and eps;
* the energy-density matrix against its spectral form on a solve whose
  subspace is the whole system, and the column identity sum eps_ij S_ji =
  sum rho_ij H_ji that (z S - H) G = I implies.
"""
import types

import numpy as np
import pytest
import scipy.linalg

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


def test_overlap_gradient_vs_builder(fo, oracle_lib):
    O = oracle_lib
    tb = W.BUNDLE_TB_OVERLAP
    g = np.random.default_rng(6)
    for _ in range(8):
        u = g.normal(size=3)
        d = u / np.linalg.norm(u) * g.uniform(0.1, 0.29)
        grad = fo.overlap_grad(d, tb)
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            sp = O.tb_build(np.array([[0.0, 0.0, 0.0], d + e]), tb).s[1]
            sm = O.tb_build(np.array([[0.0, 0.0, 0.0], d - e]), tb).s[1]
            assert np.abs((sp - sm) / 2e-6 - grad[k]).max() <= 1e-6 * np.abs(grad).max() + 1e-12


def dense_layout(n, R, E):
    """Every column j with every orbital i as a projection row: rho_ij = R[i, j]."""
    res = types.SimpleNamespace(proj_ptr=np.arange(n + 1) * n, proj_row=np.tile(np.arange(n), n),
                                rho=R.T.ravel().copy())
    return res, E.T.ravel().copy()


@pytest.mark.parametrize("overlap", [False, True])
def test_hellmann_feynman_of_the_lowest_states(fo, oracle_lib, overlap):
    """Occupy the lowest n_occ states of H c = lambda S c (a gap of 0.76 eV
    above them): -d/dR sum_{n < n_occ} lambda_n equals the force from
    rho = C_o C_o^T and eps = C_o diag(lambda_o) C_o^T with every orbital
    as a projection row.  Dropping the eps term misses by ~50 eV/nm."""
    O = oracle_lib
    wl = W.bundle_workload(2, 1, 14, overlap=overlap, config_no=120)

    def eig(xyz):
        b = O.tb_build(xyz, wl.tb)
        H = b.dense("h")
        return scipy.linalg.eigh(H, b.dense("s") if overlap else None)

    lam, C = eig(wl.xyz)
    n, n_occ = lam.size, 54
    assert lam[n_occ] - lam[n_occ - 1] > 0.5
    Co = C[:, :n_occ]
    res, eps = dense_layout(n, Co @ Co.T, Co @ np.diag(lam[:n_occ]) @ Co.T)
    F = fo.band_forces(wl.xyz, wl.tb, res, np.arange(n), wl.n_atoms, eps=eps)
    step = 1e-6
    for A in (0, 5, 13, 20, 27):
        for k in range(3):
            xp, xm = wl.xyz.copy(), wl.xyz.copy()
            xp[A, k] += step
            xm[A, k] -= step
            fd = -(eig(xp)[0][:n_occ].sum() - eig(xm)[0][:n_occ].sum()) / (2 * step)
            assert abs(fd - F[A, k]) <= 1e-9 * np.abs(F).max(), (A, k, fd, F[A, k])
    if overlap:
        F0 = fo.band_forces(wl.xyz, wl.tb, res, np.arange(n), wl.n_atoms, eps=np.zeros_like(eps))
        assert np.abs(F0 - F).max() > 1e-2 * np.abs(F).max()


def overlap_solve(O, radius=1.0, prune=True):
    wl = W.bundle_workload(2, 1, 14, overlap=True, config_no=120)
    b = O.system_for(wl)
    cols = np.arange(wl.n_orb)
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=radius, prune=prune, threads=8)
    return wl, b, cols, res


def test_overlap_force_is_the_fixed_rho_eps_gradient(fo, oracle_lib):
    O = oracle_lib
    wl, b, cols, res = overlap_solve(O)
    assert np.all(res.status == 0)
    eps = fo.energy_density(res, wl.z, wl.w)
    F = fo.band_forces(wl.xyz, wl.tb, res, cols, wl.n_atoms, eps=eps)
    R = dense_rho(res, cols, wl.n_orb)
    Ep = dense_rho(types.SimpleNamespace(proj_ptr=res.proj_ptr, proj_row=res.proj_row, rho=eps), cols, wl.n_orb)
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
    step = 1e-6
    for A in (0, 5, 13, 20, 27):
        for k in range(3):
            xp, xm = wl.xyz.copy(), wl.xyz.copy()
            xp[A, k] += step
            xm[A, k] -= step
            bp, bm = O.tb_build(xp, wl.tb), O.tb_build(xm, wl.tb)
            ep = np.sum(R * bp.dense("h")) - np.sum(Ep * bp.dense("s"))
            em = np.sum(R * bm.dense("h")) - np.sum(Ep * bm.dense("s"))
            fd = -(ep - em) / (2 * step)
            assert abs(fd - F[A, k]) <= 1e-6 * np.abs(F).max(), (A, k, fd, F[A, k])
    with pytest.raises(ValueError):
        fo.band_forces(wl.xyz, wl.tb, res, cols, wl.n_atoms)


def test_energy_density_spectral_form(fo, oracle_lib):
    """With the whole system as every column's subspace, G(z) = (z S - H)^-1
    = sum_n c_n c_n^T / (z - lambda_n), so for real weights
    eps = sum_n lambda_n f_n c_n c_n^T and rho = sum_n f_n c_n c_n^T with
    f_n = -(1/pi) sum_k Im(w_k / (z_k - lambda_n)).  (Weighting with Re z_k
    instead of z_k misses by 2e-2 here; the solve is good to 2e-11.)"""
    O = oracle_lib
    wl, b, cols, res = overlap_solve(O, radius=100.0, prune=False)
    assert np.all(res.status == 0) and np.all(np.asarray(wl.w).imag == 0)
    lam, C = scipy.linalg.eigh(b.dense("h"), b.dense("s"))
    f = -(np.asarray(wl.w)[None, :] / (np.asarray(wl.z)[None, :] - lam[:, None])).imag.sum(axis=1) / np.pi
    Rs = C @ np.diag(f) @ C.T
    Es = C @ np.diag(lam * f) @ C.T
    eps = fo.energy_density(res, wl.z, wl.w)
    for c, j in enumerate(cols):
        a, e = res.proj_ptr[c], res.proj_ptr[c + 1]
        rows = res.proj_row[a:e]
        assert np.abs(res.rho[a:e] - Rs[rows, j]).max() < 1e-10
        assert np.abs(eps[a:e] - Es[rows, j]).max() < 1e-10 * np.abs(lam).max()


def test_energy_density_column_identity(fo, oracle_lib):
    """sum_{i in P(j)} eps_ij S_ji = sum_{i in P(j)} rho_ij H_ji per column
    (real weights): z_k (G S)_jj - (G H)_jj = 1 for every shift.  Measured
    1.3e-13; with Re z_k in place of z_k, 2.3e-2."""
    O = oracle_lib
    wl, b, cols, res = overlap_solve(O)
    eps = fo.energy_density(res, wl.z, wl.w)
    H, S = b.dense("h"), b.dense("s")
    for c, j in enumerate(cols):
        a, e = res.proj_ptr[c], res.proj_ptr[c + 1]
        rows = res.proj_row[a:e]
        lhs = eps[a:e] @ S[j, rows]
        rhs = res.rho[a:e] @ H[j, rows]
        assert abs(lhs - rhs) < 1e-10, (j, lhs, rhs)
