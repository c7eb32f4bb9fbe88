"""Pins for the CPU oracle: each test checks it against something other than
itself -- dense LU, closed forms, the spectrum, invariants of the method.

The problem (paper, Introduction): solve (zS - H)x = b in place of the
generalized eigenproblem H y = lambda S y.  The oracle solves it by shifted
COCG on each column's local subspace.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.csgraph

import workloads as W


def small_bundle(nx=2, ny=2, n=30, overlap=False, config_no=90, **kw):
    wl = W.bundle_workload(nx, ny, n, overlap=overlap, config_no=config_no, n_shifts=kw.pop("n_shifts", 24), **kw)
    return wl


# ---------------------------------------------------------------------------
# Hamiltonian construction
# ---------------------------------------------------------------------------

def test_sk_block_structure(oracle_lib):
    """Slater-Koster block of one bond, checked by its rotation-invariant parts:
    H[s][s] = Vss f, H[s][p] = Vsp f * c, H[p][s] = -Vsp f * c and the pp block
    has eigenvalues (Vpp_sigma f, Vpp_pi f, Vpp_pi f) with eigenvector c for
    the sigma one; f = (r0/r)^2."""
    O = oracle_lib
    p = W.BUNDLE_TB
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = rng.normal(size=3)
        d *= rng.uniform(0.1, 0.29) / np.linalg.norm(d)
        xyz = np.array([[0.3, 0.1, -0.2], [0.3, 0.1, -0.2] + d])
        b = O.tb_build(xyz, p)
        assert list(b.row_ptr) == [0, 2, 4] and list(b.col) == [0, 1, 0, 1]
        r = np.linalg.norm(d)
        c = d / r
        f = (p.r0 / r) ** 2
        H01 = b.h[1]
        assert H01[0, 0] == pytest.approx(p.v_sss * f, rel=1e-14)
        np.testing.assert_allclose(H01[0, 1:], p.v_sps * f * c, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(H01[1:, 0], -p.v_sps * f * c, rtol=1e-13, atol=1e-14)
        ev, vec = np.linalg.eigh(H01[1:, 1:])
        np.testing.assert_allclose(sorted(ev), sorted([p.v_pps * f, p.v_ppp * f, p.v_ppp * f]), rtol=1e-12)
        sig = vec[:, np.argmin(np.abs(ev - p.v_pps * f))]
        assert abs(abs(sig @ c) - 1) < 1e-12
        # H_ba = H_ab^T, on-site blocks
        np.testing.assert_array_equal(b.h[2], H01.T)
        np.testing.assert_array_equal(b.h[0], np.diag([p.e_s, p.e_p, p.e_p, p.e_p]))


def test_overlap_block(oracle_lib):
    O = oracle_lib
    p = W.BUNDLE_TB_OVERLAP
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.2]])
    b = O.tb_build(xyz, p)
    np.testing.assert_array_equal(b.s[0], np.eye(4))
    np.testing.assert_allclose(b.s[1], 0.1 * np.exp(-(0.2 - 0.14) / 0.05) * np.eye(4), rtol=1e-14)


def test_bond_pattern_vs_brute_force(oracle_lib):
    """Cell-list neighbour search equals the O(N^2) distance test."""
    O = oracle_lib
    wl = small_bundle(3, 3, 40)
    b = O.tb_build(wl.xyz, wl.tb)
    x = wl.xyz
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    A = d2 <= wl.tb.r_cut ** 2  # includes the diagonal
    for a in range(x.shape[0]):
        np.testing.assert_array_equal(b.col[b.row_ptr[a]:b.row_ptr[a + 1]], np.nonzero(A[a])[0])
    H = b.dense("h")
    np.testing.assert_array_equal(H, H.T)


def test_bundle_sizes(oracle_lib):
    """Full bundle: 118,300 atoms; chains 0.45 nm apart share no bond."""
    O = oracle_lib
    wl = W.config_bundle()
    assert wl.xyz.shape == (118300, 3) and wl.columns.size == 473200
    b = O.tb_build(wl.xyz, wl.tb)
    assert 4.3 < b.nnzb / b.n_atoms < 4.6
    chain_of = np.repeat(np.arange(169), 700)
    rows = np.repeat(np.arange(b.n_atoms), np.diff(b.row_ptr))
    assert np.all(chain_of[rows] == chain_of[b.col])


def test_overlap_spd(oracle_lib):
    """S of the overlap workload is symmetric positive definite."""
    O = oracle_lib
    wl = small_bundle(2, 2, 60, overlap=True)
    b = O.tb_build(wl.xyz, wl.tb)
    S = b.dense("s")
    np.testing.assert_array_equal(S, S.T)
    assert np.linalg.eigvalsh(S).min() > 0.05


def test_chain_builder(oracle_lib):
    O = oracle_lib
    wl = W.chain_workload(40, 4, 8)
    b = O.chain_build(wl.onsite, wl.hopping)
    assert b.nnzb == 3 * 10 - 2
    H = b.dense("h")
    ref = np.diag(wl.onsite) + wl.hopping * (np.eye(40, k=1) + np.eye(40, k=-1))
    np.testing.assert_array_equal(H, ref)


# ---------------------------------------------------------------------------
# Local subspaces
# ---------------------------------------------------------------------------

def test_local_subspace_sizes_vs_brute_force(oracle_lib):
    O = oracle_lib
    wl = small_bundle(3, 3, 40)
    b = O.tb_build(wl.xyz, wl.tb)
    cols = np.arange(0, wl.n_orb, 37)
    R = 0.8
    n_loc, n_proj = O.plan_sizes(b, wl.xyz, cols, R, None, prune=False)
    n_loc_p, n_proj_p = O.plan_sizes(b, wl.xyz, cols, R, None, prune=True)
    x = wl.xyz
    Hpat = scipy.sparse.csr_matrix((np.ones(b.nnzb), b.col, b.row_ptr))
    for i, j in enumerate(cols):
        c = j // 4
        ball = np.nonzero(((x - x[c]) ** 2).sum(1) <= R * R)[0]
        assert n_loc[i] == ball.size
        sub = Hpat[ball][:, ball]
        _, lab = scipy.sparse.csgraph.connected_components(sub, directed=False)
        comp = ball[lab == lab[np.searchsorted(ball, c)]]
        assert n_loc_p[i] == comp.size
        nbrs = b.col[b.row_ptr[c]:b.row_ptr[c + 1]]
        assert n_proj[i] == 4 * np.isin(nbrs, ball).sum() == n_proj_p[i]


# ---------------------------------------------------------------------------
# Shifted COCG against the exact restricted solve
# ---------------------------------------------------------------------------

def _check_against_dense(O, b, wl, cols, radius, prune, rtol):
    res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=wl.tol, radius=radius, prune=prune)
    assert np.all(res.status == O.CONVERGED)
    for c, j in enumerate(cols):
        full = O.solve_full(b, wl.xyz, int(j), wl.z[:1], radius=radius, prune=prune, max_iter=1)
        H, S, idx = O.local_dense(b, full.loc_atoms)
        jl = int(np.nonzero(idx == j)[0][0])
        X = O.exact_columns(H, S, jl, wl.z)
        rows, G, rho = res.column(c)
        pos = np.searchsorted(idx, rows)
        ref = X[pos]
        err = np.abs(G - ref).max() / np.abs(ref).max()
        assert err < rtol, (j, err)
        # density matrix: rho_ij = -(1/pi) sum_k Im(w_k G_ij(z_k))
        np.testing.assert_allclose(rho, -(ref * wl.w[None, :]).imag.sum(1) / np.pi, rtol=0, atol=rtol * 10)
    return res


def test_cocg_chain_vs_dense_lu(oracle_lib):
    wl = W.chain_workload(200, 6, 16, config_no=91)
    b = oracle_lib.chain_build(wl.onsite, wl.hopping)
    _check_against_dense(oracle_lib, b, wl, wl.columns, 0.0, False, 1e-9)


@pytest.mark.parametrize("prune", [False, True])
def test_cocg_bundle_vs_dense_lu(oracle_lib, prune):
    wl = small_bundle(2, 2, 30)
    b = oracle_lib.tb_build(wl.xyz, wl.tb)
    cols = np.array([0, 5, 62, 243, 477])
    _check_against_dense(oracle_lib, b, wl, cols, 0.9, prune, 1e-9)


def test_cocg_overlap_vs_dense_lu(oracle_lib):
    wl = small_bundle(2, 2, 30, overlap=True)
    b = oracle_lib.tb_build(wl.xyz, wl.tb)
    cols = np.array([1, 7, 130, 401])
    _check_against_dense(oracle_lib, b, wl, cols, 0.9, True, 1e-9)


def test_eigen_expansion(oracle_lib):
    """G(z) = sum_lambda v v^T / (z - lambda) with S-normalised generalized
    eigenvectors, for S = I and S != I."""
    O = oracle_lib
    for overlap in (False, True):
        wl = small_bundle(1, 1, 24, overlap=overlap, n_shifts=16)
        b = O.tb_build(wl.xyz, wl.tb)
        H, S = b.dense("h"), b.dense("s")
        lam, V = scipy.linalg.eigh(H, S)
        cols = np.array([0, 13, 50, 95])
        res = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=0.0)
        for c, j in enumerate(cols):
            rows, G, rho = res.column(c)
            ref = (V[rows][:, None, :] * V[j][None, None, :] / (wl.z[None, :, None] - lam[None, None, :])).sum(-1)
            assert np.abs(G - ref).max() / np.abs(ref).max() < 1e-9
            # discrete density matrix closed form
            dens = (-(wl.w[:, None] / (wl.z[:, None] - lam[None, :])).imag / np.pi).sum(0)
            rho_ref = (V[rows] * V[j][None, :] * dens[None, :]).sum(1)
            np.testing.assert_allclose(rho, rho_ref, atol=1e-9)


def test_clean_chain_closed_form(oracle_lib):
    """Uniform chain (no disorder): lambda_m = 2t cos(m pi/(N+1)),
    v_m(i) = sqrt(2/(N+1)) sin(i m pi/(N+1)), i, m = 1..N."""
    O = oracle_lib
    N, t = 120, -1.0
    wl = W.chain_workload(N, 5, 20, disorder=0.0, config_no=92)
    b = O.chain_build(np.zeros(N), t)
    res = O.shifted_solve(b, None, wl.columns, wl.z, wl.w, tol=1e-12)
    m = np.arange(1, N + 1)
    lam = 2 * t * np.cos(m * np.pi / (N + 1))
    V = np.sqrt(2 / (N + 1)) * np.sin(np.outer(np.arange(1, N + 1), m) * np.pi / (N + 1))
    for c, j in enumerate(wl.columns):
        rows, G, _ = res.column(c)
        ref = (V[rows][:, None, :] * V[j][None, None, :] / (wl.z[None, :, None] - lam[None, None, :])).sum(-1)
        assert np.abs(G - ref).max() / np.abs(ref).max() < 1e-10


def test_isolated_atom(oracle_lib):
    """An atom with no bond: G = diag(1/(z - E_s), 1/(z - E_p) x 3)."""
    O = oracle_lib
    p = W.BUNDLE_TB
    xyz = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    b = O.tb_build(xyz, p)
    z = W.shift_grid(-10, 10, 9, 0.05)
    for o, e in enumerate([p.e_s, p.e_p, p.e_p, p.e_p]):
        res = O.shifted_solve(b, xyz, np.array([o]), z, None, tol=1e-13, radius=1.0)
        rows, G, _ = res.column(0)
        np.testing.assert_array_equal(rows, [0, 1, 2, 3])
        np.testing.assert_allclose(G[o], 1 / (z - e), rtol=1e-13)
        assert np.abs(np.delete(G, o, axis=0)).max() == 0


def test_dimer_pi_closed_form(oracle_lib):
    """Dimer along z: each p_x pair is a 2x2 problem [[Ep, V],[V, Ep]] with
    V = Vpp_pi (r0/r)^2, so G_xx(z) = (z-Ep)/((z-Ep)^2 - V^2) and
    G_x'x(z) = V/((z-Ep)^2 - V^2)."""
    O = oracle_lib
    p = W.BUNDLE_TB
    r = 0.15
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    b = O.tb_build(xyz, p)
    V = p.v_ppp * (p.r0 / r) ** 2
    z = W.shift_grid(-20, 20, 17, 0.02)
    res = O.shifted_solve(b, xyz, np.array([1]), z, None, tol=1e-13, radius=1.0)
    rows, G, _ = res.column(0)
    d = (z - p.e_p) ** 2 - V ** 2
    for row, ref in ((1, (z - p.e_p) / d), (5, V / d)):
        got = G[list(rows).index(row)]
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12


def test_symmetry_and_herglotz(oracle_lib):
    """G_ij = G_ji from two separate column solves (whole chain), and
    Im G_jj(E + i eta) < 0."""
    O = oracle_lib
    wl = W.chain_workload(160, 4, 12, config_no=93)
    b = O.chain_build(wl.onsite, wl.hopping)
    cols = np.array([40, 41, 42, 43, 44, 45])
    res = O.shifted_solve(b, None, cols, wl.z, wl.w, tol=1e-12)
    for c, j in enumerate(cols):
        rows, G, _ = res.column(c)
        for c2, i in enumerate(cols):
            if i in rows:
                rows2, G2, _ = res.column(c2)
                np.testing.assert_allclose(G[list(rows).index(i)], G2[list(rows2).index(j)], rtol=1e-9, atol=1e-12)
    assert np.all(res.g_diag(cols).imag < 0)
    wlo = small_bundle(2, 1, 20, overlap=True, n_shifts=16)
    bo = O.tb_build(wlo.xyz, wlo.tb)
    reso = O.shifted_solve(bo, wlo.xyz, np.arange(0, 160, 9), wlo.z, None, tol=1e-12, radius=0.8)
    assert np.all(reso.g_diag(np.arange(0, 160, 9)).imag < 0)


@pytest.mark.parametrize("overlap", [False, True])
def test_sum_rule(oracle_lib, overlap):
    """-(1/pi) int Im G_jj dE = 1 for S = I; -(1/pi) int Im (G S)_jj dE = 1 in
    general.  On a finite window [a, b] the broadened count is
    sum_lambda v_j^2 (1/pi)[atan((b-lambda)/eta) - atan((a-lambda)/eta)];
    the trapezoid sum over a fine grid must match it, and it must be close to 1."""
    O = oracle_lib
    wl = small_bundle(1, 1, 16, overlap=overlap, n_shifts=8)
    b = O.tb_build(wl.xyz, wl.tb)
    H, S = b.dense("h"), b.dense("s")
    lam, V = scipy.linalg.eigh(H, S)
    a_, b_, eta = -120.0, 120.0, 0.5
    z = W.shift_grid(a_, b_, 4801, eta)
    wts = np.full(z.size, (b_ - a_) / (z.size - 1))
    wts[[0, -1]] *= 0.5
    j = 6
    res = O.shifted_solve(b, wl.xyz, np.array([j]), z, None, tol=1e-11, radius=0.0)
    rows, G, _ = res.column(0)
    Srow = S[j, rows]
    gs = (G * Srow[:, None]).sum(0)  # (G S)_jj = sum_i G_ji S_ij (G symmetric)
    count = -(wts * gs.imag).sum() / np.pi
    u = V[j] * (V.T @ S[:, j])  # contribution of each eigenpair to (G S)_jj's residue
    closed = (u * (np.arctan((b_ - lam) / eta) - np.arctan((a_ - lam) / eta))).sum() / np.pi
    assert abs(count - closed) < 2e-4
    assert abs(count - 1.0) < 1e-2


def test_collinear_residuals(oracle_lib):
    """After n steps the true residual of shift k is the seed's over pi^k:
    b - (z_k S - H) x^k_n = s_n / pi^k_n."""
    O = oracle_lib
    for overlap in (False, True):
        wl = small_bundle(1, 2, 25, overlap=overlap, n_shifts=12)
        b = O.tb_build(wl.xyz, wl.tb)
        j = 41
        full = O.solve_full(b, wl.xyz, j, wl.z, tol=1e-30, radius=1.0, prune=False, max_iter=9)
        assert full.iters == 9
        H, S, idx = O.local_dense(b, full.loc_atoms)
        e = (idx == j).astype(complex)
        for k in range(wl.z.size):
            lhs = e - (wl.z[k] * S - H) @ full.x[:, k]
            np.testing.assert_allclose(lhs, full.s / full.pi[k], atol=1e-12 * np.abs(lhs).max() + 1e-15)


def test_seed_invariance(oracle_lib):
    """The seed choice changes results only within the tolerance bound."""
    O = oracle_lib
    wl = small_bundle(2, 2, 30, n_shifts=16)
    b = O.tb_build(wl.xyz, wl.tb)
    cols = np.array([3, 100, 250])
    r1 = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-11, radius=1.0, prune=True, seed_index=8)
    r2 = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-11, radius=1.0, prune=True, seed_index=0)
    r3 = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-11, radius=1.0, prune=True, seed_index=15)
    # |dx| <= tol |b| / eta per shift (S = I)
    bound = 2 * 1e-11 / 0.01
    assert np.abs(r1.G - r2.G).max() < bound and np.abs(r1.G - r3.G).max() < bound


def test_subspace_limit_and_prune(oracle_lib):
    """A radius that covers the system equals the whole-system solve; pruning
    to the connected component leaves the result unchanged."""
    O = oracle_lib
    wl = small_bundle(2, 2, 20, n_shifts=12)
    b = O.tb_build(wl.xyz, wl.tb)
    cols = np.array([0, 33, 150, 301])
    full = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=0.0)
    big = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=50.0)
    pr = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=50.0, prune=True)
    np.testing.assert_array_equal(full.proj_row, big.proj_row)
    np.testing.assert_allclose(full.G, big.G, rtol=0, atol=1e-13 * np.abs(full.G).max())
    np.testing.assert_allclose(full.G, pr.G, rtol=0, atol=1e-11 * np.abs(full.G).max())


def test_generalized_code_with_identity_overlap(oracle_lib):
    """S = I stored explicitly through the generalized path equals S = I."""
    O = oracle_lib
    wl = small_bundle(1, 2, 25, n_shifts=10)
    b = O.tb_build(wl.xyz, wl.tb)
    bI = dataclasses.replace(b, s=np.zeros_like(b.h))
    rows = np.repeat(np.arange(b.n_atoms), np.diff(b.row_ptr))
    bI.s[rows == b.col] = np.eye(4)
    cols = np.array([2, 77, 150])
    r0 = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-11, radius=0.9)
    r1 = O.shifted_solve(bI, wl.xyz, cols, wl.z, wl.w, tol=1e-11, radius=0.9)
    np.testing.assert_array_equal(r0.iters, r1.iters)
    np.testing.assert_allclose(r0.G, r1.G, rtol=0, atol=1e-14 * np.abs(r0.G).max())


def test_status_codes(oracle_lib):
    """max_iter exhaustion gives MAXITER; a NaN block gives NONFINITE only for
    the columns whose subspace contains it."""
    O = oracle_lib
    wl = small_bundle(2, 1, 20, n_shifts=8)
    b = O.tb_build(wl.xyz, wl.tb)
    cols = np.array([0, 4, 100, 150])
    r = O.shifted_solve(b, wl.xyz, cols, wl.z, None, tol=1e-12, radius=0.6, prune=True, max_iter=2)
    assert np.all(r.status == O.MAXITER) and np.all(r.iters == 2)
    bad = dataclasses.replace(b, h=b.h.copy())
    bad.h[b.row_ptr[1]] = np.nan  # first block of atom 1 (chain 0)
    r = O.shifted_solve(bad, wl.xyz, cols, wl.z, None, tol=1e-12, radius=0.6, prune=True)
    assert list(r.status) == [O.NONFINITE, O.NONFINITE, O.CONVERGED, O.CONVERGED]


# The breakdown case (workloads.breakdown_block), worked by hand in exact
# arithmetic; every value is a small Gaussian integer, so FP64 reproduces it
# bit for bit.  Column j = 0, seed z_s = i: p_0 = e_0, w_0 = (i, -1, 0, 0),
# mu_0 = i, alpha_0 = -i, s_1 = (0, -i, 0, 0), rho_1 = -1, beta_0 = -1,
# p_1 = (-1, -i, 0, 0), w_1 = z_s p_1 - H p_1 = (-2i, 2, 0, 0) and
# mu_1 = p_1^T w_1 = 2i - 2i = 0 with s_1 != 0: a breakdown in the second
# iteration.  (For a symmetric H and Im z > 0 the pivots of z - T of the
# underlying Lanczos tridiagonal T keep Im >= Im z, so mu never vanishes; the
# crafted block breaks that symmetry on purpose.)  After the one completed
# step every shift holds the one-dimensional Galerkin solution
# x^k = e_0 / (z_k - H_00) = e_0 / z_k.


@pytest.mark.parametrize("explicit_s", [False, True])
def test_breakdown_status(oracle_lib, explicit_s):
    """SGF_BREAKDOWN on the hand-worked case above, through the S = I path
    and through the generalized path with S given as the identity block."""
    O = oracle_lib
    row_ptr, col, h, z = W.breakdown_block()
    s = np.eye(4)[None].copy() if explicit_s else None
    b = O.BSR(row_ptr, col, h, s)
    xyz = np.zeros((1, 3))
    r = O.shifted_solve(b, xyz, np.array([0]), z, None, tol=1e-12, radius=1.0, prune=True, seed_index=1)
    assert r.status[0] == O.BREAKDOWN and r.iters[0] == 2
    np.testing.assert_array_equal(r.proj_row, np.arange(4))
    G = r.G.reshape(4, z.size)
    np.testing.assert_allclose(G[0], 1.0 / z, rtol=1e-15, atol=0)
    assert np.all(G[1:] == 0)


@pytest.mark.parametrize("overlap", [False, True])
def test_apply_inverts_the_dense_solve(oracle_lib, overlap):
    """The global operator apply, pinned by an independent LAPACK solve: for
    x = (z S - H)^{-1} e_j from dense LU on the whole (small) system,
    (z S - H) x returns e_j; the row-by-row form agrees with the full one."""
    import oracle
    wl = W.bundle_workload(1, 2, 6, overlap=overlap, n_shifts=4, config_no=31)
    b = oracle.system_for(wl)
    atoms = np.arange(b.n_atoms)
    H, S, idx = oracle.local_dense(b, atoms)
    z = complex(wl.z[1])
    for j in (0, 5, 4 * b.n_atoms - 1):
        x = oracle.exact_columns(H, S, j, np.array([z]))[:, 0]
        y = oracle.apply(b, z, x)
        e = np.zeros_like(y)
        e[j] = 1.0
        assert np.abs(y - e).max() < 1e-12
        rows = np.array([j, (j + 3) % x.size])
        np.testing.assert_allclose(oracle.apply(b, z, x, rows=rows), y[rows], rtol=0, atol=1e-14)
