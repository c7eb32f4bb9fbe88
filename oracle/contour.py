"""Oracle of the Fermi-Dirac density matrix from a few complex shifts (test
infrastructure only, under the same rule as the rest of ``oracle``).

The paper's order-N energy needs rho = f(H) with the Fermi occupation f, and
its method is the shifted solve (z S - H)x = b at complex z (Introduction).
A real-axis grid needs z close to the real axis and many points; the reading
here is a pole expansion of the Fermi function, the continued fraction of
Ozaki (Phys. Rev. B 75, 035123 (2007)), whose poles lie far from the real
axis, so that far fewer shifts reach a given accuracy.

The function: with y = (e - mu)/kT, f = 1/2 - tanh(y/2)/2 and Lambert's
continued fraction tanh(u) = u/(1 + u^2/(3 + u^2/(5 + ...))).  Cut after
2N partial denominators it is u e1^T (I + i u B)^{-1} e1, with B the
symmetric tridiagonal matrix of zero diagonal and off-diagonal
1/sqrt((2m-1)(2m+1)), m = 1 .. 2N-1.  With B = Q diag(l) Q^T the positive
eigenvalues l_p give the poles z_p = 2/l_p and residues R_p = Q_{1p}^2/l_p^2:
    f(y) = 1/2 - sum_p R_p (1/(y - i z_p) + 1/(y + i z_p)).
For the eigenpairs (lambda, v) of H v = lambda S v (v^T S v = 1), G(z) =
sum v v^T/(z - lambda) and sum v v^T = S^{-1}, so
    rho = sum f(lambda) v v^T = S^{-1}/2 + 2 kT sum_p R_p Re G(mu + i z_p kT),
and S^{-1} = Re(i M G(i M)) + O(|H|^2/M^2) for a large real M.  In the
library's quadrature form rho = -(1/pi) sum_k Im(w_k G(z_k)) these are the
shifts mu + i z_p kT with weights -2 pi i kT R_p, and i M with weight pi M/2.
"""
from __future__ import annotations

import numpy as np


def cf_poles(n_poles: int):
    """(z_p, R_p), p = 1 .. n_poles, ascending z_p (numpy eigh of B)."""
    n = 2 * n_poles
    m = np.arange(1, n)
    off = 1.0 / np.sqrt((2.0 * m - 1.0) * (2.0 * m + 1.0))
    B = np.diag(off, 1) + np.diag(off, -1)
    lam, Q = np.linalg.eigh(B)
    pos = lam > 0
    lam, q = lam[pos], Q[0, pos]
    z = 2.0 / lam
    R = q * q / (lam * lam)
    o = np.argsort(z)
    return z[o], R[o]


def fermi_approx(y, z, R):
    """The pole expansion of f at y = (e - mu)/kT."""
    y = np.asarray(y, np.float64)[..., None]
    return 0.5 - np.sum(R * 2.0 * y / (y * y + z * z), axis=-1)


def fermi(y):
    """1/(1 + exp(y)), written through tanh so that it does not overflow."""
    return 0.5 * (1.0 - np.tanh(0.5 * np.asarray(y, np.float64)))


def fermi_shifts(n_poles: int, kT: float, mu: float, moment: float = 1e8):
    """Shifts and weights (complex128 [n_poles + 1]): the poles nearest the
    real axis first, the moment shift i*moment last."""
    zp, R = cf_poles(n_poles)
    z = np.concatenate([mu + 1j * zp * kT, [1j * moment]])
    w = np.concatenate([-2j * np.pi * kT * R, [np.pi * moment / 2.0]])
    return z.astype(np.complex128), w.astype(np.complex128)


def fermi_rho_dense(H, S, kT: float, mu: float):
    """rho = V f(Lambda) V^T from the generalized eigenpairs of (H, S),
    V^T S V = I (the plain definition, for pins and accuracy checks)."""
    import scipy.linalg
    lam, V = scipy.linalg.eigh(H, S)
    return (V * fermi((lam - mu) / kT)) @ V.T


def fermi_rho_columns(bsr, xyz, cols, kT, mu, radius=0.0, prune=True):
    """Exact Fermi-Dirac rho on the projection rows of each column's local
    subspace: returns (proj_ptr, proj_row, rho) in the layout of the solve,
    from the dense eigen-decomposition of (H_L, S_L)."""
    import oracle
    cols = np.asarray(cols, np.int64)
    ref = oracle.shifted_solve(bsr, xyz, cols, np.array([1j]), tol=1e-3, radius=radius, prune=prune, max_iter=1)
    rho = np.zeros(ref.proj_row.size)
    for c, j in enumerate(cols):
        full = oracle.solve_full(bsr, xyz, int(j), np.array([1j]), radius=radius, prune=prune, max_iter=1)
        H, S, idx = oracle.local_dense(bsr, full.loc_atoms)
        jl = int(np.nonzero(idx == j)[0][0])
        r = fermi_rho_dense(H, S, kT, mu)[:, jl]
        a, b = ref.proj_ptr[c], ref.proj_ptr[c + 1]
        rho[a:b] = r[np.searchsorted(idx, ref.proj_row[a:b])]
    return ref.proj_ptr, ref.proj_row, rho
