"""Oracle for the wavepacket step: time propagation of a hole wavepacket by
the time-dependent Schroedinger equation with the tight-binding Hamiltonian
(Sec. 3 of the paper, transport with wavepacket dynamics, Fig. 2: d/dt Psi = -i H_WP Psi, time step 0.1 fs).

TEST INFRASTRUCTURE ONLY, under the same rule as the rest of ``oracle``: only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library.

Readings (the paper gives only the equation and the step):
* H_WP is the tight-binding H of the structure in an orthogonal basis
  (S = I), in eV; time in fs, so one step of length h is
  Psi(t + h) = exp(-i H h / hbar) Psi(t) with hbar in eV fs.
* Two forms are given here.  ``exact_propagate`` is that definition, taken
  through the eigen-decomposition of the dense H (small systems).
  ``chebyshev_propagate`` is the Chebyshev expansion of the same exponential
  (Tal-Ezer and Kosloff, J. Chem. Phys. 81, 3967 (1984)): with H = a X + b,
  the spectrum of X inside [-1, 1] and tau = h / hbar,
      exp(-i tau H) = exp(-i tau b) sum_k c_k T_k(X),
      c_0 = J_0(a tau),  c_k = 2 (-i)^k J_k(a tau)  (k >= 1),
  with T_0 = 1, T_1 = X, T_{k+1} = 2 X T_k - T_{k-1} applied to the vector.
* a and b come from Gershgorin bounds of H:
  [min_i (H_ii - R_i), max_i (H_ii + R_i)], R_i = sum_{j != i} |H_ij|.
* The series is cut at K terms, the smallest K > a tau with
  |J_k(a tau)| <= tol for k = K and K + 1 (beyond k > a tau the J_k decay
  faster than geometrically, so the tail is below ~2 tol).
"""
from __future__ import annotations

import numpy as np
from scipy.special import jv

#: hbar in eV fs (CODATA 2018: 6.582119569e-16 eV s)
HBAR_EV_FS = 0.6582119569509066


def gershgorin_bounds(bsr) -> tuple:
    """(e_min, e_max) of the Gershgorin discs of H, row by row."""
    n = 4 * bsr.n_atoms
    diag = np.zeros(n)
    rad = np.zeros(n)
    for a in range(bsr.n_atoms):
        for t in range(bsr.row_ptr[a], bsr.row_ptr[a + 1]):
            b = int(bsr.col[t])
            blk = bsr.h[t]
            for o in range(4):
                i = 4 * a + o
                for q in range(4):
                    j = 4 * b + q
                    if i == j:
                        diag[i] += blk[o, q]
                    else:
                        rad[i] += abs(blk[o, q])
    return float((diag - rad).min()), float((diag + rad).max())


def chebyshev_coefficients(a_tau: float, n_terms: int) -> np.ndarray:
    """c_k of exp(-i a_tau x) = sum_k c_k T_k(x) on [-1, 1], k < n_terms."""
    k = np.arange(n_terms)
    c = jv(k, a_tau) * (-1j) ** k
    c[1:] *= 2.0
    return c


def chebyshev_terms(a_tau: float, tol: float = 1e-13) -> int:
    """Number of series terms for argument a_tau (rule in the header)."""
    k = int(np.floor(a_tau)) + 1
    while not (abs(jv(k, a_tau)) <= tol and abs(jv(k + 1, a_tau)) <= tol):
        k += 1
    return k


def _matvec(bsr, x):
    import scipy.sparse as sp
    n = 4 * bsr.n_atoms
    return sp.bsr_matrix((bsr.h, bsr.col, bsr.row_ptr), shape=(n, n)) @ x


def chebyshev_propagate(bsr, psi, h_fs: float, n_steps: int, e_min: float, e_max: float,
                        n_terms: int) -> np.ndarray:
    """n_steps steps of length h_fs of psi ([n_orb] or [n_orb, n_packets])."""
    if bsr.s is not None:
        raise ValueError("the propagation is defined for an orthogonal basis (S = I)")
    a = 0.5 * (e_max - e_min)
    b = 0.5 * (e_max + e_min)
    tau = h_fs / HBAR_EV_FS
    c = chebyshev_coefficients(a * tau, n_terms) * np.exp(-1j * tau * b)
    psi = np.array(psi, dtype=np.complex128)
    for _ in range(n_steps):
        t_prev = psi                                   # T_0 psi
        t_cur = (_matvec(bsr, psi) - b * psi) / a      # T_1 psi
        acc = c[0] * t_prev + c[1] * t_cur
        for k in range(2, n_terms):
            t_next = 2.0 * (_matvec(bsr, t_cur) - b * t_cur) / a - t_prev
            acc = acc + c[k] * t_next
            t_prev, t_cur = t_cur, t_next
        psi = acc
    return psi


def exact_propagate(bsr, psi, t_fs: float) -> np.ndarray:
    """exp(-i H t / hbar) psi by the eigen-decomposition of the dense H."""
    if bsr.s is not None:
        raise ValueError("the propagation is defined for an orthogonal basis (S = I)")
    lam, V = np.linalg.eigh(bsr.dense("h"))
    ph = np.exp(-1j * lam * (t_fs / HBAR_EV_FS))
    psi = np.asarray(psi, dtype=np.complex128)
    coef = V.T @ psi
    if coef.ndim == 1:
        return V @ (ph * coef)
    return V @ (ph[:, None] * coef)
