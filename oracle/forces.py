"""Oracle for the band-structure (Hellmann-Feynman) forces from the density
matrix, the force step of the quantum molecular dynamics (Sec. 2 of the
paper; the method is that of its reference on the order-N solver).

TEST INFRASTRUCTURE ONLY, under the same rule as the rest of ``oracle``.

Readings:
* Orthogonal basis (S = I).  The band energy of the solved columns is
  E_band = sum_j sum_{i in P(j)} rho_ij H_ij (per spin; the tr(rho H) of
  the traces after rho), and the force is F_A = -dE_band/dR_A at fixed rho.
  Each column's rho comes from its own local subspace, so rho_ij and rho_ji
  differ and no symmetry of rho is assumed.  The term with the
  energy-density matrix that an overlap adds, and the repulsive and van der
  Waals terms, are not part of it.
* H_ij for orbital i on atom B and j on atom C (B != C) is element
  (o_i, q_j) of the Slater-Koster block h(d), d = R_C - R_B, so the term
  g = rho_ij grad h_{o_i q_j}(R_C - R_B) enters F_C with a minus sign and
  F_B with a plus sign (on-site blocks do not depend on positions).  The
  forces therefore sum to zero.
"""
from __future__ import annotations

import numpy as np


def sk_block(d, tb) -> np.ndarray:
    """The 4x4 block h(d) (orbitals s, px, py, pz; d = R_col - R_row, nm)."""
    r = float(np.linalg.norm(d))
    c = np.asarray(d, float) / r
    f = (tb.r0 / r) ** tb.power
    h = np.empty((4, 4))
    h[0, 0] = tb.v_sss * f
    h[0, 1:] = c * tb.v_sps * f
    h[1:, 0] = -c * tb.v_sps * f
    h[1:, 1:] = (np.outer(c, c) * (tb.v_pps - tb.v_ppp) + np.eye(3) * tb.v_ppp) * f
    return h


def sk_grad(d, tb) -> np.ndarray:
    """d h(d) / d d_g as an array [3][4][4] (derivative of the direction
    cosines, (delta_ag - c_a c_g)/r, and of the scaling, -power f c_g / r)."""
    r = float(np.linalg.norm(d))
    c = np.asarray(d, float) / r
    f = (tb.r0 / r) ** tb.power
    dc = (np.eye(3) - np.outer(c, c)) / r          # dc[a, g] = d c_a / d d_g
    df = -tb.power * f * c / r                      # df[g]
    g = np.empty((3, 4, 4))
    for k in range(3):
        g[k, 0, 0] = tb.v_sss * df[k]
        sp = tb.v_sps * (dc[:, k] * f + c * df[k])
        g[k, 0, 1:] = sp
        g[k, 1:, 0] = -sp
        dcc = np.outer(dc[:, k], c) + np.outer(c, dc[:, k])
        g[k, 1:, 1:] = dcc * (tb.v_pps - tb.v_ppp) * f + (np.outer(c, c) * (tb.v_pps - tb.v_ppp)
                                                          + np.eye(3) * tb.v_ppp) * df[k]
    return g


def band_forces(xyz, tb, res, cols, n_atoms) -> np.ndarray:
    """F [n_atoms][3] = -dE_band/dR at fixed rho, E_band over the columns
    solved in ``res`` (projection rows res.proj_ptr, res.proj_row, res.rho)."""
    F = np.zeros((n_atoms, 3))
    for c, j in enumerate(np.asarray(cols)):
        C, q = int(j) // 4, int(j) % 4
        for t in range(res.proj_ptr[c], res.proj_ptr[c + 1]):
            i = int(res.proj_row[t])
            B, o = i // 4, i % 4
            if B == C:
                continue
            g = res.rho[t] * sk_grad(xyz[C] - xyz[B], tb)[:, o, q]
            F[C] -= g
            F[B] += g
    return F
