"""Oracle for the band-structure (Hellmann-Feynman) forces from the density
matrix, the force step of the quantum molecular dynamics (Sec. 2 of the
paper; the method is that of its reference on the order-N solver).

TEST INFRASTRUCTURE ONLY, under the same rule as the rest of ``oracle``.

Readings:
* The band energy of the solved columns is E_band = sum_j sum_{i in P(j)}
  rho_ij H_ij (per spin; the tr(rho H) of the traces after rho).  With an
  orthogonal basis (S = I) the force is F_A = -dE_band/dR_A at fixed rho.
* With an overlap S, the generalized eigenproblem H c = lambda S c gives
  d lambda/dR = c^T (dH/dR - lambda dS/dR) c (Hellmann-Feynman), so the
  force at fixed occupations is F_A = -sum (rho_ij dH_ij/dR_A - eps_ij
  dS_ij/dR_A) with the energy-density matrix eps = sum_n f_n lambda_n c_n
  c_n^T.  From the shifted solves, eps_ij = -(1/pi) sum_k Im(w_k z_k
  G_ij(z_k)): the same quadrature as rho with the weight w_k z_k.  Because
  (z S - H) G = I, this eps satisfies sum eps_ij S_ji = sum rho_ij H_ji
  (for real weights) column by column, up to the solver's tolerance.
* Each column's rho and eps come from its own local subspace, so rho_ij and
  rho_ji differ and no symmetry is assumed.  H_ij for orbital i on atom B
  and j on atom C (B != C) is element (o_i, q_j) of the Slater-Koster block
  h(d), d = R_C - R_B, and S_ij is element (o_i, q_j) of the overlap block
  s(d) = s_amp exp(-(r - r0)/s_decay) I4, so the term g = rho_ij grad
  h_{o_i q_j}(d) - eps_ij grad s_{o_i q_j}(d) enters F_C with a minus sign
  and F_B with a plus sign (on-site blocks do not depend on positions, and
  a pair farther apart than r_cut has no block).  The forces therefore sum
  to zero.  The repulsive and van der Waals terms are
  not part of it.
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


def overlap_grad(d, tb) -> np.ndarray:
    """d s(d) / d d_g as an array [3][4][4] for the overlap block
    s(d) = s_amp exp(-(r - r0)/s_decay) I4: -s(r) c_g / s_decay on the
    diagonal."""
    r = float(np.linalg.norm(d))
    c = np.asarray(d, float) / r
    v = tb.s_amp * np.exp(-(r - tb.r0) / tb.s_decay)
    return (-v / tb.s_decay * c)[:, None, None] * np.eye(4)[None, :, :]


def energy_density(res, z, w) -> np.ndarray:
    """eps_t = -(1/pi) sum_k Im(w_k z_k G_t(z_k)) for every projection row t
    of ``res`` (which must hold G)."""
    zw = np.asarray(z, np.complex128) * np.asarray(w, np.complex128)
    return -(res.G @ zw).imag / np.pi


def band_forces(xyz, tb, res, cols, n_atoms, eps=None) -> np.ndarray:
    """F [n_atoms][3] = -d/dR (sum rho_ij H_ij - sum eps_ij S_ij) at fixed
    rho and eps, summed over the columns solved in ``res`` (projection rows
    res.proj_ptr, res.proj_row, res.rho).  ``eps`` (one value per
    projection row) is required when tb.overlap is set and ignored
    otherwise."""
    ovl = bool(getattr(tb, "overlap", 0))
    if ovl and eps is None:
        raise ValueError("band_forces: an overlap needs the energy-density matrix")
    F = np.zeros((n_atoms, 3))
    for c, j in enumerate(np.asarray(cols)):
        C, q = int(j) // 4, int(j) % 4
        for t in range(res.proj_ptr[c], res.proj_ptr[c + 1]):
            i = int(res.proj_row[t])
            B, o = i // 4, i % 4
            d = xyz[C] - xyz[B]
            if B == C or d @ d > tb.r_cut ** 2:   # on-site, or no block beyond the cut
                continue
            g = res.rho[t] * sk_grad(d, tb)[:, o, q]
            if ovl:
                g = g - eps[t] * overlap_grad(d, tb)[:, o, q]
            F[C] -= g
            F[B] += g
    return F
