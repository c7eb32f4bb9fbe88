"""Oracle of the quantum-MD time step (test infrastructure only, under the
same rule as the rest of ``oracle``: only tests, the smoke check and the
CPU-baseline leg of the benchmark use it).

The paper advances the atoms of its QMD runs with a 1 fs step (Sec. 2) and
leaves the integrator to its references; the reading here is velocity Verlet
(Swope, Andersen, Berens and Wilson 1982), written out in plain FP64 numpy:

    v_{n+1/2} = v_n + (h/2) a_n,   x_{n+1} = x_n + h v_{n+1/2},
    v_{n+1}   = v_{n+1/2} + (h/2) a_{n+1},     a = F / m.

Units: nm, fs, eV/nm, amu; a [nm/fs^2] = F/m x e/u x 1e-12 with
e = 1.602176634e-19 C and u = 1.66053906660e-27 kg.
"""
from __future__ import annotations

import numpy as np

E_CHARGE = 1.602176634e-19       # C (exact)
AMU = 1.66053906660e-27          # kg (CODATA 2018)
ACCEL = E_CHARGE / AMU * 1e-12   # nm/fs^2 per (eV/nm / amu)


def accel(force, mass):
    """a = F / m in nm/fs^2 for F [n, 3] in eV/nm and m [n] in amu."""
    return np.asarray(force, np.float64) * (ACCEL / np.asarray(mass, np.float64))[:, None]


def verlet_step(x, v, f, mass, h, force_at):
    """One velocity-Verlet step from (x, v) with forces f = F(x); force_at(x)
    returns the forces at new positions.  Returns (x, v, f) at t + h."""
    v_half = v + 0.5 * h * accel(f, mass)
    x_new = x + h * v_half
    f_new = force_at(x_new)
    return x_new, v_half + 0.5 * h * accel(f_new, mass), f_new
