"""Seeded synthetic inputs for the shifted-COCG Green's-function path.

This module is the only code shared by the CPU oracle and the GPU library's
callers.  It draws geometry, disorder, column sets, radii, shift grids and
quadrature weights; it holds none of the method's arithmetic (no Hamiltonian
elements, no Krylov steps).

The paper (Introduction) states the problem as the generalized shifted linear
equations (zS - H)x = b solved in place of H y = lambda S y, at order-N cost;
its quantum MD section describes a bundle of 169 PPV chains (about 118k atoms).
The proprietary structures are not available, so every workload here is a
seeded stand-in of that shape:

* ``chain``  -- 1-D chain, one orbital per site, nearest-neighbour hopping,
  uniform on-site disorder (the small plain-method case, 2000 sites).
* ``bundle`` -- 13 x 13 chains of 700 sp atoms at 0.14 nm along z, 0.45 nm
  apart, Gaussian jitter sigma = 0.02 nm (118,300 atoms, the size of the
  paper's PPV bundle).
* ``bundle_overlap`` -- the bundle geometry with a non-orthogonal overlap S and
  a per-column local radius drawn from U[0.6, 1.4] nm.
* ``large`` -- the bundle generator at 1,000,300 atoms (1,429 chains on the
  first sites of a 38 x 38 grid): one GPU's share of a 10^8-atom run.

Seeds: ``SeedSequence([1603, config_no, stream])`` with streams 0 geometry and
disorder, 1 columns, 2 radii, 3 learned-scheduler data.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional

import numpy as np

SEED_ROOT = 1603

STREAM_GEOMETRY = 0
STREAM_COLUMNS = 1
STREAM_RADII = 2
STREAM_MLP = 3
STREAM_WAVEPACKET = 4


def rng(config_no: int, stream: int) -> np.random.Generator:
    """Independent PCG64 stream for (configuration, purpose)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, config_no, stream])))


# ---------------------------------------------------------------------------
# Tight-binding parameter sets (inputs, in eV and nm).
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class TBParams:
    """Slater-Koster sp parameters; V(r) = V0 * (r0 / r)**power for r <= r_cut.

    overlap = 0 gives S = I.  overlap = 1 gives off-diagonal overlap blocks
    s_amp * exp(-(r - r0) / s_decay) * I4 on the same bond pattern as H and
    identity diagonal blocks.
    """
    e_s: float = -8.0
    e_p: float = 0.0
    v_sss: float = -5.0
    v_sps: float = 5.5
    v_pps: float = 6.0
    v_ppp: float = -2.5
    r0: float = 0.14
    power: float = 2.0
    r_cut: float = 0.30
    overlap: int = 0
    s_amp: float = 0.1
    s_decay: float = 0.05


BUNDLE_TB = TBParams()
BUNDLE_TB_OVERLAP = dataclasses.replace(BUNDLE_TB, overlap=1)


# ---------------------------------------------------------------------------
# Geometry.
# ---------------------------------------------------------------------------

def bundle_xyz(n_grid_x: int, n_grid_y: int, atoms_per_chain: int, *, n_chains: Optional[int] = None,
               spacing: float = 0.45, dz: float = 0.14, sigma: float = 0.02,
               config_no: int = 2) -> np.ndarray:
    """Atom positions (n_atoms, 3) float64 in nm for a bundle of straight chains.

    Chains sit on the grid sites (ix * spacing, iy * spacing) in row-major order
    c = ix * n_grid_y + iy; only the first ``n_chains`` sites are used when it is
    given.  Atom k of chain c sits at z = k * dz, and its index is
    c * atoms_per_chain + k.  Every coordinate gets i.i.d. N(0, sigma^2) jitter.
    Open boundaries in x, y and z.
    """
    n_sites = n_grid_x * n_grid_y
    if n_chains is None:
        n_chains = n_sites
    if not 0 < n_chains <= n_sites:
        raise ValueError("n_chains must be in (0, n_grid_x * n_grid_y]")
    c = np.arange(n_chains)
    ix, iy = c // n_grid_y, c % n_grid_y
    k = np.arange(atoms_per_chain)
    xyz = np.empty((n_chains, atoms_per_chain, 3), dtype=np.float64)
    xyz[:, :, 0] = (ix * spacing)[:, None]
    xyz[:, :, 1] = (iy * spacing)[:, None]
    xyz[:, :, 2] = (k * dz)[None, :]
    xyz = xyz.reshape(-1, 3)
    if sigma > 0:
        xyz = xyz + rng(config_no, STREAM_GEOMETRY).normal(0.0, sigma, size=xyz.shape)
    return np.ascontiguousarray(xyz)


# ---------------------------------------------------------------------------
# Energies and quadrature weights.
# ---------------------------------------------------------------------------

def shift_grid(e_lo: float, e_hi: float, n_shifts: int, eta: float) -> np.ndarray:
    """z_k = E_k + i*eta with E_k uniform on [e_lo, e_hi], both ends included."""
    if n_shifts < 1:
        raise ValueError("n_shifts must be >= 1")
    e = np.linspace(e_lo, e_hi, n_shifts) if n_shifts > 1 else np.array([0.5 * (e_lo + e_hi)])
    return (e + 1j * eta).astype(np.complex128)


def occupied_weights(z: np.ndarray, mu: float = 0.0) -> np.ndarray:
    """Real-axis trapezoid weights: dE (half at the two ends of the grid) where
    Re z_k <= mu, else 0.  Returned as complex128 so that any contour can be
    substituted by the caller."""
    e = np.real(z)
    n = e.size
    if n == 1:
        wt = np.ones(1)
    else:
        de = (e[-1] - e[0]) / (n - 1)
        wt = np.full(n, de)
        wt[0] *= 0.5
        wt[-1] *= 0.5
    wt = np.where(e <= mu, wt, 0.0)
    return wt.astype(np.complex128)


# ---------------------------------------------------------------------------
# Workloads.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """Everything a solve needs except the Hamiltonian itself.

    kind:      "chain" (H given by on-site energies and a hopping) or "tb"
               (H built from xyz and tb).
    xyz:       (n_atoms, 3) nm, or None for the chain.
    onsite:    chain: (n_sites,) on-site energies; tb: None (parameters apply).
    hopping:   chain nearest-neighbour hopping.
    tb:        TBParams for kind "tb".
    columns:   int64 global orbital indices (column j lives on atom j // 4).
    z, w:      complex128 shifts and quadrature weights.
    radius:    scalar local-subspace radius in nm (<= 0: the whole system).
    radius_per_col: optional per-column radii (float64, same length as columns).
    tol:       relative residual tolerance.
    """
    name: str
    kind: str
    n_orb: int
    xyz: Optional[np.ndarray]
    onsite: Optional[np.ndarray]
    hopping: float
    tb: Optional[TBParams]
    columns: np.ndarray
    z: np.ndarray
    w: np.ndarray
    radius: float
    radius_per_col: Optional[np.ndarray]
    tol: float

    @property
    def n_atoms(self) -> int:
        return self.n_orb // 4

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.xyz, self.onsite, self.columns, self.z, self.w, self.radius_per_col):
            if a is not None:
                h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((self.name, self.kind, self.n_orb, self.hopping, self.tb, self.radius, self.tol)).encode())
        return h.hexdigest()


#: Energy window of the bundle workloads (eV).  It covers the bulk of the sp
#: bands of the bundle model at the 0.14 nm bond length; rare close pairs push
#: a few eigenvalues further out, and those only set iteration counts.
BUNDLE_WINDOW = (-30.0, 30.0)
ETA = 0.01


def chain_workload(n_sites: int = 2000, n_columns: int = 16, n_shifts: int = 64, *,
                   config_no: int = 1, e_window=(-3.0, 3.0), eta: float = ETA,
                   disorder: float = 0.5, hopping: float = -1.0, tol: float = 1e-10) -> Workload:
    """Plain-method chain: S = I, one orbital per site, on-site U[-disorder, disorder],
    nearest-neighbour hopping, open ends; columns drawn without replacement."""
    if n_sites % 4:
        raise ValueError("n_sites must be a multiple of 4 (sites are grouped four to a block)")
    g = rng(config_no, STREAM_GEOMETRY)
    onsite = g.uniform(-disorder, disorder, size=n_sites) if disorder > 0 else np.zeros(n_sites)
    cols = rng(config_no, STREAM_COLUMNS).choice(n_sites, size=min(n_columns, n_sites), replace=False)
    z = shift_grid(e_window[0], e_window[1], n_shifts, eta)
    return Workload(name=f"chain{n_sites}", kind="chain", n_orb=n_sites, xyz=None, onsite=onsite,
                    hopping=hopping, tb=None, columns=np.asarray(cols, dtype=np.int64), z=z,
                    w=occupied_weights(z, 0.0), radius=0.0, radius_per_col=None, tol=tol)


def bundle_workload(n_grid_x: int = 13, n_grid_y: int = 13, atoms_per_chain: int = 700, *,
                    n_chains: Optional[int] = None, n_shifts: int = 128, radius: float = 1.0,
                    overlap: bool = False, radius_range=None, columns: Optional[np.ndarray] = None,
                    n_columns: Optional[int] = None, config_no: int = 2, tol: float = 1e-12,
                    e_window=BUNDLE_WINDOW, eta: float = ETA) -> Workload:
    """Polymer-bundle-like sp tight binding (4 orbitals per atom).

    columns: explicit global orbital indices; otherwise ``n_columns`` drawn
    without replacement (stream 1), otherwise every orbital.
    radius_range: (lo, hi) draws a per-column radius U[lo, hi] (stream 2).
    tol defaults to 1e-12: a shift frozen at relative residual tol carries an
    error up to tol/eta in G, and the density matrix sums G over ~N_s/2 shifts
    near resonances, so a 1e-10 relative accuracy on every G_ij and rho_ij
    needs the tolerance two decades below it (measured against the dense
    restricted solve: rho error 2e-10 at tol 1e-11, 4e-11 at 1e-12).
    """
    xyz = bundle_xyz(n_grid_x, n_grid_y, atoms_per_chain, n_chains=n_chains, config_no=config_no)
    n_orb = 4 * xyz.shape[0]
    if columns is None:
        if n_columns is None or n_columns >= n_orb:
            columns = np.arange(n_orb, dtype=np.int64)
        else:
            columns = np.sort(rng(config_no, STREAM_COLUMNS).choice(n_orb, size=n_columns, replace=False))
    columns = np.asarray(columns, dtype=np.int64)
    rpc = None
    if radius_range is not None:
        rpc = rng(config_no, STREAM_RADII).uniform(radius_range[0], radius_range[1], size=n_orb)[columns]
    z = shift_grid(e_window[0], e_window[1], n_shifts, eta)
    tb = BUNDLE_TB_OVERLAP if overlap else BUNDLE_TB
    return Workload(name="bundle", kind="tb", n_orb=n_orb, xyz=xyz, onsite=None, hopping=0.0, tb=tb,
                    columns=columns, z=z, w=occupied_weights(z, 0.0), radius=radius,
                    radius_per_col=rpc, tol=tol)


# Named configurations -------------------------------------------------------

def config_chain(**kw) -> Workload:
    """2000-site chain, 64 shifts on [-3, 3] + 0.01i, 16 columns, tol 1e-10."""
    return chain_workload(**kw)


def config_bundle(**kw) -> Workload:
    """169 chains x 700 atoms (118,300 atoms, 473,200 orbitals), R = 1.0 nm, 128 shifts."""
    kw.setdefault("config_no", 2)
    return bundle_workload(13, 13, 700, **kw)


def config_bundle_overlap(**kw) -> Workload:
    """Bundle geometry with the overlap S, per-column radius U[0.6, 1.4] nm, 256 shifts."""
    kw.setdefault("config_no", 3)
    kw.setdefault("n_shifts", 256)
    kw.setdefault("radius_range", (0.6, 1.4))
    return bundle_workload(13, 13, 700, overlap=True, **kw)


def config_large(**kw) -> Workload:
    """1,429 chains x 700 atoms on a 38 x 38 grid (1,000,300 atoms), 256 shifts."""
    kw.setdefault("config_no", 5)
    kw.setdefault("n_shifts", 256)
    return bundle_workload(38, 38, 700, n_chains=1429, **kw)


# ---------------------------------------------------------------------------
# Initial weights of the iteration-count network (inputs of the training).
# ---------------------------------------------------------------------------

MLP_NF, MLP_NH = 5, 64
MLP_NPARAM = 2 * MLP_NF + MLP_NH * MLP_NF + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NH + 1


def breakdown_block():
    """A crafted one-atom input for the BREAKDOWN status: one 4x4 block with
    H_01 = -1 and H_10 = 1 (deliberately not symmetric), all other entries
    0, S = I, and the shifts -1 + i, i, 1 + i with the seed at index 1.
    Returns (row_ptr, col, h [1, 4, 4], z)."""
    h = np.zeros((1, 4, 4))
    h[0, 0, 1], h[0, 1, 0] = -1.0, 1.0
    return np.array([0, 1], np.int32), np.array([0], np.int32), h, np.array([-1 + 1j, 1j, 1 + 1j])


def mlp_init(seed: int = 0) -> np.ndarray:
    """He-normal weights and zero biases in the flat layout
    [mean(5), inv_std(5), W1(64x5), b1, W2(64x64), b2, W3(64), b3];
    normalisation is the identity until it is set from training data."""
    g = rng(4, seed)
    p = np.zeros(MLP_NPARAM)
    p[MLP_NF:2 * MLP_NF] = 1.0
    o = 2 * MLP_NF
    p[o:o + MLP_NH * MLP_NF] = g.normal(0, np.sqrt(2.0 / MLP_NF), MLP_NH * MLP_NF)
    o += MLP_NH * MLP_NF + MLP_NH
    p[o:o + MLP_NH * MLP_NH] = g.normal(0, np.sqrt(2.0 / MLP_NH), MLP_NH * MLP_NH)
    o += MLP_NH * MLP_NH + MLP_NH
    p[o:o + MLP_NH] = g.normal(0, np.sqrt(1.0 / MLP_NH), MLP_NH)
    return p



# ---------------------------------------------------------------------------
# Initial wavepackets of the time-propagation workload.
# ---------------------------------------------------------------------------

def wavepacket(wl: Workload, n_packets: int = 1, *, width: float = 0.5, k_z: float = 10.0,
               config_no: int = 6) -> np.ndarray:
    """Initial wavepackets [n_orb, n_packets] complex128, each of unit 2-norm.

    Packet p is centred on a seeded atom c_p.  Atom A within 4 * width of it
    (nm; for the chain, site distance in units of one site) carries
    exp(-|r_A - r_c|^2 / (4 width^2)) * exp(i k_z (z_A - z_c)) times a seeded
    unit vector of orbital weights (the same for every atom of the packet);
    all other entries are zero.
    """
    g = rng(config_no, STREAM_WAVEPACKET)
    n_atoms = wl.n_atoms
    if wl.xyz is None:  # chain: one orbital per site, sites on a line
        pos = np.zeros((wl.n_orb, 3))
        pos[:, 2] = np.arange(wl.n_orb, dtype=np.float64)
        per_site = True
    else:
        pos = wl.xyz
        per_site = False
    out = np.zeros((wl.n_orb, n_packets), np.complex128)
    n_centres = wl.n_orb if per_site else n_atoms
    for p in range(n_packets):
        c = int(g.integers(0, n_centres))
        u = g.normal(size=4)
        u /= np.linalg.norm(u)
        d = pos - pos[c]
        r2 = (d * d).sum(axis=1)
        near = r2 <= (4.0 * width) ** 2
        amp = np.where(near, np.exp(-r2 / (4.0 * width * width)) * np.exp(1j * k_z * d[:, 2]), 0.0)
        if per_site:
            out[:, p] = amp
        else:
            out[:, p] = (amp[:, None] * u[None, :]).ravel()
        out[:, p] /= np.linalg.norm(out[:, p])
    return out
