"""CPU oracle for the shifted-COCG Green's-function path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1603_09616_amd``); the two meet only in the
seeded input generators of ``workloads``.

Contents:
* ``sgfo.c`` (plain C, FP64, OpenMP over columns): tight-binding builder,
  local subspaces, projected and full-vector shifted COCG, density matrix.
* this module: ctypes binding, plus the dense definitions the iterative result
  must agree with (exact restricted solve, eigen-expansion).
* ``mlp.py``: FP64 reference of the iteration-count network.
* ``wp.py``: wavepacket time propagation (exact by eigen-decomposition, and
  the Chebyshev series), Gershgorin bounds.
* ``forces.py``: band-structure forces at fixed rho (Slater-Koster block
  gradient) and, with an overlap, the energy-density matrix and its term.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgfo.so")
SRC_PATH = os.path.join(_HERE, "sgfo.c")

CONVERGED, MAXITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                        "-o", tmp, SRC_PATH, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _TB(ctypes.Structure):
    _fields_ = [("e_s", ctypes.c_double), ("e_p", ctypes.c_double), ("v_sss", ctypes.c_double),
                ("v_sps", ctypes.c_double), ("v_pps", ctypes.c_double), ("v_ppp", ctypes.c_double),
                ("r0", ctypes.c_double), ("power", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("overlap", ctypes.c_int32), ("s_amp", ctypes.c_double), ("s_decay", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.sgfo_tb_nnzb.restype = i64
        L.sgfo_tb_nnzb.argtypes = [i64, P, dbl]
        L.sgfo_tb_build.restype = i64
        L.sgfo_tb_build.argtypes = [i64, P, P, ctypes.POINTER(_TB), i64, P, P, P, P]
        L.sgfo_chain_build.restype = i64
        L.sgfo_chain_build.argtypes = [i64, P, dbl, i64, P, P, P]
        L.sgfo_plan_sizes.restype = i32
        L.sgfo_plan_sizes.argtypes = [i64, P, P, P, i64, P, dbl, P, i32, P, P, i32]
        L.sgfo_shifted_solve.restype = i32
        L.sgfo_shifted_solve.argtypes = [i64, P, P, P, P, P, i64, P, dbl, P, i32, i32, P, P, dbl, i32, i32, i64,
                                         P, P, P, P, P, P, P, i32]
        L.sgfo_solve_full.restype = i32
        L.sgfo_solve_full.argtypes = [i64, P, P, P, P, P, i64, dbl, i32, i32, P, dbl, i32, i32, i64, P, P, P, P, P,
                                      P, P]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _tb(params) -> _TB:
    return _TB(params.e_s, params.e_p, params.v_sss, params.v_sps, params.v_pps, params.v_ppp, params.r0,
               params.power, params.r_cut, int(params.overlap), params.s_amp, params.s_decay)


@dataclasses.dataclass
class BSR:
    """Host block-sparse row matrix: 4x4 float64 blocks, one block row per atom."""
    row_ptr: np.ndarray   # int32 [n+1]
    col: np.ndarray       # int32 [nnzb]
    h: np.ndarray         # float64 [nnzb, 4, 4]
    s: Optional[np.ndarray] = None  # float64 [nnzb, 4, 4] or None (S = I)

    @property
    def n_atoms(self) -> int:
        return self.row_ptr.size - 1

    @property
    def nnzb(self) -> int:
        return self.col.size

    def dense(self, which: str = "h") -> np.ndarray:
        vals = self.h if which == "h" else self.s
        n = self.n_atoms
        M = np.zeros((4 * n, 4 * n))
        if vals is None:
            return np.eye(4 * n)
        for a in range(n):
            for t in range(self.row_ptr[a], self.row_ptr[a + 1]):
                b = self.col[t]
                M[4 * a:4 * a + 4, 4 * b:4 * b + 4] = vals[t]
        return M


def tb_build(xyz: np.ndarray, params, onsite: Optional[np.ndarray] = None) -> BSR:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    n = xyz.shape[0]
    L = lib()
    nnzb = L.sgfo_tb_nnzb(n, _p(xyz), params.r_cut)
    if nnzb < 0:
        raise ValueError(f"sgfo_tb_nnzb failed ({nnzb})")
    row_ptr = np.zeros(n + 1, np.int32)
    col = np.zeros(nnzb, np.int32)
    h = np.zeros((nnzb, 4, 4))
    s = np.zeros((nnzb, 4, 4)) if params.overlap else None
    tb = _tb(params)
    ons = None if onsite is None else np.ascontiguousarray(onsite, dtype=np.float64)
    got = L.sgfo_tb_build(n, _p(xyz), _p(ons), ctypes.byref(tb), nnzb, _p(row_ptr), _p(col), _p(h), _p(s))
    if got != nnzb:
        raise ValueError(f"sgfo_tb_build failed ({got})")
    return BSR(row_ptr, col, h, s)


def chain_build(eps: np.ndarray, t: float) -> BSR:
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    n = eps.size
    nb = n // 4
    cap = 3 * nb
    row_ptr = np.zeros(nb + 1, np.int32)
    col = np.zeros(cap, np.int32)
    h = np.zeros((cap, 4, 4))
    got = lib().sgfo_chain_build(n, _p(eps), float(t), cap, _p(row_ptr), _p(col), _p(h))
    if got < 0:
        raise ValueError(f"sgfo_chain_build failed ({got})")
    return BSR(row_ptr, col[:got].copy(), h[:got].copy(), None)


def system_for(wl) -> BSR:
    """Oracle-built Hamiltonian (and overlap) of a workload."""
    if wl.kind == "chain":
        return chain_build(wl.onsite, wl.hopping)
    return tb_build(wl.xyz, wl.tb)


@dataclasses.dataclass
class Result:
    proj_ptr: np.ndarray   # int64 [n_cols+1]
    proj_row: np.ndarray   # int32 [sum P] global orbital of each projection row
    G: np.ndarray          # complex128 [sum P, n_shifts]
    rho: np.ndarray        # float64 [sum P]
    iters: np.ndarray      # int32 [n_cols]
    status: np.ndarray     # int32 [n_cols]
    resid: np.ndarray      # float64 [n_cols, n_shifts]

    def column(self, c: int):
        a, b = self.proj_ptr[c], self.proj_ptr[c + 1]
        return self.proj_row[a:b], self.G[a:b], self.rho[a:b]

    def g_diag(self, cols: np.ndarray) -> np.ndarray:
        """G_jj(z_k) for each column j: [n_cols, n_shifts]."""
        out = np.empty((cols.size, self.G.shape[1]), np.complex128)
        for c, j in enumerate(cols):
            rows, G, _ = self.column(c)
            out[c] = G[int(np.nonzero(rows == j)[0][0])]
        return out


def _cplx(a: Optional[np.ndarray]) -> Optional[np.ndarray]:
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


def plan_sizes(bsr: BSR, xyz, cols, radius=0.0, radius_per_col=None, prune=False, threads=0):
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    xyz = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
    rpc = None if radius_per_col is None else np.ascontiguousarray(radius_per_col, dtype=np.float64)
    n_loc = np.zeros(cols.size, np.int64)
    n_proj = np.zeros(cols.size, np.int64)
    rc = lib().sgfo_plan_sizes(bsr.n_atoms, _p(bsr.row_ptr), _p(bsr.col), _p(xyz), cols.size, _p(cols),
                               float(radius), _p(rpc), int(prune), _p(n_loc), _p(n_proj), int(threads))
    if rc:
        raise ValueError(f"sgfo_plan_sizes failed ({rc})")
    return n_loc, n_proj


def shifted_solve(bsr: BSR, xyz, cols, z, w=None, tol=1e-10, radius=0.0, radius_per_col=None, prune=False,
                  max_iter=0, seed_index=-1, threads=0) -> Result:
    """Plain FP64 shifted COCG on every column (OpenMP over columns)."""
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    xyz = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
    rpc = None if radius_per_col is None else np.ascontiguousarray(radius_per_col, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    ns = z.size
    _, n_proj = plan_sizes(bsr, xyz, cols, radius, rpc, prune, threads)
    total = int(n_proj.sum())
    proj_ptr = np.zeros(cols.size + 1, np.int64)
    proj_row = np.zeros(max(total, 1), np.int32)
    G = np.zeros((max(total, 1), ns), np.complex128)
    rho = np.zeros(max(total, 1))
    iters = np.zeros(cols.size, np.int32)
    status = np.zeros(cols.size, np.int32)
    resid = np.zeros((cols.size, ns))
    zf, wf = _cplx(z), _cplx(w)
    rc = lib().sgfo_shifted_solve(bsr.n_atoms, _p(bsr.row_ptr), _p(bsr.col), _p(bsr.h), _p(bsr.s), _p(xyz),
                                  cols.size, _p(cols), float(radius), _p(rpc), int(prune), ns, _p(zf), _p(wf),
                                  float(tol), int(max_iter), int(seed_index), max(total, 1), _p(proj_ptr),
                                  _p(proj_row), _p(G.view(np.float64)), _p(rho), _p(iters), _p(status), _p(resid),
                                  int(threads))
    if rc:
        raise ValueError(f"sgfo_shifted_solve failed ({rc})")
    return Result(proj_ptr, proj_row[:total], G[:total], rho[:total], iters, status, resid)


@dataclasses.dataclass
class FullResult:
    loc_atoms: np.ndarray  # int32 [n_loc]
    x: np.ndarray          # complex128 [nl, n_shifts]
    s: np.ndarray          # complex128 [nl] final seed residual
    pi: np.ndarray         # complex128 [n_shifts] final pi^k
    resid: np.ndarray
    iters: int
    status: int


def solve_full(bsr: BSR, xyz, j: int, z, tol=1e-10, radius=0.0, prune=False, max_iter=0, seed_index=-1):
    """Full-vector shifted COCG for column j (keeps x^k on every local row)."""
    xyz_c = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
    n_loc, _ = plan_sizes(bsr, xyz_c, np.array([j]), radius, None, prune)
    nloc = int(n_loc[0])
    z = np.ascontiguousarray(z, dtype=np.complex128)
    ns = z.size
    loc = np.zeros(nloc, np.int32)
    x = np.zeros((4 * nloc, ns), np.complex128)
    s = np.zeros(4 * nloc, np.complex128)
    pi = np.zeros(ns, np.complex128)
    resid = np.zeros(ns)
    it = np.zeros(1, np.int32)
    st = np.zeros(1, np.int32)
    rc = lib().sgfo_solve_full(bsr.n_atoms, _p(bsr.row_ptr), _p(bsr.col), _p(bsr.h), _p(bsr.s), _p(xyz_c), int(j),
                               float(radius), int(prune), ns, _p(_cplx(z)), float(tol), int(max_iter),
                               int(seed_index), nloc, _p(loc), _p(x.view(np.float64)), _p(s.view(np.float64)),
                               _p(pi.view(np.float64)), _p(resid), _p(it), _p(st))
    if rc:
        raise ValueError(f"sgfo_solve_full failed ({rc})")
    return FullResult(loc, x, s, pi, resid, int(it[0]), int(st[0]))


def solve_workload(wl, bsr: Optional[BSR] = None, cols=None, prune=True, threads=0, **kw) -> Result:
    """Oracle solve of a workload (optionally on a subset of its columns)."""
    bsr = system_for(wl) if bsr is None else bsr
    if cols is None:
        cols = wl.columns
        rpc = wl.radius_per_col
    else:
        cols = np.asarray(cols, np.int64)
        rpc = None
        if wl.radius_per_col is not None:
            pos = {int(j): i for i, j in enumerate(wl.columns)}
            rpc = wl.radius_per_col[[pos[int(j)] for j in cols]]
    kw.setdefault("tol", wl.tol)
    return shifted_solve(bsr, wl.xyz, cols, wl.z, wl.w, radius=wl.radius, radius_per_col=rpc, prune=prune,
                         threads=threads, **kw)


# ---------------------------------------------------------------------------
# Dense definitions (for pins): the exact restricted solve and the spectrum.
# ---------------------------------------------------------------------------

def local_dense(bsr: BSR, loc_atoms: np.ndarray):
    """Dense principal submatrices H_L, S_L on the orbitals of loc_atoms (sorted)."""
    loc = np.asarray(loc_atoms, np.int64)
    where = {int(a): i for i, a in enumerate(loc)}
    n = 4 * loc.size
    H = np.zeros((n, n))
    S = np.eye(n) if bsr.s is None else np.zeros((n, n))
    for A, a in enumerate(loc):
        for t in range(bsr.row_ptr[a], bsr.row_ptr[a + 1]):
            B = where.get(int(bsr.col[t]))
            if B is None:
                continue
            H[4 * A:4 * A + 4, 4 * B:4 * B + 4] = bsr.h[t]
            if bsr.s is not None:
                S[4 * A:4 * A + 4, 4 * B:4 * B + 4] = bsr.s[t]
    idx = (4 * loc[:, None] + np.arange(4)[None, :]).ravel()
    return H, S, idx


def apply(bsr: BSR, z: complex, x: np.ndarray, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """(z S - H) x over the whole system (the operator of the shifted
    equations in the Introduction), for x of shape [n_orb] or [n_orb, k].
    With ``rows``, only those orbital rows of the result, each summed
    directly over its block row."""
    if rows is None:
        import scipy.sparse as sp
        n = 4 * bsr.n_atoms
        Hm = sp.bsr_matrix((bsr.h, bsr.col, bsr.row_ptr), shape=(n, n))
        Sx = x if bsr.s is None else sp.bsr_matrix((bsr.s, bsr.col, bsr.row_ptr), shape=(n, n)) @ x
        return z * Sx - Hm @ x
    out = []
    for i in np.asarray(rows):
        a, o = int(i) // 4, int(i) % 4
        acc_h = 0.0
        acc_s = 0.0 if bsr.s is not None else x[i]
        for t in range(bsr.row_ptr[a], bsr.row_ptr[a + 1]):
            xb = x[4 * int(bsr.col[t]):4 * int(bsr.col[t]) + 4]
            acc_h = acc_h + bsr.h[t][o] @ xb
            if bsr.s is not None:
                acc_s = acc_s + bsr.s[t][o] @ xb
        out.append(z * acc_s - acc_h)
    return np.array(out)


def exact_columns(H: np.ndarray, S: np.ndarray, jl: int, z: np.ndarray) -> np.ndarray:
    """x^k = (z_k S - H)^{-1} e_jl for every shift: [n, n_shifts] (dense LU)."""
    n = H.shape[0]
    e = np.zeros(n, np.complex128)
    e[jl] = 1.0
    return np.stack([np.linalg.solve(zk * S - H, e) for zk in z], axis=1)


# ---------------------------------------------------------------------------
# After rho: traces, electron count, band energy, Fermi level.
# ---------------------------------------------------------------------------

def _block_entry(bsr: BSR, m: np.ndarray, i: int, j: int) -> float:
    """Entry (i, j) of the block matrix with blocks m (bsr.h or bsr.s)."""
    a, b = i // 4, j // 4
    for t in range(int(bsr.row_ptr[a]), int(bsr.row_ptr[a + 1])):
        if int(bsr.col[t]) == b:
            return float(m[t, i % 4, j % 4])
    return 0.0


def traces(bsr: BSR, res: Result, cols):
    """Per-shift traces over the solved columns from the projected G.

    Row j of the restricted equations (z S_L - H_L) x = e_j involves only the
    orbitals that share a stored block with j, i.e. the projection rows P(j),
    so  T_k = sum_j sum_{i in P(j)} S_ji G_ij(z_k)  and
        U_k = sum_j sum_{i in P(j)} H_ji G_ij(z_k).
    Returns (T, U), complex128 [n_shifts]."""
    cols = np.asarray(cols, np.int64)
    ns = res.G.shape[1]
    T = np.zeros(ns, np.complex128)
    U = np.zeros(ns, np.complex128)
    for c, j in enumerate(cols):
        rows, G, _ = res.column(c)
        for r, i in enumerate(rows):
            sji = (1.0 if int(i) == int(j) else 0.0) if bsr.s is None else _block_entry(bsr, bsr.s, int(j), int(i))
            hji = _block_entry(bsr, bsr.h, int(j), int(i))
            T += sji * G[r]
            U += hji * G[r]
    return T, U


def rho_traces(bsr: BSR, res: Result, cols):
    """(tr(rho S), tr(rho H)) over the solved columns from the projected rho."""
    cols = np.asarray(cols, np.int64)
    ts = th = 0.0
    for c, j in enumerate(cols):
        rows, _, rho = res.column(c)
        for r, i in enumerate(rows):
            sji = (1.0 if int(i) == int(j) else 0.0) if bsr.s is None else _block_entry(bsr, bsr.s, int(j), int(i))
            ts += sji * rho[r]
            th += _block_entry(bsr, bsr.h, int(j), int(i)) * rho[r]
    return ts, th


def occupation(T, U, w):
    """Electron count and band energy for weights w:
    -(1/pi) sum_k Im(w_k T_k), -(1/pi) sum_k Im(w_k U_k)."""
    T, U, w = (np.asarray(a, np.complex128) for a in (T, U, w))
    return float(-np.sum((w * T).imag) / np.pi), float(-np.sum((w * U).imag) / np.pi)


def fermi_level(z, T, U, n_target):
    """Scan of the real-axis grid: the first E_m at which the electron count
    with trapezoid weights (the spacing, halved at the two grid ends) on
    E_k <= E_m reaches n_target.  Returns (mu, n_e, e_band); raises when the
    whole grid holds fewer electrons."""
    e = np.real(np.asarray(z, np.complex128))
    n = e.size
    w = np.full(n, (e[-1] - e[0]) / (n - 1) if n > 1 else 1.0)
    if n > 1:
        w[0] *= 0.5
        w[-1] *= 0.5
    T, U = np.asarray(T, np.complex128), np.asarray(U, np.complex128)
    ne = eb = 0.0
    for m in range(n):
        ne += -w[m] * T[m].imag / np.pi
        eb += -w[m] * U[m].imag / np.pi
        if ne >= n_target:
            return float(e[m]), float(ne), float(eb)
    raise ValueError("target exceeds the occupation of the whole grid")
