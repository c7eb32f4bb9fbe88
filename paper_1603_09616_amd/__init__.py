"""Python binding of the gfx950 shifted-COCG Green's-function library.

Argument marshalling only: every step of the path (neighbour search,
Hamiltonian assembly, local subspaces, the shifted solve) runs in the HIP
kernels of ``libsgf.so`` behind the C ABI declared in ``include/sgf.h``.
PyTorch supplies device memory and the stream.  Importing this module does
not load the library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgf.so")

SGF_OK, SGF_EINVAL, SGF_ENOMEM, SGF_EHIP, SGF_EUNSUPPORTED = 0, -1, -2, -3, -4
CONVERGED, MAXITER, BREAKDOWN, NONFINITE, DRIFT, BADCOLUMN, DIAG_ONLY = 0, 1, 2, 3, 4, 5, 6

EXPORTED = (
    "sgf_last_error", "sgf_version", "sgf_build_workspace", "sgf_build_pattern", "sgf_build_hamiltonian",
    "sgf_build_chain", "sgf_to_f32", "sgf_plan_workspace", "sgf_plan_count", "sgf_plan_build", "sgf_proj_layout",
    "sgf_proj_rows", "sgf_solve_workspace", "sgf_shifted_solve", "sgf_solve_profile", "sgf_features", "sgf_mlp_normalize",
    "sgf_mlp_forward", "sgf_mlp_train_step", "sgf_mlp_gradient", "sgf_order_workspace", "sgf_order_by_prediction",
    "sgf_bsr_apply", "sgf_solve_stage_shifts", "sgf_trace_workspace", "sgf_traces", "sgf_occupation",
    "sgf_fermi_level", "sgf_wp_workspace", "sgf_wp_bounds", "sgf_wp_terms", "sgf_wp_propagate",
    "sgf_band_forces", "sgf_energy_density", "sgf_shifted_solve_static", "sgf_hamiltonian_size",
    "sgf_system_from_bsr", "sgf_system_destroy", "sgf_md_kick", "sgf_md_drift", "sgf_fermi_shifts",
    "sgf_order_groups_workspace", "sgf_order_groups_by_prediction",
)
MLP_NFEAT, MLP_NPARAM, MLP_BATCH, MLP_NH = 5, 4619, 128, 64
STATIC_SCRATCH_BYTES = 256 << 20   # SGF_STATIC_SCRATCH_BYTES
ACCEL_EV_NM_AMU = 9.648533215665326e-5   # SGF_ACCEL_EV_NM_AMU: nm/fs^2 per eV/nm per amu


class SgfError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


# --- C structures (mirror include/sgf.h) --------------------------------------
P = ctypes.c_void_p
i32, i64, dbl, szt = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class TBParamsC(ctypes.Structure):
    _fields_ = [("e_s", dbl), ("e_p", dbl), ("v_sss", dbl), ("v_sps", dbl), ("v_pps", dbl), ("v_ppp", dbl),
                ("r0", dbl), ("power", dbl), ("r_cut", dbl), ("overlap", i32), ("s_amp", dbl), ("s_decay", dbl)]


class SystemC(ctypes.Structure):
    _fields_ = [("n_atoms", i64), ("nnzb", i64), ("row_ptr", P), ("col", P), ("h", P), ("s", P), ("h32", P),
                ("s32", P), ("xyz", P), ("s_orbital_diagonal", i32)]


class PlanC(ctypes.Structure):
    _fields_ = [("n_plans", i64), ("center", P), ("radius", P), ("prune", i32), ("atom_off", P), ("blk_off", P),
                ("pa_off", P), ("loc_atom", P), ("lrow", P), ("lblk", P), ("pa_loc", P), ("center_loc", P)]


class PlanTotalsC(ctypes.Structure):
    _fields_ = [("n_loc_atoms", i64), ("n_loc_blocks", i64), ("n_proj_atoms", i64), ("max_loc_atoms", i32),
                ("max_loc_blocks", i32), ("max_proj_atoms", i32), ("max_row_blocks", i32)]


class SolveOptsC(ctypes.Structure):
    _fields_ = [("precision", i32), ("tol", dbl), ("max_iter", i32), ("seed_index", i32), ("monitor_every", i32),
                ("stage_lds", i32), ("grid", i32), ("profile", i32), ("batch_cols", i64),
                ("shifts_per_lane", i32), ("shifts_staged", i32), ("drift_tol", dbl), ("g_tol", dbl),
                ("queue_len", i64), ("eps_out", P), ("g_diag_out", P)]


class BsrC(ctypes.Structure):
    _fields_ = [("n_atoms", i64), ("nnzb", i64), ("row_ptr", P), ("col", P), ("h", P), ("s", P), ("h32", P),
                ("s32", P), ("s_orbital_diagonal", i32)]


_lib = None


def lib():
    """Load libsgf.so (built by ``paper_1603_09616_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1603_09616_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        L.sgf_last_error.restype = ctypes.c_char_p
        L.sgf_version.restype = ctypes.c_int
        sigs = {
            "sgf_build_workspace": [i64, P],
            "sgf_build_pattern": [i64, P, dbl, P, szt, P, P, P],
            "sgf_build_hamiltonian": [i64, P, P, P, P, szt, P, i64, P, P, P, P],
            "sgf_build_chain": [i64, P, dbl, P, P, P, P],
            "sgf_solve_stage_shifts": [i32, P, P, P, szt, P],
            "sgf_bsr_apply": [P, i32, i32, P, P, P, P],
            "sgf_to_f32": [P, i64, P, P],
            "sgf_plan_workspace": [P, i64, i32, P],
            "sgf_plan_count": [P, P, i32, P, szt, P, szt, P, P],
            "sgf_plan_build": [P, P, i32, P, szt, P, szt, P],
            "sgf_proj_layout": [P, i64, P, P, P, P, P, P],
            "sgf_proj_rows": [P, i64, P, P, P, P],
            "sgf_solve_workspace": [P, P, i64, i32, P, P],
            "sgf_shifted_solve": [P, P, P, i64, P, P, P, i32, P, P, P, P, szt, P, P, P, P, P, P, P, P],
            "sgf_shifted_solve_static": [P, P, P, i64, P, P, P, i32, P, P, P, P, P, P, P, P, P, P, P],
            "sgf_solve_profile": [P, P, P],
            "sgf_features": [P, P, i64, P, P, P, P],
            "sgf_mlp_normalize": [P, P, i64, P],
            "sgf_mlp_forward": [P, P, i64, P, P],
            "sgf_mlp_train_step": [P, P, P, i32, ctypes.c_float, P, P, i32, P, P],
            "sgf_mlp_gradient": [P, P, P, i32, P, P, P],
            "sgf_order_workspace": [P],
            "sgf_order_by_prediction": [P, i64, ctypes.c_float, ctypes.c_float, P, P, szt, P],
            "sgf_trace_workspace": [i64, i32, P],
            "sgf_traces": [P, i64, P, P, P, P, i64, P, P, i32, P, szt, P, P, P, P],
            "sgf_occupation": [i32, P, P, P, P, P],
            "sgf_fermi_level": [i32, P, P, P, dbl, P, P, P],
            "sgf_wp_workspace": [i64, i32, P],
            "sgf_wp_bounds": [P, P, szt, P, P, P],
            "sgf_wp_terms": [dbl, dbl, P],
            "sgf_wp_propagate": [P, i32, P, dbl, i32, dbl, dbl, i32, P, szt, P],
            "sgf_band_forces": [P, P, P, i64, P, P, P, P, P, P, P, P],
            "sgf_energy_density": [i64, i32, P, P, P, P, P],
            "sgf_hamiltonian_size": [i64, P, P, P, szt, P, P],
            "sgf_system_from_bsr": [P, P, P],
            "sgf_md_kick": [i64, P, P, dbl, P, P],
            "sgf_md_drift": [i64, P, dbl, P, P],
            "sgf_fermi_shifts": [i32, dbl, dbl, dbl, P, P],
            "sgf_order_groups_workspace": [i64, P],
            "sgf_order_groups_by_prediction": [P, i64, P, i64, ctypes.c_float, ctypes.c_float, P, P, szt, P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        L.sgf_system_destroy.restype = None
        L.sgf_system_destroy.argtypes = [P]
        _lib = L
    return _lib


def _check(fn: str, code: int):
    if code != SGF_OK:
        raise SgfError(fn, code, lib().sgf_last_error().decode())


def _call(name: str, *args):
    _check(name, getattr(lib(), name)(*args))


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(a, dtype, device="cuda"):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _bytes(n: int, device="cuda"):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


# --- system -----------------------------------------------------------------

@dataclasses.dataclass
class System:
    """Device-resident block-sparse H (and S), with the spatial hash of its atoms."""
    n_atoms: int
    nnzb: int
    row_ptr: "object"
    col: "object"
    h: "object"
    s: "object" = None
    h32: "object" = None
    s32: "object" = None
    xyz: "object" = None
    build_ws: "object" = None
    s_orbital_diagonal: bool = False  # every block of s is a multiple of I4

    def c(self) -> SystemC:
        return SystemC(self.n_atoms, self.nnzb, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.h), _ptr(self.s),
                       _ptr(self.h32), _ptr(self.s32), _ptr(self.xyz),
                       int(bool(self.s_orbital_diagonal) and self.s is not None))

    def add_f32(self, stream=None) -> "System":
        """FP32 shadows of H (and S) for the mixed-precision path."""
        torch = _torch()
        self.h32 = torch.empty(self.h.shape, dtype=torch.float32, device=self.h.device)
        _call("sgf_to_f32", _ptr(self.h), self.h.numel(), _ptr(self.h32), _stream(stream))
        if self.s is not None:
            self.s32 = torch.empty(self.s.shape, dtype=torch.float32, device=self.s.device)
            _call("sgf_to_f32", _ptr(self.s), self.s.numel(), _ptr(self.s32), _stream(stream))
        return self


def _tb_c(p) -> TBParamsC:
    return TBParamsC(p.e_s, p.e_p, p.v_sss, p.v_sps, p.v_pps, p.v_ppp, p.r0, p.power, p.r_cut, int(p.overlap),
                     p.s_amp, p.s_decay)


def build_hamiltonian(xyz, params, onsite=None, device="cuda", stream=None) -> System:
    """Neighbour search and Slater-Koster assembly of H (and S) on the GPU."""
    torch = _torch()
    d_xyz = _dev(xyz, torch.float64, device)
    n = d_xyz.shape[0]
    ws = ctypes.c_size_t()
    _call("sgf_build_workspace", n, ctypes.byref(ws))
    d_ws = _bytes(ws.value, device)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=device)
    nnzb = ctypes.c_int64()
    st = _stream(stream)
    _call("sgf_build_pattern", n, _ptr(d_xyz), float(params.r_cut), _ptr(d_ws), ws.value, _ptr(row_ptr),
          ctypes.byref(nnzb), st)
    nb = nnzb.value
    col = torch.empty(nb, dtype=torch.int32, device=device)
    h = torch.empty((nb, 4, 4), dtype=torch.float64, device=device)
    s = torch.empty((nb, 4, 4), dtype=torch.float64, device=device) if params.overlap else None
    d_on = None if onsite is None else _dev(onsite, torch.float64, device)
    tb = _tb_c(params)
    _call("sgf_build_hamiltonian", n, _ptr(d_xyz), _ptr(d_on), ctypes.byref(tb), _ptr(d_ws), ws.value,
          _ptr(row_ptr), nb, _ptr(col), _ptr(h), _ptr(s), st)
    # the builder's overlap blocks are s(r) I4 exactly
    return System(n, nb, row_ptr, col, h, s, xyz=d_xyz, build_ws=d_ws, s_orbital_diagonal=bool(params.overlap))


def build_chain(eps, t: float, device="cuda", stream=None) -> System:
    """One-orbital chain (four sites per 4x4 block), S = I."""
    torch = _torch()
    d_eps = _dev(eps, torch.float64, device)
    n_sites = d_eps.numel()
    nb = n_sites // 4
    nnzb = 1 if nb == 1 else 3 * nb - 2
    row_ptr = torch.empty(nb + 1, dtype=torch.int32, device=device)
    col = torch.empty(nnzb, dtype=torch.int32, device=device)
    h = torch.empty((nnzb, 4, 4), dtype=torch.float64, device=device)
    _call("sgf_build_chain", n_sites, _ptr(d_eps), float(t), _ptr(row_ptr), _ptr(col), _ptr(h), _stream(stream))
    return System(nb, nnzb, row_ptr, col, h)


def hamiltonian_size(xyz, params, device="cuda", stream=None) -> int:
    """Block count of the Hamiltonian build_hamiltonian would build (bonds
    within params.r_cut plus the diagonal blocks), from a GPU neighbour
    search."""
    torch = _torch()
    d_xyz = _dev(xyz, torch.float64, device)
    n = d_xyz.shape[0]
    ws = ctypes.c_size_t()
    _call("sgf_build_workspace", n, ctypes.byref(ws))
    d_ws = _bytes(ws.value, device)
    nnzb = ctypes.c_int64()
    tb = _tb_c(params)
    _call("sgf_hamiltonian_size", n, _ptr(d_xyz), ctypes.byref(tb), _ptr(d_ws), ws.value, ctypes.byref(nnzb),
          _stream(stream))
    return nnzb.value


def system_from_bsr(row_ptr, col, h, s=None, xyz=None, h32=None, s32=None, hash_cell=0.3, s_orbital_diagonal=False,
                    stream=None) -> System:
    """A System around a caller's block-sparse matrix (device tensors:
    row_ptr int32 [n+1], col int32 [nnzb], h (and s) float64 [nnzb, 4, 4];
    xyz float64 [n, 3] in nm for radius-limited subspaces).  The C call
    checks the sizes; the tensors are borrowed, not copied.  With xyz, the
    spatial hash that finds the atoms of a local subspace is built by the
    library's neighbour search (sgf_hamiltonian_size with cells of
    hash_cell nm).  s_orbital_diagonal: the caller states that every block
    of s is a multiple of I4 (the solve then inverts the overlap per atom
    pair; a column whose blocks are not of that form ends BADCOLUMN)."""
    n, nb = int(row_ptr.numel()) - 1, int(col.numel())
    m = BsrC(n, nb, _ptr(row_ptr), _ptr(col), _ptr(h), _ptr(s), _ptr(h32), _ptr(s32),
             int(bool(s_orbital_diagonal) and s is not None))
    out = ctypes.c_void_p()
    _call("sgf_system_from_bsr", ctypes.byref(m), _ptr(xyz), ctypes.byref(out))
    try:
        c = SystemC.from_address(out.value)
        assert c.n_atoms == n and c.nnzb == nb and c.row_ptr == _ptr(row_ptr) and c.h == _ptr(h)
        assert c.s_orbital_diagonal == m.s_orbital_diagonal
    finally:
        lib().sgf_system_destroy(out)
    build_ws = None
    if xyz is not None:
        ws = ctypes.c_size_t()
        _call("sgf_build_workspace", n, ctypes.byref(ws))
        build_ws = _bytes(ws.value, row_ptr.device)
        cnt = ctypes.c_int64()
        tb = TBParamsC(0, 0, 0, 0, 0, 0, 1.0, 0.0, float(hash_cell), 0, 0.0, 1.0)
        _call("sgf_hamiltonian_size", n, _ptr(xyz), ctypes.byref(tb), _ptr(build_ws), ws.value, ctypes.byref(cnt),
              _stream(stream))
    return System(n, nb, row_ptr, col, h, s, h32, s32, xyz, build_ws, bool(s_orbital_diagonal) and s is not None)


def system_for(wl, device="cuda") -> System:
    """GPU-built system of a workload from ``workloads``."""
    if wl.kind == "chain":
        return build_chain(wl.onsite, wl.hopping, device)
    return build_hamiltonian(wl.xyz, wl.tb, device=device)


# --- plans --------------------------------------------------------------------

@dataclasses.dataclass
class Plan:
    n_plans: int
    center: "object"
    radius: "object"
    prune: int
    atom_off: "object"
    blk_off: "object"
    pa_off: "object"
    loc_atom: "object"
    lrow: "object"
    lblk: "object"
    pa_loc: "object"
    center_loc: "object"
    totals: PlanTotalsC

    def c(self) -> PlanC:
        return PlanC(self.n_plans, _ptr(self.center), _ptr(self.radius), int(self.prune), _ptr(self.atom_off),
                     _ptr(self.blk_off), _ptr(self.pa_off), _ptr(self.loc_atom), _ptr(self.lrow), _ptr(self.lblk),
                     _ptr(self.pa_loc), _ptr(self.center_loc))


def make_plan(system: System, centers, radii, prune: bool = True, max_loc_atoms: int = 2048, stream=None) -> Plan:
    """Local subspaces (ball of each radius around each centre atom)."""
    torch = _torch()
    dev = system.row_ptr.device
    center = _dev(centers if isinstance(centers, torch.Tensor) else np.asarray(centers, np.int32), torch.int32, dev)
    radius = _dev(radii if isinstance(radii, torch.Tensor) else np.asarray(radii, np.float64), torch.float64, dev)
    n = center.numel()
    off = [torch.zeros(n + 1, dtype=torch.int64, device=dev) for _ in range(3)]
    ws = ctypes.c_size_t()
    sc = system.c()
    _call("sgf_plan_workspace", ctypes.byref(sc), n, int(max_loc_atoms), ctypes.byref(ws))
    d_ws = _bytes(ws.value, dev)
    plan = Plan(n, center, radius, int(prune), off[0], off[1], off[2], None, None, None, None, None,
                PlanTotalsC())
    pc = plan.c()
    bws = system.build_ws
    bws_bytes = 0 if bws is None else bws.numel()
    st = _stream(stream)
    _call("sgf_plan_count", ctypes.byref(sc), ctypes.byref(pc), int(max_loc_atoms), _ptr(bws), bws_bytes,
          _ptr(d_ws), ws.value, ctypes.byref(plan.totals), st)
    t = plan.totals
    plan.loc_atom = torch.empty(max(t.n_loc_atoms, 1), dtype=torch.int32, device=dev)
    plan.lrow = torch.empty(max(t.n_loc_atoms, 1), dtype=torch.int32, device=dev)
    plan.lblk = torch.empty(max(2 * t.n_loc_blocks, 1), dtype=torch.int32, device=dev)
    plan.pa_loc = torch.empty(max(t.n_proj_atoms, 1), dtype=torch.int32, device=dev)
    plan.center_loc = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    pc = plan.c()
    # the fill's LDS is sized from the largest counted subspace
    _call("sgf_plan_build", ctypes.byref(sc), ctypes.byref(pc), max(int(t.max_loc_atoms), 1), _ptr(bws), bws_bytes,
          _ptr(d_ws), ws.value, st)
    return plan


def plan_columns(columns, radius=0.0, radius_per_col=None):
    """Group columns by (atom, radius): returns (centers, radii, col_plan)."""
    cols = np.asarray(columns, np.int64)
    atoms = cols // 4
    rad = np.full(cols.size, float(radius)) if radius_per_col is None else np.asarray(radius_per_col, np.float64)
    keys = np.stack([atoms.astype(np.float64), rad], axis=1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    return uniq[:, 0].astype(np.int32), uniq[:, 1].copy(), inv.reshape(-1).astype(np.int32)


# --- solve --------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    proj_off: "object"   # int64 [n_cols+1]
    proj_row: "object"   # int32 [rows]
    G: "object"          # complex128 [rows, n_shifts] or None
    rho: "object"        # float64 [rows]
    iters: "object"      # int32 [n_cols]
    status: "object"     # int32 [n_cols]
    resid: "object"      # float64 [n_cols, n_shifts] or None

    def numpy(self):
        cv = (lambda t: t.cpu().numpy() if hasattr(t, "cpu") else t)
        r = Result(*(cv(getattr(self, f.name)) for f in dataclasses.fields(self)))
        for extra in ("n_fallback", "shift_iters", "G_diag", "eps"):
            if hasattr(self, extra):
                setattr(r, extra, cv(getattr(self, extra)))
        return r

    def column(self, c: int):
        a, b = int(self.proj_off[c]), int(self.proj_off[c + 1])
        return self.proj_row[a:b], (None if self.G is None else self.G[a:b]), self.rho[a:b]


@dataclasses.dataclass
class Prepared:
    """Everything a repeated solve reuses: plan, column map, output layout, workspace."""
    system: System
    plan: Plan
    cols: "object"
    col_plan: "object"
    proj_off: "object"
    proj_row: "object"
    n_rows: int


def prepare(system: System, columns, radius=0.0, radius_per_col=None, prune=True, max_loc_atoms=2048,
            stream=None) -> Prepared:
    """Plans (one per distinct atom and radius) and the output layout of the columns."""
    torch = _torch()
    dev = system.row_ptr.device
    centers, radii, col_plan = plan_columns(columns, radius, radius_per_col)
    return prepare_planned(system, _dev(np.asarray(columns, np.int64), torch.int64, dev),
                           _dev(col_plan, torch.int32, dev), _dev(centers, torch.int32, dev),
                           _dev(radii, torch.float64, dev), prune, max_loc_atoms, stream)


def prepare_planned(system: System, d_cols, d_col_plan, d_centers, d_radii, prune=True, max_loc_atoms=2048,
                    stream=None) -> Prepared:
    """Same as prepare() for inputs already on the device: columns, their plan
    index, and the centre atom and radius of every plan."""
    torch = _torch()
    dev = system.row_ptr.device
    plan = make_plan(system, d_centers, d_radii, prune, max_loc_atoms, stream)
    n = d_cols.numel()
    proj_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    total = ctypes.c_int64()
    pc = plan.c()
    _call("sgf_proj_layout", ctypes.byref(pc), n, _ptr(d_cols), _ptr(d_col_plan), _ptr(proj_off), None,
          ctypes.byref(total), _stream(stream))
    proj_row = torch.empty(max(total.value, 1), dtype=torch.int32, device=dev)
    _call("sgf_proj_rows", ctypes.byref(pc), n, _ptr(d_col_plan), _ptr(proj_off), _ptr(proj_row), _stream(stream))
    return Prepared(system, plan, d_cols, d_col_plan, proj_off, proj_row[:total.value], total.value)


def _cplx_host(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, np.complex128)).view(np.float64)


def solve_prepared(prep: Prepared, z, w=None, tol=1e-10, precision="fp64", max_iter=0, seed_index=-1,
                   g_out=True, order=None, batch_cols=0, stage_lds=-1, grid=0, monitor_every=50, out=None,
                   profile=False, shift_iters=False, shifts_per_lane=0, drift_tol=0.0, g_tol=0.0, queue_len=0,
                   fallback=True, fallback_tol=1e-9, shifts_staged=False, eps_out=False, stream=None) -> Result:
    """Shifted COCG on every prepared column (asynchronous on the stream).

    g_out: True or "proj" keeps G on every projection row (``Result.G``);
    "diag" keeps only the diagonal element G_jj(z_k) of every column
    (``Result.G_diag``, complex [n_cols, n_shifts]; ``Result.G`` is None);
    False or "none" keeps neither (rho only).  "proj" also fills G_diag when
    ``out`` holds a "G_diag" buffer.

    eps_out: also form the energy-density matrix on the projection rows in
    the shift pass (``Result.eps``; FP64 only, needs w).

    precision "mixed" builds the FP32 shadow of H first if the system has
    none; with ``fallback`` the columns the mixed path does not accept
    (DRIFT, MAXITER, ...) are then re-solved in FP64 at ``fallback_tol`` into
    the same outputs (this reads the status array, so it synchronises the
    stream); ``Result.n_fallback`` counts them."""
    torch = _torch()
    dev = prep.cols.device
    n = prep.cols.numel()
    zh = _cplx_host(z)
    wh = _cplx_host(w)
    ns = zh.size // 2
    if precision == "mixed" and prep.system.h32 is None:
        prep.system.add_f32(stream)
    if g_out not in (True, False, "proj", "diag", "none"):
        raise ValueError(f"g_out must be True/'proj', 'diag' or False/'none', not {g_out!r}")
    keep_g = g_out is True or g_out == "proj"
    opts = SolveOptsC({"fp64": 0, "mixed": 1}[precision], float(tol), int(max_iter), int(seed_index),
                      int(monitor_every), int(stage_lds), int(grid), int(bool(profile)), int(batch_cols),
                      int(shifts_per_lane), int(bool(shifts_staged)), float(drift_tol), float(g_tol), int(queue_len))
    sc = prep.system.c()
    pc = prep.plan.c()
    ws = ctypes.c_size_t()
    _call("sgf_solve_workspace", ctypes.byref(sc), ctypes.byref(prep.plan.totals), n, ns, ctypes.byref(opts),
          ctypes.byref(ws))
    if out is None:
        out = {
            "ws": _bytes(ws.value, dev),
            "G": torch.empty((max(prep.n_rows, 1), ns), dtype=torch.complex128, device=dev) if keep_g else None,
            "rho": torch.empty(max(prep.n_rows, 1), dtype=torch.float64, device=dev),
            "iters": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            "status": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            "resid": torch.empty((max(n, 1), ns), dtype=torch.float64, device=dev),
            "nk": torch.empty((max(n, 1), ns), dtype=torch.int32, device=dev) if shift_iters else None,
            "G_diag": (torch.empty((max(n, 1), ns), dtype=torch.complex128, device=dev) if g_out == "diag"
                       else None),
        }
    opts.g_diag_out = _ptr(out.get("G_diag"))
    if eps_out and out.get("eps") is None:
        out["eps"] = torch.empty(max(prep.n_rows, 1), dtype=torch.float64, device=dev)
    if eps_out:
        opts.eps_out = _ptr(out["eps"])
    d_order = None if order is None else _dev(order, torch.int32, dev)
    out["order"] = d_order
    _call("sgf_shifted_solve", ctypes.byref(sc), ctypes.byref(pc), ctypes.byref(prep.plan.totals), n,
          _ptr(prep.cols), _ptr(prep.col_plan), _ptr(d_order), ns, zh.ctypes.data_as(P),
          None if wh is None else wh.ctypes.data_as(P), ctypes.byref(opts), _ptr(out["ws"]), out["ws"].numel(),
          _ptr(prep.proj_off), _ptr(out["G"]), _ptr(out["rho"]), _ptr(out["iters"]), _ptr(out["status"]),
          _ptr(out["resid"]), _ptr(out.get("nk")), _stream(stream))
    n_fallback = 0
    if precision == "mixed" and fallback and n > 0 and queue_len == 0:
        torch.cuda.current_stream(dev).synchronize() if stream is None else stream.synchronize()
        st_now = out["status"][:n]
        bad = torch.nonzero((st_now != CONVERGED) & (st_now != DIAG_ONLY)).flatten().to(torch.int32)
        n_fallback = int(bad.numel())
        if n_fallback:
            out["fallback_order"] = bad
            opts64 = SolveOptsC(0, float(fallback_tol), 0, int(seed_index), 0, -1, int(grid), 0, 0,
                                int(shifts_per_lane), 0, 0.0, 0.0, n_fallback)
            opts64.g_diag_out = opts.g_diag_out
            _call("sgf_shifted_solve", ctypes.byref(sc), ctypes.byref(pc), ctypes.byref(prep.plan.totals), n,
                  _ptr(prep.cols), _ptr(prep.col_plan), _ptr(bad), ns, zh.ctypes.data_as(P),
                  None if wh is None else wh.ctypes.data_as(P), ctypes.byref(opts64), _ptr(out["ws"]),
                  out["ws"].numel(), _ptr(prep.proj_off), _ptr(out["G"]), _ptr(out["rho"]), _ptr(out["iters"]),
                  _ptr(out["status"]), _ptr(out["resid"]), _ptr(out.get("nk")), _stream(stream))
    G = None if out["G"] is None else out["G"][:prep.n_rows]
    res = Result(prep.proj_off, prep.proj_row, G, out["rho"][:prep.n_rows], out["iters"][:n], out["status"][:n],
                 out["resid"][:n])
    res.n_fallback = n_fallback
    res.shift_iters = None if out.get("nk") is None else out["nk"][:n]
    res.eps = out["eps"][:prep.n_rows] if eps_out else None
    res.G_diag = None if out.get("G_diag") is None else out["G_diag"][:n]
    res._out = out  # keep buffers alive with the result
    return res


def shifted_solve_static(prep: Prepared, z, w=None, tol=1e-10, max_iter=0, seed_index=-1, g_out=True, order=None,
                         batch_cols=0, stage_lds=-1, grid=0, shifts_per_lane=0, shifts_staged=False, out=None,
                         shift_iters=False, stream=None) -> Result:
    """FP64 shifted COCG through sgf_shifted_solve_static: the library's
    static device scratch serves as the workspace, so the C call allocates
    nothing.  Output tensors are allocated here unless ``out`` (a dict with
    "G", "rho", "iters", "status", "resid" and optionally "nk") is given."""
    torch = _torch()
    dev = prep.cols.device
    n = prep.cols.numel()
    zh = _cplx_host(z)
    wh = _cplx_host(w)
    ns = zh.size // 2
    opts = SolveOptsC(0, float(tol), int(max_iter), int(seed_index), 0, int(stage_lds), int(grid), 0,
                      int(batch_cols), int(shifts_per_lane), int(bool(shifts_staged)), 0.0, 0.0, 0)
    if out is None:
        out = {
            "G": torch.empty((max(prep.n_rows, 1), ns), dtype=torch.complex128, device=dev) if g_out else None,
            "rho": torch.empty(max(prep.n_rows, 1), dtype=torch.float64, device=dev),
            "iters": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            "status": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            "resid": torch.empty((max(n, 1), ns), dtype=torch.float64, device=dev),
            "nk": torch.empty((max(n, 1), ns), dtype=torch.int32, device=dev) if shift_iters else None,
        }
    d_order = None if order is None else _dev(order, torch.int32, dev)
    sc = prep.system.c()
    pc = prep.plan.c()
    _call("sgf_shifted_solve_static", ctypes.byref(sc), ctypes.byref(pc), ctypes.byref(prep.plan.totals), n,
          _ptr(prep.cols), _ptr(prep.col_plan), _ptr(d_order), ns, zh.ctypes.data_as(P),
          None if wh is None else wh.ctypes.data_as(P), ctypes.byref(opts), _ptr(prep.proj_off), _ptr(out["G"]),
          _ptr(out["rho"]), _ptr(out["iters"]), _ptr(out["status"]), _ptr(out["resid"]), _ptr(out.get("nk")),
          _stream(stream))
    G = None if out["G"] is None else out["G"][:prep.n_rows]
    res = Result(prep.proj_off, prep.proj_row, G, out["rho"][:prep.n_rows], out["iters"][:n], out["status"][:n],
                 out["resid"][:n])
    res.n_fallback = 0
    res.shift_iters = None if out.get("nk") is None else out["nk"][:n]
    res.eps = None
    res._out = out
    return res


def batch_limit(prep: Prepared, n_shifts, budget_bytes, max_iter=0, precision="fp64"):
    """Largest number of columns per launch whose solve workspace (Krylov
    history and per-column scalars) fits in budget_bytes."""
    n = prep.cols.numel()
    sc = prep.system.c()

    def ws(batch):
        opts = SolveOptsC({"fp64": 0, "mixed": 1}[precision], 1e-10, int(max_iter), -1, 50, -1, 0, 0, int(batch),
                          0, 0, 0.0, 0.0, 0)
        out = ctypes.c_size_t()
        _call("sgf_solve_workspace", ctypes.byref(sc), ctypes.byref(prep.plan.totals), max(n, 2), int(n_shifts),
              ctypes.byref(opts), ctypes.byref(out))
        return out.value

    w1, w2 = ws(1), ws(2)
    per = max(w2 - w1, 1)
    fixed = w1 - per
    return int(max(1, min(max(n, 1), (int(budget_bytes) - fixed) // per)))


class SolveGraph:
    """One shifted solve of a prepared column set, captured into a HIP graph
    (through torch.cuda.CUDAGraph) and replayed on demand.

    The constructor runs the solve once eagerly, which allocates the outputs
    and the workspace and stages z and w into it; the captured solve then
    consists of kernel launches only (ticket clear, seed pass, shift pass per
    batch) and writes the same output buffers on every replay.  Device data
    the graph reads (H, the plan, the column order) may change in place
    between replays, e.g. new Hamiltonian values on the same bond pattern.
    The column order, if any, must be a device tensor.  ``out`` (the _out of
    an earlier Result of the same prepared set) reuses that solve's output
    buffers and workspace instead of allocating new ones."""

    def __init__(self, prep: Prepared, z, w=None, tol=1e-10, order=None, out=None, **kw):
        torch = _torch()
        if kw.get("precision", "fp64") == "mixed":
            kw["fallback"] = False   # the FP64 re-solve reads the status array (a synchronisation)
        if order is not None and not isinstance(order, torch.Tensor):
            raise TypeError("SolveGraph: order must be a device tensor")
        kw.pop("profile", None)
        self.prep, self.z, self.w, self.tol, self.order, self.kw = prep, z, w, tol, order, kw
        self.result = solve_prepared(prep, z, w, tol, order=order, out=out, **kw)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            solve_prepared(prep, z, w, tol, order=order, out=self.result._out, shifts_staged=True, **kw)
        torch.cuda.synchronize()

    def replay(self) -> Result:
        self.graph.replay()
        return self.result


def solve_profile():
    """(seed_ms, shift_ms, batches) of the last solve run with profile=True on this thread."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _call("sgf_solve_profile", ctypes.byref(a), ctypes.byref(b), ctypes.byref(n))
    return a.value, b.value, n.value


def shifted_solve(system: System, columns, z, w=None, tol=1e-10, radius=0.0, radius_per_col=None, prune=True,
                  precision="fp64", max_iter=0, seed_index=-1, g_out=True, order=None, batch_cols=0, stage_lds=-1,
                  grid=0, max_loc_atoms=2048, shifts_per_lane=0, monitor_every=50, drift_tol=0.0, g_tol=0.0,
                  fallback=True, schedule="natural", model=None, stream=None) -> Result:
    """Green's-function elements and density-matrix entries for many columns.

    columns: global orbital indices j; each is solved on the local subspace of
    its atom (radius in nm; <= 0 means the whole system), pruned to the
    connected component when ``prune``.  z, w: complex shifts and weights.
    g_out: True/"proj" (G on the projection rows), "diag" (G_jj only) or
    False/"none" (rho only).  schedule: "natural" takes the columns in the
    given order (or ``order``); "learned" queues them longest-predicted-first
    from ``model`` (an IterationModel) through sgf_features, sgf_mlp_forward
    and sgf_order_by_prediction.  The order never changes a result.
    """
    prep = prepare(system, columns, radius, radius_per_col, prune, max_loc_atoms, stream)
    if schedule == "learned":
        if model is None:
            raise ValueError("schedule='learned' needs a trained IterationModel")
        order = learned_order(prep, model, stream)
    elif schedule != "natural":
        raise ValueError(f"schedule must be 'natural' or 'learned', not {schedule!r}")
    return solve_prepared(prep, z, w, tol, precision, max_iter, seed_index, g_out, order, batch_cols, stage_lds,
                          grid, monitor_every=monitor_every, shifts_per_lane=shifts_per_lane, drift_tol=drift_tol,
                          g_tol=g_tol, fallback=fallback, stream=stream)


def solve_workload(wl, system: Optional[System] = None, cols=None, prune=True, **kw) -> Result:
    """GPU solve of a workload from ``workloads`` (optionally a column subset)."""
    system = system_for(wl) if system is None else system
    rpc = wl.radius_per_col
    if cols is None:
        cols = wl.columns
    else:
        cols = np.asarray(cols, np.int64)
        if rpc is not None:
            pos = {int(j): i for i, j in enumerate(wl.columns)}
            rpc = rpc[[pos[int(j)] for j in cols]]
    kw.setdefault("tol", wl.tol)
    return shifted_solve(system, cols, wl.z, wl.w, radius=wl.radius, radius_per_col=rpc, prune=prune, **kw)


# --- Fermi-Dirac shifts -------------------------------------------------------------

def fermi_shifts(n_poles: int, kT: float, mu: float, moment: float = 1e8):
    """(z, w) complex128 [n_poles + 1]: the pole expansion of the Fermi
    function as shifts and weights of the shifted solve, so that its rho is
    f(H) at temperature kT (eV) and chemical potential mu (eV).  The pole
    nearest the real axis comes first; solve with seed_index=-2."""
    z = np.zeros(2 * (n_poles + 1))
    w = np.zeros(2 * (n_poles + 1))
    _call("sgf_fermi_shifts", int(n_poles), float(kT), float(mu), float(moment), z.ctypes.data_as(P),
          w.ctypes.data_as(P))
    return z.view(np.complex128), w.view(np.complex128)


# --- global operator ------------------------------------------------------------

def bsr_apply(system: System, z, x, precision="fp64", out=None, stream=None):
    """y = (z S - H) x over the whole system for x of shape [n_orb] or
    [n_orb, n_rhs] (n_rhs in 1, 2, 4, 8); complex128 (fp64) or complex64
    (fp32, on the FP32 shadows, built here if missing)."""
    torch = _torch()
    prec = {"fp64": 0, "fp32": 1}[precision]
    if prec == 1 and system.h32 is None:
        system.add_f32(stream)
    dt = torch.complex128 if prec == 0 else torch.complex64
    assert x.dtype == dt and x.is_contiguous() and x.shape[0] == 4 * system.n_atoms
    n_rhs = 1 if x.dim() == 1 else x.shape[1]
    y = torch.empty_like(x) if out is None else out
    zh = np.array([complex(z).real, complex(z).imag], np.float64)
    sc = system.c()
    _call("sgf_bsr_apply", ctypes.byref(sc), prec, n_rhs, zh.ctypes.data_as(P), _ptr(x), _ptr(y), _stream(stream))
    return y


# --- after rho: traces, electron count, band energy, Fermi level ----------------

def traces(prep: Prepared, res: Result, converged_only=True, stream=None):
    """Per-shift traces over the solved columns from a solve's outputs:
    T_k = sum_j (G S)_jj and U_k = sum_j (G H)_jj (complex128 [n_shifts],
    None when the solve kept no G), and (tr(rho S), tr(rho H)) at the solve's
    own weights; with ``converged_only`` a column that did not converge
    contributes nothing.  Synchronises the stream."""
    torch = _torch()
    dev = prep.cols.device
    n = prep.cols.numel()
    rows = int(prep.n_rows)
    ns = 1 if res.G is None else int(res.G.shape[1])
    ws = ctypes.c_size_t()
    _call("sgf_trace_workspace", rows, ns, ctypes.byref(ws))
    d_ws = _bytes(ws.value, dev)
    T = torch.empty(ns, dtype=torch.complex128, device=dev) if res.G is not None else None
    U = torch.empty(ns, dtype=torch.complex128, device=dev) if res.G is not None else None
    rtr = torch.empty(2, dtype=torch.float64, device=dev)
    sc = prep.system.c()
    status = res.status if converged_only else None
    _call("sgf_traces", ctypes.byref(sc), n, _ptr(prep.cols), _ptr(prep.proj_off), _ptr(prep.proj_row), _ptr(status),
          rows, _ptr(res.G), _ptr(res.rho), ns, _ptr(d_ws), ws.value, _ptr(T), _ptr(U), _ptr(rtr), _stream(stream))
    out_t = None if T is None else T.cpu().numpy()
    out_u = None if U is None else U.cpu().numpy()
    r = rtr.cpu().numpy()
    return out_t, out_u, (float(r[0]), float(r[1]))


def occupation(T, U, w):
    """(electron count, band energy) = -(1/pi) sum_k Im(w_k T_k), -(1/pi) sum_k Im(w_k U_k)."""
    t, u, wv = (np.ascontiguousarray(np.asarray(a, np.complex128)) for a in (T, U, w))
    ne, eb = ctypes.c_double(), ctypes.c_double()
    _call("sgf_occupation", t.size, t.ctypes.data_as(P), u.ctypes.data_as(P), wv.ctypes.data_as(P),
          ctypes.byref(ne), ctypes.byref(eb))
    return ne.value, eb.value


def fermi_level(z, T, U, n_target):
    """(mu, electron count, band energy): the first grid energy at which the
    trapezoid-weighted electron count reaches n_target."""
    zz, t, u = (np.ascontiguousarray(np.asarray(a, np.complex128)) for a in (z, T, U))
    mu, ne, eb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _call("sgf_fermi_level", zz.size, zz.ctypes.data_as(P), t.ctypes.data_as(P), u.ctypes.data_as(P),
          float(n_target), ctypes.byref(mu), ctypes.byref(ne), ctypes.byref(eb))
    return mu.value, ne.value, eb.value


# --- learned scheduling ---------------------------------------------------------

def features(prep: Prepared, stream=None):
    """float32 [n_cols, 5] features of the prepared columns (see include/sgf.h)."""
    torch = _torch()
    n = prep.cols.numel()
    out = torch.empty((max(n, 1), MLP_NFEAT), dtype=torch.float32, device=prep.cols.device)
    sc, pc = prep.system.c(), prep.plan.c()
    _call("sgf_features", ctypes.byref(sc), ctypes.byref(pc), n, _ptr(prep.cols), _ptr(prep.col_plan), _ptr(out),
          _stream(stream))
    return out[:n]


class IterationModel:
    """The iteration-count network; params is its flat FP32 parameter vector
    (initial weights are an input, e.g. workloads.mlp_init)."""

    def __init__(self, params, device="cuda"):
        torch = _torch()
        self.params = _dev(np.asarray(params, np.float32) if not isinstance(params, torch.Tensor) else params,
                           torch.float32, device)
        assert self.params.numel() == MLP_NPARAM
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def normalize(self, feat, stream=None):
        _call("sgf_mlp_normalize", _ptr(self.params), _ptr(feat.contiguous()), feat.shape[0], _stream(stream))

    def predict(self, feat, stream=None):
        torch = _torch()
        y = torch.empty(max(feat.shape[0], 1), dtype=torch.float32, device=feat.device)
        _call("sgf_mlp_forward", _ptr(self.params), _ptr(feat.contiguous()), feat.shape[0], _ptr(y), _stream(stream))
        return y[:feat.shape[0]]

    def gradient(self, feat, target, stream=None):
        torch = _torch()
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _call("sgf_mlp_gradient", _ptr(self.params), _ptr(feat.contiguous()), _ptr(target.contiguous()),
              feat.shape[0], _ptr(g), _ptr(loss), _stream(stream))
        return g, loss

    def train_step(self, feat, target, lr=1e-3, stream=None):
        torch = _torch()
        self.step += 1
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _call("sgf_mlp_train_step", _ptr(self.params), _ptr(self.m), _ptr(self.v), self.step, float(lr),
              _ptr(feat.contiguous()), _ptr(target.contiguous()), feat.shape[0], _ptr(loss), _stream(stream))
        return loss

    def fit(self, feat, target, epochs=20, lr=1e-3, seed=0, holdout=0.2, stream=None):
        """Minibatch Adam on (feat, target) with a seeded shuffle; returns the
        per-epoch mean training loss (on the standardised target) and the
        held-out MSE (on the target itself).

        The network is trained on the target standardised with the training
        split's mean m and standard deviation s, and the map back,
        y = s (W3 . h2 + b3) + m, is then folded into the output layer
        (W3 <- s W3, b3 <- s b3 + m), so that predict() returns the target's
        own units.  Iteration counts vary by about 15 % around their mean:
        trained on log(iterations) itself, most of the optimiser's steps went
        to moving the output bias and the held-out error stayed near the
        target's variance."""
        torch = _torch()
        n = feat.shape[0]
        perm = np.random.default_rng(seed).permutation(n)
        n_test = int(holdout * n)
        test = torch.as_tensor(perm[:n_test], device=feat.device)
        train = perm[n_test:]
        train_d = torch.as_tensor(train, device=feat.device)
        self.normalize(feat[train_d])
        t_train = target[train_d].to(torch.float64)
        t_mean = float(t_train.mean())
        t_std = float(t_train.std()) if train.size > 1 else 0.0
        t_std = t_std if t_std > 1e-12 else 1.0
        scaled = ((target.to(torch.float64) - t_mean) / t_std).to(torch.float32)
        rng = np.random.default_rng(seed + 1)
        hist = []
        for _ in range(epochs):
            order = torch.as_tensor(rng.permutation(train), device=feat.device)
            losses = []
            for b in range(0, order.numel() - MLP_BATCH + 1, MLP_BATCH):
                idx = order[b:b + MLP_BATCH]
                losses.append(self.train_step(feat[idx], scaled[idx], lr, stream))
            hist.append(float(torch.cat(losses).mean()))
        w3 = slice(MLP_NPARAM - 1 - MLP_NH, MLP_NPARAM - 1)
        self.params[w3] *= t_std
        self.params[MLP_NPARAM - 1] = self.params[MLP_NPARAM - 1] * t_std + t_mean
        self.target_scale = (t_mean, t_std)
        test_mse = float(((self.predict(feat[test]) - target[test]) ** 2).mean()) if n_test else float("nan")
        return hist, test_mse


def learned_order(prep: Prepared, model: "IterationModel", stream=None, y_lo=0.0, y_hi=float(np.log(4096.0))):
    """Work-queue order of the prepared columns: plans by the largest
    predicted iteration count among their columns, the columns of a plan
    together (features -> network -> grouped counting sort on the device)."""
    return order_groups_by_prediction(model.predict(features(prep, stream), stream), prep.col_plan,
                                      prep.plan.n_plans, y_lo, y_hi, stream)


def order_groups_by_prediction(pred, col_plan, n_plans, y_lo, y_hi, stream=None):
    """Permutation of the columns with the columns of each plan together,
    plans by their largest prediction first."""
    torch = _torch()
    n = pred.numel()
    ws = ctypes.c_size_t()
    _call("sgf_order_groups_workspace", int(n_plans), ctypes.byref(ws))
    d_ws = _bytes(ws.value, pred.device)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=pred.device)
    _call("sgf_order_groups_by_prediction", _ptr(pred.contiguous()), n, _ptr(col_plan), int(n_plans), float(y_lo),
          float(y_hi), _ptr(order), _ptr(d_ws), ws.value, _stream(stream))
    return order[:n]


def order_by_prediction(pred, y_lo, y_hi, stream=None):
    """Permutation of the columns, largest predicted work first."""
    torch = _torch()
    n = pred.numel()
    ws = ctypes.c_size_t()
    _call("sgf_order_workspace", ctypes.byref(ws))
    d_ws = _bytes(ws.value, pred.device)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=pred.device)
    _call("sgf_order_by_prediction", _ptr(pred.contiguous()), n, float(y_lo), float(y_hi), _ptr(order), _ptr(d_ws),
          ws.value, _stream(stream))
    return order[:n]



# --- wavepacket propagation ---------------------------------------------------

HBAR_EV_FS = 0.6582119569509066  # eV fs


def wp_bounds(system: System, stream=None):
    """(e_min, e_max): Gershgorin bounds of H (synchronous)."""
    ws = ctypes.c_size_t()
    _call("sgf_wp_workspace", int(system.n_atoms), 1, ctypes.byref(ws))
    d_ws = _bytes(ws.value, system.row_ptr.device)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _call("sgf_wp_bounds", ctypes.byref(system.c()), _ptr(d_ws), ws.value, ctypes.byref(lo), ctypes.byref(hi),
          _stream(stream))
    return lo.value, hi.value


def wp_terms(a_tau: float, tol: float = 1e-13) -> int:
    """Series length for argument a tau (smallest K > |a tau| with
    |J_K|, |J_{K+1}| <= tol, at least 3)."""
    k = ctypes.c_int32()
    _call("sgf_wp_terms", float(a_tau), float(tol), ctypes.byref(k))
    return k.value


def wp_propagate(system: System, psi, h_fs: float, n_steps: int, e_min: float, e_max: float, n_terms: int,
                 stream=None):
    """n_steps Chebyshev steps of length h_fs of the packets in psi, in place:
    complex128 device tensor [n_orb] or [n_orb, n_rhs] (n_rhs in 1, 2, 4, 8),
    contiguous.  Returns psi."""
    torch = _torch()
    if psi.dtype != torch.complex128 or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous complex128 tensor")
    n_rhs = 1 if psi.dim() == 1 else int(psi.shape[1])
    if psi.shape[0] != 4 * system.n_atoms:
        raise ValueError("psi must have 4 * n_atoms rows")
    ws = ctypes.c_size_t()
    _call("sgf_wp_workspace", int(system.n_atoms), n_rhs, ctypes.byref(ws))
    d_ws = _bytes(ws.value, psi.device)
    _call("sgf_wp_propagate", ctypes.byref(system.c()), n_rhs, _ptr(psi), float(h_fs), int(n_steps), float(e_min),
          float(e_max), int(n_terms), _ptr(d_ws), ws.value, _stream(stream))
    return psi


# --- band-structure forces ---------------------------------------------------------

def band_forces(prep: Prepared, res: Result, params, xyz=None, eps=None, converged_only=True, stream=None):
    """Band forces at fixed rho (and, with an overlap, fixed energy-density
    matrix ``eps``, one value per projection row, e.g. from
    energy_density): float64 [n_atoms, 3] on the device (eV/nm).  params:
    the tight-binding parameters the system was built with; xyz: positions
    [n_atoms, 3] (nm; the system's own when omitted)."""
    torch = _torch()
    dev = prep.cols.device
    d_xyz = _dev(prep.system.xyz if xyz is None else xyz, torch.float64, dev)
    F = torch.empty((prep.system.n_atoms, 3), dtype=torch.float64, device=dev)
    sc = prep.system.c()
    tb = _tb_c(params)
    status = res.status if converged_only else None
    _call("sgf_band_forces", ctypes.byref(sc), _ptr(d_xyz), ctypes.byref(tb), int(prep.cols.numel()), _ptr(prep.cols),
          _ptr(prep.proj_off), _ptr(prep.proj_row), _ptr(status), _ptr(res.rho), _ptr(eps), _ptr(F),
          _stream(stream))
    return F


def energy_density(res: Result, z, w, stream=None):
    """eps_t = -(1/pi) sum_k Im(w_k z_k G_t(z_k)) on every projection row of
    a solve that kept G: float64 [rows] on the device."""
    torch = _torch()
    if res.G is None:
        raise ValueError("energy_density: the solve did not keep G")
    dev = res.G.device
    rows, ns = int(res.G.shape[0]), int(res.G.shape[1])
    d_z = _dev(np.asarray(z, np.complex128), torch.complex128, dev)
    d_w = _dev(np.asarray(w, np.complex128), torch.complex128, dev)
    if d_z.numel() != ns or d_w.numel() != ns:
        raise ValueError(f"energy_density: {d_z.numel()} shifts and {d_w.numel()} weights for G with {ns}")
    eps = torch.empty(max(rows, 1), dtype=torch.float64, device=dev)
    _call("sgf_energy_density", rows, ns, _ptr(d_z), _ptr(d_w), _ptr(res.G), _ptr(eps), _stream(stream))
    return eps[:rows]


# --- quantum molecular dynamics ------------------------------------------------------

def md_kick(force, mass, h_fs, vel, stream=None):
    """vel += (h/2) force / mass in place (nm/fs; force eV/nm, mass amu)."""
    n = int(vel.shape[0])
    _call("sgf_md_kick", n, _ptr(force), _ptr(mass), float(h_fs), _ptr(vel), _stream(stream))
    return vel


def md_drift(vel, h_fs, xyz, stream=None):
    """xyz += h vel in place (nm)."""
    n = int(xyz.shape[0])
    _call("sgf_md_drift", n, _ptr(vel), float(h_fs), _ptr(xyz), _stream(stream))
    return xyz


class QMD:
    """Quantum molecular dynamics with the band forces of the shifted solves:
    every step is velocity Verlet around the whole path at the new positions
    (neighbour list and H / S, local subspaces, shifted solve of every
    column, band forces with the energy-density term when S != I).

    xyz, vel: [n_atoms, 3] (nm, nm/fs), mass: [n_atoms] amu; z, w: shifts and
    quadrature weights; radius: local-subspace radius (nm); ws_budget: bytes
    of solve workspace per step (the columns run in launches of what it
    holds, which follows the subspaces as the atoms move)."""

    def __init__(self, xyz, vel, mass, params, z, w, tol=1e-12, radius=1.0, prune=True, device="cuda",
                 ws_budget=None, **solve_kw):
        torch = _torch()
        self.xyz = _dev(xyz, torch.float64, device).clone()
        self.vel = _dev(vel, torch.float64, device).clone()
        self.mass = _dev(mass, torch.float64, device).contiguous()
        self.params, self.z, self.w, self.tol, self.radius, self.prune = params, z, w, tol, radius, prune
        self.solve_kw = solve_kw
        self.ws_budget = ws_budget   # bytes of solve workspace per step (None: all columns in one launch)
        self.columns = np.arange(4 * self.xyz.shape[0], dtype=np.int64)
        # the column -> subspace-centre map does not change with the positions
        centers, radii, col_plan = plan_columns(self.columns, radius)
        self._plan_in = tuple(_dev(a, t, device) for a, t in ((self.columns, torch.int64), (col_plan, torch.int32),
                                                              (centers, torch.int32), (radii, torch.float64)))
        self.force, self.last = self.forces()

    def forces(self):
        """Band forces at the current positions (and the solve behind them)."""
        system = build_hamiltonian(self.xyz, self.params, device=self.xyz.device)
        prep = prepare_planned(system, *self._plan_in, prune=self.prune)
        ovl = bool(self.params.overlap)
        kw = dict(self.solve_kw)
        if self.ws_budget is not None:
            kw["batch_cols"] = batch_limit(prep, len(self.z), self.ws_budget)
        res = solve_prepared(prep, self.z, self.w, tol=self.tol, g_out=False, eps_out=ovl, **kw)
        return band_forces(prep, res, self.params, xyz=self.xyz, eps=res.eps if ovl else None), (prep, res)

    def step(self, h_fs=1.0):
        md_kick(self.force, self.mass, h_fs, self.vel)
        md_drift(self.vel, h_fs, self.xyz)
        self.force, self.last = self.forces()
        md_kick(self.force, self.mass, h_fs, self.vel)
        return self
