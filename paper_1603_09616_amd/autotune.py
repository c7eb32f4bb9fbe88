"""Autotuner for the launch choices of the shifted solve.

The choices that do not change the method, only how it maps onto the chip:

* ``stage_lds``: the seed-pass variant.  S = I: -1, when every local
  subspace fits a wavefront, four columns of a plan per wavefront with its
  blocks in LDS up to 128 shifts, two columns up to 256 and register rows
  above; 5: two columns per wavefront; 3: register rows, one column per
  wavefront; 1: local operator staged in LDS; 0: operator read from global
  memory.  S != I, for the subspaces of more than 16
  atoms: -1 the library's default (two wavefronts per column); 4 (overlap
  blocks s_ab I4) one wavefront per column with two rows per lane; 2 (a
  general overlap) one wavefront per column with the orbital-level inverse;
* ``shifts_per_lane``: shifts handled by one lane of the shift pass (1, 2);
* ``grid``: persistent seed-pass workgroups (0: as many as fit the device).

Each candidate is timed with HIP events on the launch stream, on a seeded
sample of the prepared columns (whole plans, their columns next to each
other, solved through the work-queue order, so no re-planning), median of
``reps`` runs after a warm-up.  The winner is cached
in a JSON file keyed by the device and the shape of the workload (precision,
shift count, largest subspace, largest row, projection size, overlap), and
reused by later calls with the same key.  Results do not depend on the
choice beyond rounding order.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import numpy as np


def cache_path() -> str:
    return os.environ.get("SGF_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "sgf",
                                                                 "autotune.json")


def signature(totals, n_shifts: int, precision: str, has_overlap: bool, device_name: str) -> str:
    return (f"{device_name}|{precision}|ns={n_shifts}|loc_atoms={totals.max_loc_atoms}|"
            f"row_blocks={totals.max_row_blocks}|proj_atoms={totals.max_proj_atoms}|S={int(has_overlap)}")


def candidates(totals, precision: str, has_overlap: bool, per_atom_overlap: bool = False) -> list:
    """The launch choices that apply to this workload shape."""
    register_ok = totals.max_loc_atoms <= 16 and totals.max_row_blocks <= 8 and not has_overlap
    if precision == "mixed":
        seeds = [-1]
    elif has_overlap:
        # the variants differ only where some subspace has more than 16 atoms
        seeds = [-1] if totals.max_loc_atoms <= 16 else [-1, 4 if per_atom_overlap else 2]
    else:
        seeds = [-1, 5, 3, 1, 0] if register_ok else [-1, 0]
    lanes = [1, 2] if (precision == "fp64" and totals.max_proj_atoms <= 5) else [1]
    grids = [0, 2048, 1024]
    out = []
    for sv in seeds:
        for ln in lanes:
            for g in grids:
                out.append({"stage_lds": sv, "shifts_per_lane": ln, "grid": g})
    return out


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, table: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(prep, z, w=None, tol=1e-10, precision="fp64", sample=32768, reps=3, seed=0, use_cache=True,
         path: Optional[str] = None, log=None) -> dict:
    """Best launch choices for solving ``prep`` at these shifts; returns
    {"choice": {...}, "key": ..., "timings_ms": {...} or None, "cached": bool}."""
    import torch
    from . import solve_prepared

    path = path or cache_path()
    totals = prep.plan.totals
    ns = int(np.asarray(z).size)
    has_s = prep.system.s is not None
    key = signature(totals, ns, precision, has_s, torch.cuda.get_device_name(prep.cols.device))
    table = _load(path) if use_cache else {}
    if key in table:
        return {"choice": table[key]["choice"], "key": key, "timings_ms": None, "cached": True}

    # whole plans, drawn at random, with each plan's columns together (the
    # four-column seed pass takes a plan's columns in one wavefront)
    cp = prep.col_plan.cpu().numpy()
    by_plan = np.argsort(cp, kind="stable")
    plans = np.unique(cp)
    chosen = np.random.default_rng(seed).permutation(plans)
    per_plan = max(1, int(round(cp.size / max(plans.size, 1))))
    chosen = np.sort(chosen[:max(1, sample // per_plan)])
    keep = np.isin(cp[by_plan], chosen)
    pick = by_plan[keep].astype(np.int32)
    order = torch.as_tensor(pick, device=prep.cols.device)
    out = None
    timings = {}
    for cand in candidates(totals, precision, has_s, bool(getattr(prep.system, "s_orbital_diagonal", False))):
        name = json.dumps(cand, sort_keys=True)
        ms = []
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            res = solve_prepared(prep, z, w, tol, precision=precision, order=order, queue_len=pick.size, out=out,
                                 fallback=False, g_out=True, batch_cols=int(pick.size), **cand)
            e1.record()
            torch.cuda.synchronize()
            out = res._out
            if r:
                ms.append(e0.elapsed_time(e1))
        timings[name] = float(np.median(ms))
        if log:
            log(f"[autotune] {name}: {timings[name]:.3f} ms")
    best = min(timings, key=timings.get)
    choice = json.loads(best)
    if use_cache:
        table = _load(path)
        table[key] = {"choice": choice, "timings_ms": timings, "sample_columns": int(pick.size)}
        _store(path, table)
    return {"choice": choice, "key": key, "timings_ms": timings, "cached": False}
