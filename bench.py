#!/usr/bin/env python3
"""Benchmark: converged (column x shift) solves/s of the shifted-COCG path.

Workload (one GPU): the 118,300-atom polymer bundle (169 chains of 700 sp
atoms, Slater-Koster tight binding, S = I), every one of its 473,200 basis
columns on its R = 1.0 nm local subspace (pruned to the connected component),
128 shifts E + 0.01i on [-30, 30] eV, tol 1e-12 (FP64 accuracy 1e-10 per
result).  One step = the whole hot path on that input: neighbour list,
Hamiltonian assembly, local-subspace plans, projection layout and the
two-pass shifted solve (Green's function on the projection rows and the
density matrix).  Inputs (atom positions, the column list and the column ->
subspace-centre map) are resident in HBM before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector peak
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_flops(nblk, nl, nrow, iters, nk, ns):
    """Algorithmic FP64 flops of the two passes (per launch set of one solve).

    Seed pass, per column-iteration: 64 per local 4x4 block (real block x
    complex vector) + 44 per local orbital (w = z_s p - Hp, mu, s update,
    rho', ||s||^2, p update); per shift-iteration while the shift is active:
    28 (pi recurrence and freeze test).
    Shift pass, per shift-step: 30 (UL pivot: diagonal, one complex product,
    reciprocal, next multiplier) + 8 per projection row (Horner step).
    """
    nk_sum = nk.sum(axis=1).astype(np.float64)
    seed = float(np.sum(iters * (64.0 * nblk + 44.0 * nl)) + 28.0 * nk_sum.sum())
    shift = float(np.sum(nk_sum * (30.0 + 8.0 * nrow)))
    return seed, shift


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=8192, help="columns per history batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-g", action="store_true", help="skip writing G (rho only)")
    ap.add_argument("--shifts-per-lane", type=int, default=0)
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every run of this path uses a single MI355X; columns are "
              "independent, so a multi-GPU run shards columns spatially with no communication in the "
              "Krylov loop (see DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    import paper_1603_09616_amd as sgf
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = W.config_bundle()
    ns = wl.z.size
    # resident inputs: positions, columns and their subspace centres
    centers, radii, col_plan = sgf.plan_columns(wl.columns, wl.radius)
    d_xyz = torch.as_tensor(wl.xyz, device=dev)
    d_cols = torch.as_tensor(wl.columns, device=dev)
    d_cp = torch.as_tensor(col_plan, device=dev)
    d_centers = torch.as_tensor(centers, device=dev)
    d_radii = torch.as_tensor(radii, device=dev)
    log(f"[bench] workload {wl.name}: {wl.n_atoms} atoms, {wl.columns.size} columns, {ns} shifts, "
        f"batch {args.batch}")

    out_buf = {}

    def step(profile):
        s = sgf.build_hamiltonian(d_xyz, wl.tb, device=dev)
        prep = sgf.prepare_planned(s, d_cols, d_cp, d_centers, d_radii, prune=True)
        res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=not args.no_g, batch_cols=args.batch,
                                 out=out_buf.get("out"), profile=profile, shift_iters=True,
                                 shifts_per_lane=args.shifts_per_lane)
        out_buf["out"] = res._out
        return s, prep, res

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = []
    for i in range(args.steps):
        s, prep, res = step(True)
        prof.append(sgf.solve_profile())   # waits only for this step's solve events
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    seed_ms = float(np.mean([p[0] for p in prof]))
    shift_ms = float(np.mean([p[1] for p in prof]))
    launches = prof[-1][2]
    log(f"[bench] {args.steps} steps: {ms_step:.2f} ms/step; seed pass {seed_ms:.2f} ms, shift pass "
        f"{shift_ms:.2f} ms ({launches} launches each)")

    iters = res.iters.cpu().numpy().astype(np.float64)
    status = res.status.cpu().numpy()
    resid = res.resid.cpu().numpy()
    nk = res.shift_iters.cpu().numpy()
    converged = int(np.sum(resid <= wl.tol))
    plan = prep.plan
    cp = prep.col_plan.cpu().numpy()
    nl = 4 * np.diff(plan.atom_off.cpu().numpy())[cp]
    nblk = np.diff(plan.blk_off.cpu().numpy())[cp]
    nrow = 4 * np.diff(plan.pa_off.cpu().numpy())[cp]
    f_seed, f_shift = pass_flops(nblk, nl, nrow, iters, nk, ns)
    value = converged / (ms_step * 1e-3)
    seed_tf = f_seed / (seed_ms * 1e-3) / 1e12
    shift_tf = f_shift / (shift_ms * 1e-3) / 1e12
    dominant = "k_shift" if shift_ms >= seed_ms else "k_seed"
    dom_ms, dom_f = (shift_ms, f_shift) if dominant == "k_shift" else (seed_ms, f_seed)
    achieved = dom_f / (dom_ms * 1e-3) / 1e12

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_seconds)

    line = {
        "metric": "converged (column x shift) solves/s at tol 1e-12",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "polymer bundle 13x13 chains x 700 sp atoms (118,300 atoms), all 473,200 columns, "
                        "128 shifts E+0.01i on [-30,30] eV, R=1.0 nm pruned, tol 1e-12, FP64",
            "columns": int(wl.columns.size), "shifts": ns, "batch_cols": args.batch,
            "step": "build_hamiltonian + plan + shifted_solve (seed pass + shift pass)",
        },
        "roofline": {
            "kernel": dominant,
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": None,
            "launches_per_step": launches,
            "passes": {
                "k_seed": {"ms_per_step": seed_ms, "tflop_per_step": f_seed / 1e12, "tflops": seed_tf},
                "k_shift": {"ms_per_step": shift_ms, "tflop_per_step": f_shift / 1e12, "tflops": shift_tf},
            },
        },
        "cpu_baseline": cpu,
        "converged_solves": converged,
        "columns_not_converged": int(np.sum(status != 0)),
        "iters_mean": float(iters.mean()),
    }
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline(wl, seconds):
    """The FP64 oracle on a seeded sample of the same columns, for ~`seconds`."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    b = oracle.system_for(wl)
    order = np.random.default_rng(1603).permutation(wl.columns.size)
    done = conv = 0
    chunk = 1024
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < order.size:
        cols = np.sort(wl.columns[order[done:done + chunk]])
        r = oracle.solve_workload(wl, b, cols=cols, threads=threads)
        conv += int(np.sum(r.resid <= wl.tol))
        done += cols.size
    dt = time.perf_counter() - t0
    log(f"[bench] oracle: {done} columns in {dt:.1f} s on {threads} threads")
    return {"value": conv / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} seeded random columns of the same workload (all 128 shifts), {dt:.1f} s wall"}


if __name__ == "__main__":
    sys.exit(main())
