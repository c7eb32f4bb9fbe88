#!/usr/bin/env python3
"""Benchmark: converged (column x shift) solves/s of the shifted-COCG path.

Workload (one GPU): the 118,300-atom polymer bundle (169 chains of 700 sp
atoms, Slater-Koster tight binding, S = I), every one of its 473,200 basis
columns on its R = 1.0 nm local subspace (pruned to the connected component),
128 shifts E + 0.01i on [-30, 30] eV, tol 1e-12 (FP64 accuracy 1e-10 per
result).  One step = the whole hot path on that input: neighbour list,
Hamiltonian assembly, local-subspace plans, projection layout and the
per-column features, the iteration-count network's predictions and the
longest-predicted-first column order, and the two-pass shifted solve
(Green's function on the projection rows and the density matrix).  The
network is trained before the timed region on iteration counts logged by
solves of a differently seeded bundle.  Inputs (atom positions, the column list and the column ->
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


def train_scheduler(sgf, W, dev, n_logged=50000):
    """The learned scheduler's setup (outside the timed region): log the
    iteration counts of n_logged solves of a differently seeded bundle of the
    same shape, then train the iteration-count network on them with the
    library's own kernels."""
    import torch
    tw = W.config_bundle(config_no=20)
    cols = np.sort(np.random.default_rng(5).choice(tw.columns, n_logged, replace=False))
    ts = sgf.system_for(tw)
    tp = sgf.prepare(ts, cols, radius=tw.radius, prune=True)
    tr = sgf.solve_prepared(tp, tw.z, tw.w, tol=tw.tol, g_out=False,
                            batch_cols=sgf.batch_limit(tp, tw.z.size, 16 << 30))
    feat = sgf.features(tp)
    target = torch.log(tr.iters.to(torch.float32))
    model = sgf.IterationModel(W.mlp_init(3))
    t0 = time.perf_counter()
    hist, test_mse = model.fit(feat, target, epochs=10, lr=1e-3, seed=4)
    torch.cuda.synchronize()
    info = {"logged_solves": int(cols.size), "epochs": 10, "train_s": round(time.perf_counter() - t0, 3),
            "final_train_mse": hist[-1], "heldout_mse": test_mse, "target_var": float(target.var())}
    del tp, tr, ts
    torch.cuda.empty_cache()
    return model, info


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=0, help="columns per launch (0: as many as --ws-gib holds)")
    ap.add_argument("--ws-gib", type=float, default=112.0, help="solve workspace budget for the automatic batch")
    ap.add_argument("--plain-batch", type=int, default=8192, help="columns per launch of the plain variant")
    ap.add_argument("--no-variants", action="store_true", help="time only the full solver")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-g", action="store_true", help="skip writing G (rho only)")
    ap.add_argument("--shifts-per-lane", type=int, default=0)
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every run of this path uses a single MI355X; columns are "
              "independent, so a multi-GPU run shards columns spatially with no communication in the "
              "Krylov loop. Run with --gpus 1.", file=sys.stderr)
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

    model, train_info = train_scheduler(sgf, W, dev)
    log(f"[bench] scheduler trained on {train_info['logged_solves']} logged solves in {train_info['train_s']} s: "
        f"held-out MSE {train_info['heldout_mse']:.4f} (target variance {train_info['target_var']:.4f})")

    s0 = sgf.build_hamiltonian(d_xyz, wl.tb, device=dev)
    p0 = sgf.prepare_planned(s0, d_cols, d_cp, d_centers, d_radii, prune=True)
    batch = args.batch or sgf.batch_limit(p0, ns, int(args.ws_gib * (1 << 30)))
    del s0, p0
    log(f"[bench] workload {wl.name}: {wl.n_atoms} atoms, {wl.columns.size} columns, {ns} shifts, "
        f"batch {batch}")

    def make_step(order_mode, batch_cols):
        out_buf = {}

        def step(profile):
            s = sgf.build_hamiltonian(d_xyz, wl.tb, device=dev)
            prep = sgf.prepare_planned(s, d_cols, d_cp, d_centers, d_radii, prune=True)
            order = None
            if order_mode == "learned":
                pred = model.predict(sgf.features(prep))
                order = sgf.order_by_prediction(pred, 0.0, float(np.log(4096.0)))
            res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=not args.no_g, batch_cols=batch_cols,
                                     order=order, out=out_buf.get("out"), profile=profile, shift_iters=True,
                                     shifts_per_lane=args.shifts_per_lane)
            out_buf["out"] = res._out
            return s, prep, res
        return step

    def timed(step, steps, warmup, name):
        for i in range(warmup):
            step(False)
            torch.cuda.synchronize()
            log(f"[bench] {name}: warmup {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prof = []
        for _ in range(steps):
            s, prep, res = step(True)
            prof.append(sgf.solve_profile())   # waits only for this step's solve events
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        seed_ms = float(np.mean([p[0] for p in prof]))
        shift_ms = float(np.mean([p[1] for p in prof]))
        log(f"[bench] {name}: {steps} steps, {ms:.2f} ms/step; seed pass {seed_ms:.2f} ms, shift pass "
            f"{shift_ms:.2f} ms ({prof[-1][2]} launches each)")
        return ms, seed_ms, shift_ms, prof[-1][2], (s, prep, res)

    ms_step, seed_ms, shift_ms, launches, (s, prep, res) = timed(make_step("learned", batch), args.steps,
                                                                 args.warmup, "fp64 batched+learned")
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
    variants = {"fp64_batched_learned": {"ms_per_step": ms_step, "solves_per_s": value, "seed_ms": seed_ms,
                                         "shift_ms": shift_ms, "launches": launches, "batch_cols": batch,
                                         "order": "learned"}}
    if not args.no_variants:
        rho_ref = res.rho.clone()
        del res, prep, s
        for name, mode, b in [("fp64_batched", "natural", batch), ("fp64_plain", "natural", args.plain_batch)]:
            torch.cuda.empty_cache()
            ms_v, sd_v, sh_v, l_v, (_, _, r_v) = timed(make_step(mode, b), max(2, args.steps // 2), 1, name)
            same = bool(torch.equal(r_v.rho, rho_ref))
            variants[name] = {"ms_per_step": ms_v, "solves_per_s": converged / (ms_v * 1e-3), "seed_ms": sd_v,
                              "shift_ms": sh_v, "launches": l_v, "batch_cols": b, "order": mode,
                              "rho_bitwise_equal": same}
            del r_v
        variants["speedup_vs_fp64_plain"] = variants["fp64_plain"]["ms_per_step"] / ms_step
        variants["learned_gain_vs_natural_order"] = variants["fp64_batched"]["ms_per_step"] / ms_step

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
            "columns": int(wl.columns.size), "shifts": ns, "batch_cols": batch,
            "step": "build_hamiltonian + plan + features + MLP prediction + order + shifted_solve "
                    "(seed pass + shift pass)",
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
        "variants": variants,
        "scheduler": train_info,
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
