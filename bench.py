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
# columns (whole plans) the autotuner times each launch candidate on: enough
# persistent waves per compute unit that the tail of a launch weighs as it
# does on the whole bundle
TUNE_SAMPLE = 131072


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def model_flops(nblk, nrow, iters, nk):
    """Algorithmic FP64 flops of the method's two arithmetic steps, per launch
    set of one solve (the per-unit counts the roofline is stated in):

    seed operator w = z_s p - H p: 64 per local 4x4 block per
    column-iteration (a real block times a complex vector: 16 complex-by-real
    multiply-adds);
    projected G updates X^k += alpha^k P^k, P^k = r_P / pi^k + beta^k P^k:
    16 per projection row per active shift-step (two complex multiply-adds).
    Returns (seed operator, projected updates)."""
    a4 = float(np.sum(iters * 64.0 * nblk))
    a8 = float(np.sum(nk.sum(axis=1).astype(np.float64) * 16.0 * nrow))
    return a4, a8


def executed_flops(nblk, nl, nrow, iters, nk):
    """FP64 flops the two kernels execute (a fuller count than model_flops).

    Seed pass, per column-iteration: 64 per local 4x4 block + 44 per local
    orbital (w = z_s p - Hp, mu, s update, rho', ||s||^2, p update); per
    shift-iteration while the shift is active: 28 (pi recurrence and freeze
    test).  Shift pass, per shift-step: 30 (UL pivot: diagonal, one complex
    product, reciprocal, next multiplier) + 8 per projection row (Horner
    step)."""
    nk_sum = nk.sum(axis=1).astype(np.float64)
    seed = float(np.sum(iters * (64.0 * nblk + 44.0 * nl)) + 28.0 * nk_sum.sum())
    shift = float(np.sum(nk_sum * (30.0 + 8.0 * nrow)))
    return seed, shift


def path_bytes(nrow, iters, ns, g_out):
    """Algorithmic HBM bytes of one solve: the seed pass writes, per
    column-iteration, 1/alpha and beta/alpha (32 B) and the residual on the
    projection rows (16 B per row), plus r_0; the shift pass reads that
    history back once and writes G (16 B per row and shift, when kept), rho
    (8 B per row) and per shift the residual (8 B) and the step count (4 B)."""
    hist = float(np.sum(iters * (32.0 + 16.0 * nrow) + 16.0 * nrow))
    out = float(np.sum(nrow) * (8.0 + (16.0 * ns if g_out else 0.0))) + iters.size * ns * 12.0
    return 2.0 * hist + out


def seed_kernel_name(ns, max_row_blocks, stage_lds=-1):
    """The S = I seed kernel the library launches for subspaces of <= 16
    atoms: with the default choice four columns per wavefront (k_seed_q4) up
    to 128 shifts and two (k_seed_q2) up to 256; with stage_lds 5 two; one
    column per wavefront (k_seed_r1) otherwise."""
    b = 5 if max_row_blocks <= 5 else 6 if max_row_blocks <= 6 else 8
    ns_pad = (ns + 63) // 64 * 64
    if stage_lds == -1 and ns_pad <= 128:
        return f"k_seed_q4<{ns_pad // 16}, {b}>"
    if stage_lds in (-1, 5) and ns_pad <= 256:
        return f"k_seed_q2<{4 if ns_pad <= 128 else 8}, {b}>"
    m = (ns + 63) // 64
    m = {1: 1, 2: 2, 3: 4, 4: 4}.get(m, 8)
    return f"k_seed_r1<{m}, {b}>"


def shift_kernel_name(max_proj_atoms):
    return f"k_shift<{min(max(max_proj_atoms, 1), 8)}, 1>"


def solve_figures(prep, res, ns, seed_ms, shift_ms, g_out, stage_lds=-1):
    """Roofline figures of one S = I solve from its plan and per-column
    counts: the seed pass against the FP64 vector peak (seed-operator flops
    only), the whole path (both passes, both flop terms), the kernels'
    executed count, and the algorithmic HBM bytes of the path."""
    plan = prep.plan
    cp = prep.col_plan.cpu().numpy()
    nl = 4 * np.diff(plan.atom_off.cpu().numpy())[cp]
    nblk = np.diff(plan.blk_off.cpu().numpy())[cp]
    nrow = 4 * np.diff(plan.pa_off.cpu().numpy())[cp]
    iters = res.iters.cpu().numpy().astype(np.float64)
    nk = res.shift_iters.cpu().numpy()
    a4, a8 = model_flops(nblk, nrow, iters, nk)
    e_seed, e_shift = executed_flops(nblk, nl, nrow, iters, nk)
    nbytes = path_bytes(nrow, iters, ns, g_out)
    t = plan.totals
    seed_tf = a4 / (seed_ms * 1e-3) / 1e12
    whole_tf = (a4 + a8) / ((seed_ms + shift_ms) * 1e-3) / 1e12
    r1 = t.max_loc_atoms <= 16 and t.max_row_blocks <= 8
    return {
        "seed_kernel": (seed_kernel_name(ns, t.max_row_blocks, stage_lds) if r1 and stage_lds in (-1, 3, 5)
                        else "k_seed (LDS-staged or global operator)"),
        "shift_kernel": shift_kernel_name(t.max_proj_atoms),
        "column_iterations": float(iters.sum()), "active_shift_steps": float(nk.sum()),
        "mean_local_blocks": float(nblk.mean()), "mean_local_orbitals": float(nl.mean()),
        "mean_projection_rows": float(nrow.mean()),
        "seed_pass": {"ms": seed_ms, "tflop": a4 / 1e12, "tflops": seed_tf, "frac": seed_tf / PEAK_FP64_TFLOPS,
                      "flop_model": "64 per local 4x4 block per column-iteration"},
        "whole_path": {"ms": seed_ms + shift_ms, "tflop": (a4 + a8) / 1e12, "tflops": whole_tf,
                       "frac": whole_tf / PEAK_FP64_TFLOPS,
                       "flop_model": "64 per local block per column-iteration + 16 per projection row per "
                                     "active shift-step"},
        "executed": {"seed_tflop": e_seed / 1e12, "shift_tflop": e_shift / 1e12,
                     "seed_tflops": e_seed / (seed_ms * 1e-3) / 1e12,
                     "shift_tflops": e_shift / (shift_ms * 1e-3) / 1e12},
        "hbm_algorithmic": {"bytes": nbytes, "GBps": nbytes / ((seed_ms + shift_ms) * 1e-3) / 1e9,
                            "frac": nbytes / ((seed_ms + shift_ms) * 1e-3) / 1e9 / PEAK_HBM_GBS},
    }


def roofline_line(fig, seed_ms, shift_ms, launches, traffic_seed, traffic_shift, hbm_counted):
    """The bench line's roofline object: the longer of the two passes (the
    dominant kernel) at its algorithmic flop rate (model_flops) against the
    FP64 vector peak, timed live per launch with HIP events on the solve
    stream; the whole path and the HBM figures beside it."""
    seed_dom = seed_ms >= shift_ms
    if seed_dom:
        kernel, ms, tflop, model = fig["seed_kernel"], seed_ms, fig["seed_pass"]["tflop"], fig["seed_pass"]["flop_model"]
        traffic = traffic_seed
    else:
        tflop = fig["whole_path"]["tflop"] - fig["seed_pass"]["tflop"]
        kernel, ms, model = fig["shift_kernel"], shift_ms, "16 per projection row per active shift-step"
        traffic = traffic_shift
    achieved = tflop / (ms * 1e-3)   # per launch: (tflop / launches) / (ms / launches)
    return {
        "kernel": kernel, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_TFLOPS,
        "traffic": traffic,
        "traffic_source": "recorded FETCH_SIZE + WRITE_SIZE per launch for this kernel source (not measured in "
                          "this run)" if traffic is not None else "no counter record for this kernel source",
        "flop_model": model, "launches_per_step": launches, "ms_per_launch": ms / launches,
        "passes": {"seed": fig["seed_pass"], "shift_ms": shift_ms},
        "whole_path": fig["whole_path"],
        "executed_flops": fig["executed"],
        "hbm": {"algorithmic": fig["hbm_algorithmic"], "counters": hbm_counted},
        "per_column": {k: fig[k] for k in ("column_iterations", "active_shift_steps", "mean_local_blocks",
                                            "mean_local_orbitals", "mean_projection_rows")},
    }


def train_scheduler(sgf, W, dev, n_logged=50000, kind="bundle"):
    """The learned scheduler's setup (outside the timed region): log the
    iteration counts of n_logged solves of a differently seeded workload of
    the same shape (kind "bundle": the S = I bundle; "overlap": the overlap
    bundle with its radius per column), then train the iteration-count
    network on them with the library's own kernels."""
    import torch
    if kind == "overlap":
        tw = W.config_bundle_overlap(config_no=30)
    else:
        tw = W.config_bundle(config_no=20)
    pick = np.sort(np.random.default_rng(5).choice(tw.columns.size, n_logged, replace=False))
    cols = tw.columns[pick]
    rpc = None if tw.radius_per_col is None else tw.radius_per_col[pick]
    ts = sgf.system_for(tw)
    tp = sgf.prepare(ts, cols, radius=tw.radius, radius_per_col=rpc, prune=True)
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


CSRC = os.path.join(ROOT, "paper_1603_09616_amd", "csrc")


def kernel_fingerprint(kind):
    """sha256 over the source a kernel is built from: its own function text
    (for the solver passes) or file, and the shared device helpers.  Counter
    figures recorded in profiles/ apply only while this matches."""
    import hashlib
    import re
    common = open(os.path.join(CSRC, "common.hpp")).read()
    if kind != "apply":  # the solver passes also depend on their shared header (layout, chunk sizes)
        common += open(os.path.join(CSRC, "scocg.hpp")).read()
    if kind == "apply":
        text = open(os.path.join(CSRC, "apply.hip")).read()
    else:
        src = open(os.path.join(CSRC, "scocg.hip")).read()
        head = {"seed": r"template <int M, int BMAX>\n__global__ __launch_bounds__\(SEED_T\) void k_seed_r1",
                "seed_q4": r"template <int M4, int BMAX>\n__global__ __launch_bounds__\(SEED_T\) void k_seed_q4",
                "shift": r"template <int NPA, int MS>\n__global__ __launch_bounds__\(512\)[^\n]* void k_shift"}[kind]
        m = re.search(head, src)
        if m is None:
            return None
        start = m.start()
        if kind == "seed_q4":   # with the row-sum helper and constants in front of it
            h = src.find("constexpr int Q4_HS")
            start = h if 0 <= h < start else start
        end = src.find("\n}\n", m.start())
        text = src[start:end + 3]
    return hashlib.sha256((text + common).encode()).hexdigest()


def recorded_traffic(kernel, kind):
    """HBM bytes per launch from the committed counter record, scaled by the
    copy reference; None when absent or when the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("fingerprint") != kernel_fingerprint(kind):
        return None
    sc = rec["copy_reference"]
    return k["fetch_kib"] * 1024 * sc["fetch_scale"] + k["write_kib"] * 1024 * sc["write_scale"]


def record_traffic(dirs):
    """Write profiles/pmc_traffic.json from four rocprofv3 --pmc CSV folders:
    FETCH_SIZE and WRITE_SIZE of one bench step (the solver passes: the
    second dispatch of each, the full bundle, after the scheduler's training
    solve) and of `--spmv-only` (the operator apply, mean over its
    dispatches, and the ten 1 GiB copies that scale the counters).  Each
    kernel's entry carries the fingerprint of the source it was measured
    on; recorded_traffic() ignores it once the source changes."""
    import collections
    import csv
    import glob
    import re
    mf, mw, sf, sw = dirs.split(",")

    def load(d):
        out = collections.defaultdict(list)
        for f in sorted(glob.glob(os.path.join(d, "*counter_collection.csv"))):
            rows = sorted(csv.DictReader(open(f)), key=lambda r: int(r["Dispatch_Id"]))
            for r in rows:
                out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return out

    F, Wr, SF, SW = load(mf), load(mw), load(sf), load(sw)
    cf = [v for v in SF["__amd_rocclr_copyBuffer"] if v > 1000]
    cw = [v for v in SW["__amd_rocclr_copyBuffer"] if v > 1000]
    sc = {"bytes": 1 << 30, "dispatches": len(cf), "fetch_kib": sum(cf) / len(cf), "write_kib": sum(cw) / len(cw)}
    sc["fetch_scale"] = (1 << 20) / sc["fetch_kib"]
    sc["write_scale"] = (1 << 20) / sc["write_kib"]
    kernels = {}
    for name, vals in F.items():
        kind = ("seed_q4" if ("k_seed_q4<" in name or "k_seed_q2<" in name) else "seed" if "k_seed_r1<" in name else
                "shift" if "k_shift<" in name else None)
        if kind is None or len(vals) < 2 or len(Wr.get(name, [])) < 2:
            continue
        short = re.search(r"(k_\w+<[^>]*>)", name).group(1)
        kernels[short] = {"launch": "full bundle, 473,200 columns, one launch (second dispatch of the run)",
                          "fetch_kib": vals[1], "write_kib": Wr[name][1], "fingerprint": kernel_fingerprint(kind)}
    for name, vals in SF.items():
        if "k_bsr_apply" not in name or name not in SW:
            continue
        short = re.search(r"(k_\w+<[^>]*>)", name).group(1)
        kernels[short] = {"launch": f"1,000,300-atom operator, mean of {len(vals)} dispatches",
                          "fetch_kib": sum(vals) / len(vals), "write_kib": sum(SW[name]) / len(SW[name]),
                          "fingerprint": kernel_fingerprint("apply")}
    for v in kernels.values():
        v["traffic_bytes"] = v["fetch_kib"] * 1024 * sc["fetch_scale"] + v["write_kib"] * 1024 * sc["write_scale"]
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    json.dump({"copy_reference": sc, "kernels": kernels}, open(path, "w"), indent=1)
    for k, v in kernels.items():
        print(f"{k}: {v['traffic_bytes'] / 1e9:.3f} GB per launch")


def hbm_stream(sgf, W, dev, reps=50):
    """The global operator apply y = (z - H) x on the 1,000,300-atom share
    (570 MB of FP64 blocks, larger than the 256 MB last-level cache), timed
    with HIP events over `reps` launches per case on the launch stream.
    Algorithmic bytes per launch: the blocks, their column indices and row
    pointers once, x read once and y written once."""
    import torch
    wl = W.config_large(n_columns=16)
    s = sgf.system_for(wl)
    s.add_f32()
    n = 4 * s.n_atoms
    z = complex(wl.z[128])
    g = torch.Generator(device=dev).manual_seed(3)
    cases = {}
    for prec, dt, bc, dtn in (("fp64", torch.float64, 16, "double"), ("fp32", torch.float32, 8, "float")):
        for k in (1, 4, 8):
            x = torch.complex(torch.randn((n, k), dtype=dt, device=dev, generator=g),
                              torch.randn((n, k), dtype=dt, device=dev, generator=g)).contiguous()
            y = torch.empty_like(x)
            for _ in range(3):
                sgf.bsr_apply(s, z, x, prec, out=y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                sgf.bsr_apply(s, z, x, prec, out=y)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = s.nnzb * (16 * bc // 2 + 4) + (s.n_atoms + 1) * 4 + 2 * n * k * bc
            rpt = 2 if k == 8 or (k == 4 and prec == "fp32") else 1
            name = (f"k_bsr_apply<{dtn}, 1, false>" if k == 1 else
                    f"k_bsr_apply_lx<{dtn}, {k}, {rpt}, false>")
            traffic = recorded_traffic(name, "apply")
            cases[f"{prec}_rhs{k}"] = {"ms": ms, "bytes": nbytes, "GBps": nbytes / ms / 1e6,
                                       "frac": nbytes / ms / 1e6 / PEAK_HBM_GBS, "traffic": traffic,
                                       "traffic_GBps": None if traffic is None else traffic / ms / 1e6}
            log(f"[bench] bsr_apply {prec} x{k}: {ms * 1e3:.1f} us, {nbytes / ms / 1e6:.0f} GB/s")
            del x, y
    best = max(cases, key=lambda c: cases[c]["GBps"])
    return {"kernel": "k_bsr_apply", "workload": "y = (z - H) x on the 1,000,300-atom bundle share "
            f"({s.n_atoms} block rows, {s.nnzb} 4x4 blocks)", "peak_GBps": PEAK_HBM_GBS, "reps": reps,
            "cases": cases, "best": best, "best_frac": cases[best]["frac"]}


def wp_stream(sgf, W, dev, steps=10):
    """Wavepacket propagation (Chebyshev steps of exp(-i H h / hbar), h = 0.1
    fs) on the 1,000,300-atom share, 1 and 8 packets, `steps` steps timed with
    HIP events after one warm-up step.  Algorithmic bytes per step: each of
    the K series terms reads the blocks, their column indices and row
    pointers once, plus the vectors it streams (first term: T_0 read, T_1 and
    the sum written; middle terms: T_k read, T_{k-1} read and written, the sum
    read and written; last term: T_k read, T_{k-1} read and written, the sum
    read)."""
    import torch
    wl = W.config_large(n_columns=16)
    s = sgf.system_for(wl)
    n = 4 * s.n_atoms
    lo, hi = sgf.wp_bounds(s)
    a_tau = 0.5 * (hi - lo) * 0.1 / sgf.HBAR_EV_FS
    K = sgf.wp_terms(a_tau, 1e-13)
    cases = {}
    for k in (1, 8):
        psi0 = torch.as_tensor(W.wavepacket(wl, k), device=dev)
        psi = (psi0[:, 0] if k == 1 else psi0).contiguous().clone()
        sgf.wp_propagate(s, psi, 0.1, 1, lo, hi, K)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sgf.wp_propagate(s, psi, 0.1, steps, lo, hi, K)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        mat = s.nnzb * (128 + 4) + (s.n_atoms + 1) * 4
        vec = n * k * 16
        nbytes = K * mat + vec * (3 + 5 * (K - 3) + 4)
        norm = torch.linalg.vector_norm(psi.reshape(n, k), dim=0).cpu().numpy()
        cases[f"rhs{k}"] = {"ms_per_step": ms, "terms": K, "bytes_per_step": nbytes, "GBps": nbytes / ms / 1e6,
                            "frac": nbytes / ms / 1e6 / PEAK_HBM_GBS, "fs_per_s": 0.1 / (ms * 1e-3),
                            "norm_drift": float(np.abs(norm - 1).max())}
        log(f"[bench] wavepacket x{k}: {ms:.2f} ms per 0.1 fs step ({K} terms), {nbytes / ms / 1e6:.0f} GB/s")
        del psi, psi0
    return {"kernel": "k_cheb_term (1 packet), k_cheb_term_atom (8 packets)", "workload": "wavepacket steps of 0.1 fs on the 1,000,300-atom bundle share "
            f"({s.n_atoms} block rows, {s.nnzb} 4x4 blocks), Gershgorin bounds [{lo:.2f}, {hi:.2f}] eV",
            "peak_GBps": PEAK_HBM_GBS, "steps": steps, "cases": cases}


def extra_workloads(sgf, W, dev, ws_gib, check_n, reps=5, only=None, models=None,
                    graph_cases=("bundle_overlap_uneven",), plain_cases=("bundle_overlap_uneven",),
                    plain_cols=16384, mixed_cases=("large_share",)):
    """The other workloads, each a warm-up solve and then `reps` timed solves
    (median), with the seed and shift passes timed per launch by HIP events:

    chain: the 2000-site chain, 16 columns on the whole system, 64 shifts;
    bundle_unpruned: the bundle with unpruned R = 1.0 nm subspaces (~126
      atoms, ~505 orbitals), all 473,200 columns, 128 shifts;
    bundle_overlap_uneven: the overlap bundle (S != I, per-column radius
      U[0.6, 1.4] nm, 256 shifts, all 473,200 columns);
    large_share: the 1,000,300-atom share (256 shifts, all 4,001,200 columns,
      density matrix only: G alone would be 328 GB) in streamed launches.

    All FP64 at the workloads' own tolerances, in workspace-sized launches.
    A workload with a trained iteration-count network in `models` is also
    timed in the learned order (features, prediction and the grouped order
    inside the timed region), `reps` solves after a warm-up, and the gain
    over the natural order reported; the results of the two orders are
    checked to be the same bits.  Returns the timings and, per workload, the
    outputs of `check_n` seeded columns (all of them for the chain) for the
    oracle comparison.  The workloads in `graph_cases` are also timed as
    replays of that solve captured into a HIP graph, and those in
    `plain_cases` in fixed launches of `plain_cols` columns, natural order
    against the learned one (median of 2 after a warm-up); those in
    `mixed_cases` also run once on the mixed-precision path."""
    import torch
    out, keep = {}, {}
    cases = (("chain", W.config_chain(), True, True, "2000-site chain (S = I, whole system)"),
             ("bundle_unpruned", W.config_bundle(), True, False,
              "bundle, R = 1.0 nm unpruned subspaces (S = I)"),
             ("bundle_overlap_uneven", W.config_bundle_overlap(), True, True,
              "bundle (S != I, radius per column U[0.6, 1.4] nm)"),
             ("large_share", W.config_large(), False, True, "bundle (1,000,300 atoms)"))
    for name, wl, g_out, prune, what in cases:
        if only is not None and name not in only:
            continue
        s = sgf.system_for(wl)
        prep = sgf.prepare(s, wl.columns, radius=wl.radius, radius_per_col=wl.radius_per_col, prune=prune)
        ns = wl.z.size
        batch = sgf.batch_limit(prep, ns, int(ws_gib * (1 << 30)))
        buf = None
        n_reps = reps if name != "bundle_unpruned" else max(2, reps // 2)
        times, seeds, shifts = [], [], []
        for rep in range(n_reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=g_out, batch_cols=batch, out=buf,
                                     profile=True, shift_iters=True)
            prof = sgf.solve_profile()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            buf = res._out
            if rep:
                times.append(ms)
                seeds.append(prof[0])
                shifts.append(prof[1])
            log(f"[bench] {name}: {'warm-up' if rep == 0 else f'rep {rep}/{n_reps}'} {ms:.1f} ms")
        ms, seed_ms, shift_ms = (float(np.median(v)) for v in (times, seeds, shifts))
        st = res.status.cpu().numpy()
        conv = int(np.sum(res.resid.cpu().numpy() <= wl.tol))
        t = prep.plan.totals
        out[name] = {"workload": wl.name + " " + what if wl.kind != "chain" else what,
                     "atoms": int(wl.n_orb if wl.kind == "chain" else wl.n_atoms), "columns": int(wl.columns.size), "shifts": int(ns), "tol": wl.tol,
                     "pruned": prune, "outputs": "G and rho" if g_out else "rho only", "reps": n_reps,
                     "ms": ms, "ms_all_reps": times, "solves_per_s": conv / (ms * 1e-3),
                     "seed_ms": seed_ms, "shift_ms": shift_ms, "launches": prof[2], "batch_cols": int(batch),
                     "columns_not_converged": int(np.sum(st != 0)),
                     "iters_mean": float(res.iters.float().mean()), "max_loc_atoms": int(t.max_loc_atoms)}
        if not wl.tb or not wl.tb.overlap:
            fig = solve_figures(prep, res, ns, seed_ms, shift_ms, g_out)
            out[name]["roofline"] = {"kernel": fig["seed_kernel"] if seed_ms >= shift_ms else fig["shift_kernel"],
                                     "seed_pass": fig["seed_pass"], "whole_path": fig["whole_path"],
                                     "hbm_algorithmic": fig["hbm_algorithmic"], "executed": fig["executed"]}
        else:
            cp = prep.col_plan.cpu().numpy()
            nl = 4 * np.diff(prep.plan.atom_off.cpu().numpy())[cp].astype(np.float64)
            nblk = np.diff(prep.plan.blk_off.cpu().numpy())[cp].astype(np.float64)
            it = res.iters.cpu().numpy().astype(np.float64)
            # w = z_s q - H p: 64 per local block (q = S p comes from its own
            # recurrence); r = S_L^{-1} s: a real n_L x n_L matrix times a
            # complex vector, 4 n_L^2, or with blocks s_ab I4 the per-atom
            # inverse (S_a^{-1} (x) I4), 4 n_L (n_L / 4) = n_L^2
            per_atom = bool(prep.system.s_orbital_diagonal)
            f = float(np.sum(it * (64.0 * nblk + (1.0 if per_atom else 4.0) * nl * nl)))
            out[name]["roofline"] = {"seed_pass": {"ms": seed_ms, "tflop": f / 1e12,
                                                   "tflops": f / (seed_ms * 1e-3) / 1e12,
                                                   "frac": f / (seed_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                                                   "flop_model": "64 per local block (H p) + "
                                                                 + ("n_L^2 (per-atom S^-1 s)" if per_atom else
                                                                    "4 n_L^2 (orbital S_L^-1 s)")
                                                                 + " per column-iteration",
                                                   "kernel": "k_seed_kr" if per_atom else "k_seed_gen2s / k_seed_gen2"}}
        log(f"[bench] {name}: {wl.columns.size} columns x {ns} shifts in {ms:.1f} ms (median of {n_reps}; "
            f"{conv / (ms * 1e-3):.3g} solves/s, {prof[2]} launches)")
        if models and name in models:
            lt = []
            rho_nat = res.rho.clone()
            for rep in range(n_reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                order = sgf.learned_order(prep, models[name])
                res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=g_out, batch_cols=batch, out=buf,
                                         order=order, shift_iters=True)
                torch.cuda.synchronize()
                if rep:
                    lt.append((time.perf_counter() - t0) * 1e3)
            same = bool(torch.equal(res.rho, rho_nat))
            lms = float(np.median(lt))
            out[name]["learned_order"] = {"ms": lms, "ms_all_reps": lt, "gain_vs_natural": ms / lms,
                                          "rho_bitwise_equal": same}
            log(f"[bench] {name}: learned order {lms:.1f} ms (gain {ms / lms:.4f} over natural order; "
                f"rho bitwise equal: {same})")
            if name in mixed_cases:
                # the mixed path on this workload (complex-FP32 Krylov vectors,
                # FP64 scalars, FP64 true-residual monitor every 50
                # iterations), columns it does not certify re-solved in FP64;
                # one solve, its diagonal density-matrix entries checked
                # against the oracle
                torch.cuda.empty_cache()
                mb = sgf.batch_limit(prep, ns, int(ws_gib * (1 << 30)), precision="mixed")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rm = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-5, precision="mixed", g_out=g_out,
                                        batch_cols=mb, monitor_every=50, profile=True)
                torch.cuda.synchronize()
                mms = (time.perf_counter() - t0) * 1e3
                stm = rm.status.cpu().numpy()
                acc_cols = int(np.sum((stm == sgf.CONVERGED) | (stm == sgf.DIAG_ONLY)))
                out[name]["mixed"] = {"ms": mms, "tol": 1e-5, "monitor_every": 50, "batch_cols": int(mb),
                                      "fp64_fallback_columns": int(rm.n_fallback),
                                      "columns_accepted": acc_cols,
                                      "solves_per_s": acc_cols * ns / (mms * 1e-3)}
                log(f"[bench] {name}: mixed {mms:.0f} ms ({int(rm.n_fallback)} of {wl.columns.size} columns "
                    f"re-solved in FP64)")
                mpick = np.sort(np.random.default_rng(1603).choice(wl.columns.size, min(check_n, wl.columns.size),
                                                                   replace=False))
                moff = prep.proj_off.cpu().numpy()
                mrows = np.concatenate([np.arange(moff[c], moff[c + 1]) for c in mpick])
                keep[name + "_mixed"] = (wl, mpick, None, rm.rho[torch.as_tensor(mrows, device=dev)].cpu().numpy(),
                                         stm[mpick], prune)
                del rm
                torch.cuda.empty_cache()
            if name in plain_cases:
                # fixed launches of plain_cols columns (each waits for its
                # slowest column): natural order against the learned one
                pt = {"natural": [], "learned": []}
                for mode in ("natural", "learned"):
                    for rep in range(3):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        od = sgf.learned_order(prep, models[name]) if mode == "learned" else None
                        res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=g_out,
                                                 batch_cols=min(plain_cols, batch), out=buf, order=od)
                        torch.cuda.synchronize()
                        if rep:
                            pt[mode].append((time.perf_counter() - t0) * 1e3)
                pn, pl_ = float(np.median(pt["natural"])), float(np.median(pt["learned"]))
                out[name]["plain_launches"] = {"batch_cols": int(min(plain_cols, batch)), "natural_ms": pn,
                                               "learned_ms": pl_, "gain_vs_natural": pn / pl_,
                                               "rho_bitwise_equal": bool(torch.equal(res.rho, rho_nat))}
                log(f"[bench] {name}: launches of {min(plain_cols, batch)} columns: natural {pn:.1f} ms, "
                    f"learned {pl_:.1f} ms (gain {pn / pl_:.4f})")
            if name in graph_cases:
                # the same solve (learned order) captured once into a HIP graph
                # and replayed: kernel launches only, on the solve's own buffers
                gr = sgf.SolveGraph(prep, wl.z, wl.w, tol=wl.tol, order=order, out=buf, g_out=g_out,
                                    batch_cols=batch)
                gt = []
                for rep in range(n_reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    gr.replay()
                    torch.cuda.synchronize()
                    if rep:
                        gt.append((time.perf_counter() - t0) * 1e3)
                    if rep == 1:
                        # eager work between replays (a graph must not depend on what ran before it)
                        sgf.learned_order(prep, models[name])
                gsame = bool(torch.equal(gr.result.rho, rho_nat))
                gms = float(np.median(gt))
                out[name]["graph_replay"] = {"ms": gms, "ms_all_reps": gt, "rho_bitwise_equal": gsame,
                                             "what": "solve in the learned order captured into one HIP graph "
                                                     "(ticket clears, seed and shift passes of every batch)"}
                log(f"[bench] {name}: HIP-graph replay {gms:.1f} ms (rho bitwise equal: {gsame})")
                res = gr.result
                del gr
            del rho_nat
        if wl.tb and wl.tb.overlap:
            out[name]["after_rho"] = overlap_forces(sgf, prep, res, wl)
        n_check = wl.columns.size if name == "chain" else min(check_n, wl.columns.size)
        pick = np.sort(np.random.default_rng(1603).choice(wl.columns.size, n_check, replace=False))
        if name == "bundle_unpruned":
            pick = pick[:64]
        off = prep.proj_off.cpu().numpy()
        rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in pick])
        idx = torch.as_tensor(rows, device=dev)
        keep[name] = (wl, pick, None if res.G is None else res.G[idx].cpu().numpy(), res.rho[idx].cpu().numpy(),
                      st[pick], prune)
        del res, buf, prep, s
        torch.cuda.empty_cache()
    return out, keep


def overlap_forces(sgf, prep, res, wl, reps=3):
    """After an S != I solve that kept G: the energy-density matrix
    eps = -(1/pi) sum_k Im(w_k z_k G(z_k)) on every projection row (one HBM
    pass over G), the band forces with its term, and the whole-solve
    identity tr(eps S) = tr(rho H) (from the traces of rho and of eps)."""
    import dataclasses
    import torch

    def timed(fn):
        ts, r = [], None
        for i in range(reps + 1):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn()
            e1.record()
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1))
        return r, float(np.median(ts))

    n_rows, ns = int(prep.n_rows), int(res.G.shape[1])
    eps, e_ms = timed(lambda: sgf.energy_density(res, wl.z, wl.w))
    F, f_ms = timed(lambda: sgf.band_forces(prep, res, wl.tb, eps=eps))
    alg = n_rows * ns * 16 + n_rows * 8
    _, _, (_, rho_h) = sgf.traces(prep, dataclasses.replace(res, G=None))
    _, _, (eps_s, _) = sgf.traces(prep, dataclasses.replace(res, G=None, rho=eps))
    Fh = F.cpu().numpy()
    log(f"[bench] energy density {e_ms:.2f} ms ({alg / (e_ms * 1e-3) / 1e12:.2f} TB/s), forces {f_ms:.2f} ms, "
        f"tr(eps S) - tr(rho H) = {eps_s - rho_h:.2e}")
    return {"energy_density": {"ms": e_ms, "alg_bytes": alg, "GBps": alg / (e_ms * 1e-3) / 1e9,
                               "frac_of_8TBps": alg / (e_ms * 1e-3) / 8e12},
            "band_forces": {"ms": f_ms, "rows_per_s": n_rows / (f_ms * 1e-3),
                            "max_abs_eV_per_nm": float(np.abs(Fh).max()),
                            "sum_over_atoms_max": float(np.abs(Fh.sum(axis=0)).max())},
            "tr_eps_S": eps_s, "tr_rho_H_eV": rho_h, "identity_gap": eps_s - rho_h, "reps": reps}


def check_extra(keep):
    """Oracle results for the sampled columns of the extra workloads (part of
    the CPU-baseline leg) and the errors of the GPU outputs against them."""
    import oracle
    threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", 1 << 30)))
    acc = {}
    for name, (wl, pick, G, rho, st, prune) in keep.items():
        b = oracle.system_for(wl)
        t0 = time.perf_counter()
        ref = oracle.solve_workload(wl, b, cols=wl.columns[pick], prune=prune, threads=threads)
        dt = time.perf_counter() - t0
        a = {"columns": int(pick.size), "oracle_s": dt, "oracle_threads": threads}
        e_rho = e_g = e_jj = e_rjj = 0.0
        for i in range(pick.size):
            lo, hi = ref.proj_ptr[i], ref.proj_ptr[i + 1]
            e_rho = max(e_rho, np.abs(rho[lo:hi] - ref.rho[lo:hi]).max() / max(np.abs(ref.rho[lo:hi]).max(), 1e-300))
            d = lo + int(np.nonzero(ref.proj_row[lo:hi] == wl.columns[pick[i]])[0][0])
            e_rjj = max(e_rjj, abs(rho[d] - ref.rho[d]) / max(np.abs(ref.rho[lo:hi]).max(), 1e-300))
            if G is not None:
                e_g = max(e_g, np.abs(G[lo:hi] - ref.G[lo:hi]).max() / np.abs(ref.G[lo:hi]).max())
                d = lo + int(np.nonzero(ref.proj_row[lo:hi] == wl.columns[pick[i]])[0][0])
                e_jj = max(e_jj, float((np.abs(G[d] - ref.G[d]) / np.abs(ref.G[d])).max()))
        a["rho_normwise"] = e_rho
        a["rho_jj"] = e_rjj
        if G is not None:
            a["G_rows_normwise"] = e_g
            a["G_jj_worst_shift"] = e_jj
        if name.endswith("_mixed"):   # accepted mixed columns end DIAG_ONLY (only G_jj, rho_jj certified)
            a["not_accepted"] = int(np.sum((st != 0) & (st != 6)))
        else:
            a["not_converged"] = int(np.sum(st != 0))
            a["status_equal"] = bool(np.array_equal(st, ref.status))
        acc[name] = a
        log(f"[bench] {name}: oracle on {pick.size} columns in {dt:.1f} s; rho err {e_rho:.2e}")
    return acc


def copy_reference(dev, nbytes=1 << 30, reps=10):
    """A plain device copy of known size (for scaling HBM counters)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "launches": reps}


def after_rho(sgf, prep, res, wl, reps=5):
    """The steps after rho on the timed step's outputs: the traces of the
    projected G (an HBM-bound pass that streams all of G once), then the
    half-filling Fermi level, electron count and band energy from them, the
    row identity z_k T_k - U_k = n_cols as a check, and the band forces
    -dE_band/dR at fixed rho."""
    import torch
    n_rows, ns = int(prep.n_rows), int(res.G.shape[1])
    ms = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        T, U, (ts, th) = sgf.traces(prep, res)
        e1.record()
        torch.cuda.synchronize()
        if r:
            ms.append(e0.elapsed_time(e1))
    n = int(prep.cols.numel())
    g_bytes = n_rows * ns * 16
    # G once; per row the coefficient written and read back (16 + 16 B) and its proj_row entry
    alg = g_bytes + n_rows * (16 + 16 + 4) + n * (8 + 8 + 4)
    t = float(np.median(ms))
    mu, ne, eb = sgf.fermi_level(wl.z, T, U, 0.5 * n)
    # band forces -dE_band/dR at fixed rho from the same step
    fms = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        F = sgf.band_forces(prep, res, wl.tb)
        e1.record()
        torch.cuda.synchronize()
        if r:
            fms.append(e0.elapsed_time(e1))
    Fh = F.cpu().numpy()
    return {"what": "T_k = sum_j (G S)_jj, U_k = sum_j (G H)_jj over all columns, then the half-filling Fermi level",
            "ms": t, "G_bytes": g_bytes, "alg_bytes": alg, "GBps": alg / (t * 1e-3) / 1e9,
            "frac_of_8TBps": alg / (t * 1e-3) / 8e12, "reps": reps,
            "identity_gap_max": float(np.abs(wl.z * T - U - n).max()), "identity_bound": 10 * wl.tol * n,
            "mu_half_filling_eV": mu, "n_e": ne, "e_band_eV": eb, "tr_rho_S": ts, "tr_rho_H_eV": th,
            "band_forces": {"ms": float(np.median(fms)), "rows_per_s": n_rows / (float(np.median(fms)) * 1e-3),
                            "max_abs_eV_per_nm": float(np.abs(Fh).max()),
                            "sum_over_atoms_max": float(np.abs(Fh.sum(axis=0)).max())}}


def qmd_steps(sgf, wl, steps=5, h_fs=0.1, ws_budget=24 << 30):
    """Quantum molecular dynamics on the bundle: velocity-Verlet steps, each
    one the whole path at the moved positions (neighbour list and H, local
    subspaces, the shifted solve of all 473,200 columns with rho only, band
    forces) plus the two kicks and the drift.  Carbon masses, seeded thermal
    velocities (300 K).  The band forces have no repulsive partner here, so
    the jittered close pairs (down to 0.034 nm, forces near 1e4 eV/nm) pull
    together; at the paper's 1 fs step they merge chains within one step and
    the subspaces grow, so the steps are 0.1 fs, over which the subspaces
    keep their shape.  Timed with wall clock around each step after one
    warm-up step.  The solve runs in launches of what ws_budget holds, so
    that its workspace fits beside the timed step's buffers."""
    import torch
    n = wl.n_atoms
    kT = 8.617333262e-5 * 300.0                        # eV
    sigma_v = np.sqrt(kT / 12.011 * sgf.ACCEL_EV_NM_AMU)   # nm/fs
    vel = np.random.default_rng(1603).normal(size=(n, 3)) * sigma_v
    run = sgf.QMD(wl.xyz, vel, np.full(n, 12.011), wl.tb, wl.z, wl.w, tol=wl.tol, radius=wl.radius,
                  ws_budget=ws_budget)
    run.step(h_fs)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        run.step(h_fs)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(ts))
    moved = float((run.xyz.cpu() - torch.as_tensor(wl.xyz)).abs().max())
    st = run.last[1].status.cpu().numpy()
    t = run.last[0].plan.totals
    log(f"[bench] QMD: {ms:.1f} ms per {h_fs} fs step ({n} atoms, {4 * n} columns, subspaces <= "
        f"{t.max_loc_atoms} atoms)")
    return {"what": f"velocity-Verlet steps of {h_fs} fs, each the whole path at the new positions plus the band "
                    "forces (no repulsive term)",
            "atoms": int(n), "columns": int(4 * n), "h_fs": h_fs, "ms_per_step": ms, "steps": steps,
            "fs_per_s": h_fs / (ms * 1e-3), "max_displacement_nm": moved, "max_loc_atoms": int(t.max_loc_atoms),
            "columns_not_converged": int(np.sum(st != 0))}


def fermi_poles_leg(sgf, W, dev, ws_gib, kT=0.1, mu=0.0, n_poles=48, reps=5, check_n=300):
    """Fewer shifts: the bundle's 473,200 columns with the 49 shifts of the
    Fermi-Dirac pole expansion at kT = 0.1 eV (seed at the pole nearest the
    real axis), timed like the other workloads.  Returns the timings and the
    rho of `check_n` seeded columns from these shifts and from the real-axis
    grid (the headline step's 128 shifts), which the CPU-baseline leg checks
    against the plain definition f(H_L) (check_fermi)."""
    import torch
    wl = W.config_bundle()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    z, w = sgf.fermi_shifts(n_poles, kT, mu)
    batch = sgf.batch_limit(prep, z.size, int(ws_gib * (1 << 30)))
    buf, times, seeds, shifts = None, [], [], []
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sgf.solve_prepared(prep, z, w, tol=wl.tol, seed_index=-2, batch_cols=batch, out=buf, profile=True)
        prof = sgf.solve_profile()
        torch.cuda.synchronize()
        if rep:
            times.append((time.perf_counter() - t0) * 1e3)
            seeds.append(prof[0])
            shifts.append(prof[1])
        buf = res._out
    ms = float(np.median(times))
    st = res.status.cpu().numpy()
    conv = int(np.sum(res.resid.cpu().numpy() <= wl.tol))
    pick = np.sort(np.random.default_rng(1603).choice(wl.columns.size, check_n, replace=False))
    off = prep.proj_off.cpu().numpy()
    rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in pick])
    rho = res.rho[torch.as_tensor(rows, device=dev)].cpu().numpy()
    grid = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=False, batch_cols=batch)
    rho_grid = grid.rho[torch.as_tensor(rows, device=dev)].cpu().numpy()
    iters_grid = float(grid.iters.float().mean())
    del grid
    out = {"workload": "bundle, all 473,200 columns, R = 1.0 nm pruned, Fermi-Dirac rho at kT = 0.1 eV, mu = 0",
           "shifts": int(z.size), "poles": n_poles, "tol": wl.tol, "ms": ms, "reps": reps, "seed_ms": float(np.median(seeds)),
           "shift_ms": float(np.median(shifts)), "solves_per_s": conv / (ms * 1e-3),
           "iters_mean": float(res.iters.float().mean()), "columns_not_converged": int(np.sum(st != 0)),
           "real_axis_grid": {"shifts": int(wl.z.size), "iters_mean": iters_grid}}
    log(f"[bench] Fermi poles: {z.size} shifts in {ms:.1f} ms, {out['iters_mean']:.1f} iterations "
        f"(real-axis grid: {iters_grid:.1f})")
    del res, buf, prep, s
    torch.cuda.empty_cache()
    return out, (wl, pick, rho, rho_grid, kT, mu)


def check_fermi(keep):
    """CPU-baseline leg: the plain definition rho = f(H_L) (dense
    eigen-decomposition of each sampled column's local subspace, oracle)
    against the pole-expansion rho and the real-axis grid's rho."""
    import oracle
    from oracle import contour
    wl, pick, rho, rho_grid, kT, mu = keep
    b = oracle.system_for(wl)
    poff, _, exact = contour.fermi_rho_columns(b, wl.xyz, wl.columns[pick], kT, mu, radius=wl.radius, prune=True)
    e_pole = e_grid = 0.0
    for i in range(pick.size):
        a, c = poff[i], poff[i + 1]
        sc = np.abs(exact[a:c]).max()
        e_pole = max(e_pole, np.abs(rho[a:c] - exact[a:c]).max() / sc)
        e_grid = max(e_grid, np.abs(rho_grid[a:c] - exact[a:c]).max() / sc)
    log(f"[bench] Fermi poles: rho vs f(H_L) {e_pole:.2e} (real-axis grid {e_grid:.2e})")
    return {"columns": int(pick.size), "poles": e_pole, "real_axis_grid": e_grid}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=0, help="columns per launch (0: as many as --ws-gib holds)")
    ap.add_argument("--ws-gib", type=float, default=112.0, help="solve workspace budget for the automatic batch")
    ap.add_argument("--plain-batch", type=int, default=8192, help="columns per launch of the plain variant")
    ap.add_argument("--no-variants", action="store_true", help="time only the full solver")
    ap.add_argument("--variant-only", default="", help="comma list: time only these variants (no ratios)")
    ap.add_argument("--record-traffic", default="",
                    help="no GPU work: write profiles/pmc_traffic.json from the rocprofv3 CSV folders "
                         "MAIN_FETCH,MAIN_WRITE,SPMV_FETCH,SPMV_WRITE of the FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-g", action="store_true", help="skip writing G (rho only)")
    ap.add_argument("--shifts-per-lane", type=int, default=0)
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-bound operator-apply measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the overlap and 1M-atom workloads")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library default launch (for profiler runs, which distort the tuner's timings)")
    ap.add_argument("--spmv-only", action="store_true",
                    help="only the operator-apply measurement and a 1 GiB copy (for counter passes)")
    ap.add_argument("--wp-only", action="store_true", help="only the wavepacket-propagation measurement")
    ap.add_argument("--only", default="", help="comma-separated subset of the extra workloads (chain, "
                    "bundle_unpruned, bundle_overlap_uneven, large_share)")
    ap.add_argument("--extra-only", action="store_true",
                    help="only the overlap and 1,000,300-atom workloads (one timed solve each)")
    args = ap.parse_args(argv)
    if args.record_traffic:
        record_traffic(args.record_traffic)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every run of this path uses a single MI355X; columns are "
              "independent, so a multi-GPU run shards columns spatially with no communication in the "
              "Krylov loop. Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    import paper_1603_09616_amd as sgf
    import workloads as W
    only = set(x for x in args.only.split(",") if x) or None

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.spmv_only:
        print(json.dumps({"hbm_stream": hbm_stream(sgf, W, dev), "copy": copy_reference(dev)}), flush=True)
        return 0
    if args.wp_only:
        print(json.dumps({"wavepacket": wp_stream(sgf, W, dev)}), flush=True)
        return 0
    if args.extra_only:
        models = {}
        if only is None or "large_share" in only:
            models["large_share"] = train_scheduler(sgf, W, dev)[0]
        if only is None or "bundle_overlap_uneven" in only:
            models["bundle_overlap_uneven"] = train_scheduler(sgf, W, dev, kind="overlap")[0]
        extra, _ = extra_workloads(sgf, W, dev, min(args.ws_gib, 64.0), 1, only=only, models=models)
        print(json.dumps({"other_workloads": extra}), flush=True)
        return 0
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

    s_probe = sgf.build_hamiltonian(d_xyz, wl.tb, device=dev)
    p_probe = sgf.prepare_planned(s_probe, d_cols, d_cp, d_centers, d_radii, prune=True)
    batch = args.batch or sgf.batch_limit(p_probe, ns, int(args.ws_gib * (1 << 30)))
    # launch choices for this workload shape (timed on a 32,768-column sample)
    from paper_1603_09616_amd import autotune
    if args.no_autotune:
        tuned = {"choice": {}, "timings_ms": None}
    else:
        tuned = autotune.tune(p_probe, wl.z, wl.w, wl.tol, use_cache=False, log=log, sample=TUNE_SAMPLE)
    launch = tuned["choice"]
    torch.cuda.empty_cache()
    log(f"[bench] autotuned launch: {launch}")
    log(f"[bench] workload {wl.name}: {wl.n_atoms} atoms, {wl.columns.size} columns, {ns} shifts, "
        f"batch {batch}")

    def make_step(order_mode, batch_cols, precision="fp64", tol=wl.tol, launch_opts=None):
        lo = dict(launch_opts or {})
        lo.setdefault("shifts_per_lane", args.shifts_per_lane)
        out_buf = {}

        def step(profile):
            s = sgf.build_hamiltonian(d_xyz, wl.tb, device=dev)
            prep = sgf.prepare_planned(s, d_cols, d_cp, d_centers, d_radii, prune=True)
            order = None
            if order_mode == "learned":
                order = sgf.learned_order(prep, model)
            res = sgf.solve_prepared(prep, wl.z, wl.w, tol=tol, precision=precision, g_out=not args.no_g,
                                     batch_cols=batch_cols, order=order, out=out_buf.get("out"), profile=profile,
                                     shift_iters=True, **lo)
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

    # columns whose outputs are checked against the oracle (the first chunk of
    # the CPU-baseline sample)
    check_cols = None if args.no_cpu_baseline else baseline_sample(wl)[:1024]
    samples = {}

    def keep_sample(name, prep, res):
        if check_cols is None or res.G is None:
            return
        off = prep.proj_off.cpu().numpy()
        rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in check_cols])
        idx = torch.as_tensor(rows, device=dev)
        samples[name] = (res.G[idx].cpu().numpy(), res.rho[idx].cpu().numpy(), res.status.cpu().numpy()[check_cols])

    ms_step, seed_ms, shift_ms, launches, (s, prep, res) = timed(make_step("learned", batch, launch_opts=launch),
                                                                 args.steps, args.warmup, "fp64 batched+learned")
    iters = res.iters.cpu().numpy().astype(np.float64)
    status = res.status.cpu().numpy()
    resid = res.resid.cpu().numpy()
    converged = int(np.sum(resid <= wl.tol))
    value = converged / (ms_step * 1e-3)
    fig = solve_figures(prep, res, ns, seed_ms, shift_ms, not args.no_g, launch.get("stage_lds", -1))
    traffic_seed = recorded_traffic(fig["seed_kernel"], "seed_q4" if fig["seed_kernel"].startswith(
        ("k_seed_q4", "k_seed_q2")) else "seed")
    traffic_shift = recorded_traffic(fig["shift_kernel"], "shift")
    hbm_counted = None
    if traffic_seed is not None and traffic_shift is not None:
        tb = traffic_seed + traffic_shift
        hbm_counted = {"bytes": tb, "GBps": tb / ((seed_ms + shift_ms) * 1e-3) / 1e9,
                       "frac": tb / ((seed_ms + shift_ms) * 1e-3) / 1e9 / PEAK_HBM_GBS,
                       "source": "FETCH_SIZE and WRITE_SIZE of both passes recorded by rocprofv3 for this kernel "
                                 "source (profiles/pmc_traffic.json), scaled by a 1 GiB copy; not measured in "
                                 "this run"}
    variants = {"fp64_batched_learned": {"ms_per_step": ms_step, "solves_per_s": value, "seed_ms": seed_ms,
                                         "shift_ms": shift_ms, "launches": launches, "batch_cols": batch,
                                         "order": "learned", "tol": wl.tol, "launch": launch}}
    keep_sample("fp64_batched_learned", prep, res)
    post = None
    if res.G is not None:
        post = after_rho(sgf, prep, res, wl)
        log(f"[bench] after rho: traces in {post['ms']:.2f} ms ({post['GBps']:.0f} GB/s), "
            f"mu(half filling) = {post['mu_half_filling_eV']:.4f} eV")
    if post is not None:
        post["qmd"] = qmd_steps(sgf, wl)
    if not args.no_variants:
        rho_ref = res.rho.clone()
        del res, prep, s
        mixed_batch = args.batch or sgf.batch_limit(p_probe, ns, int(args.ws_gib * (1 << 30)), precision="mixed")
        specs = [("fp64_batched", "natural", batch, "fp64", wl.tol, launch),
                 # one column per wavefront, rows in registers: the FP64 form of the
                 # mixed path's seed kernel (the same mapping)
                 ("fp64_batched_register_rows", "natural", batch, "fp64", wl.tol, {"stage_lds": 3}),
                 ("fp64_plain", "natural", args.plain_batch, "fp64", wl.tol, None),
                 ("fp64_plain_learned", "learned", args.plain_batch, "fp64", wl.tol, None),
                 ("fp64_batched_learned_tol1e-13", "learned", batch, "fp64", 1e-13, launch),
                 ("mixed_batched_learned", "learned", mixed_batch, "mixed", 1e-5, None),
                 ("fp64_batched_learned_tol1e-8", "learned", batch, "fp64", 1e-8, launch),
                 ("fp64_plain_tol1e-8", "natural", args.plain_batch, "fp64", 1e-8, None)]
        if args.variant_only:
            keep_v = set(args.variant_only.split(","))
            specs = [sp for sp in specs if sp[0] in keep_v]
        for name, mode, b, prec, tol, lopts in specs:
            torch.cuda.empty_cache()
            ms_v, sd_v, sh_v, l_v, (_, p_v, r_v) = timed(make_step(mode, b, prec, tol, lopts),
                                                          max(2, args.steps // 2), 1, name)
            st_v = r_v.status.cpu().numpy()
            conv_v = int(np.sum((st_v == sgf.CONVERGED) | (st_v == sgf.DIAG_ONLY))) * ns
            variants[name] = {"ms_per_step": ms_v, "solves_per_s": conv_v / (ms_v * 1e-3), "seed_ms": sd_v,
                              "shift_ms": sh_v, "launches": l_v, "batch_cols": b, "order": mode, "tol": tol,
                              "precision": prec, "launch": lopts or "library defaults"}
            if prec == "mixed":
                variants[name]["fp64_fallback_columns"] = int(getattr(r_v, "n_fallback", 0))
            if tol == wl.tol:
                variants[name]["rho_bitwise_equal"] = bool(torch.equal(r_v.rho, rho_ref))
            keep_sample(name, p_v, r_v)
            del r_v, p_v
        if not args.variant_only:
            plain_eq = variants["fp64_plain_tol1e-8"]["ms_per_step"]
            variants["speedup_vs_fp64_plain"] = variants["fp64_plain"]["ms_per_step"] / ms_step
            variants["learned_gain_vs_natural_order"] = variants["fp64_batched"]["ms_per_step"] / ms_step
            variants["learned_gain_vs_natural_order_plain_launches"] = (
                variants["fp64_plain"]["ms_per_step"] / variants["fp64_plain_learned"]["ms_per_step"])
            variants["speedup_mixed_vs_fp64_plain_equal_accuracy"] = plain_eq / variants["mixed_batched_learned"][
                "ms_per_step"]
            variants["speedup_fp64_batched_learned_vs_plain_equal_accuracy"] = plain_eq / variants[
                "fp64_batched_learned_tol1e-8"]["ms_per_step"]

    hbm = None
    if not args.no_hbm:
        del s_probe, p_probe
        torch.cuda.empty_cache()
        hbm = hbm_stream(sgf, W, dev)
        hbm["wavepacket"] = wp_stream(sgf, W, dev)

    extra, extra_keep = None, None
    fewer, fewer_keep = None, None
    if not args.no_extra:
        torch.cuda.empty_cache()
        fewer, fewer_keep = fermi_poles_leg(sgf, W, dev, min(args.ws_gib, 64.0))
    if not args.no_extra:
        torch.cuda.empty_cache()
        models = {"large_share": model}
        if only is None or "bundle_overlap_uneven" in only:
            models["bundle_overlap_uneven"], train_ovl = train_scheduler(sgf, W, dev, kind="overlap")
            train_info["overlap"] = train_ovl
            log(f"[bench] overlap scheduler: held-out MSE {train_ovl['heldout_mse']:.4f} (target variance "
                f"{train_ovl['target_var']:.4f})")
        torch.cuda.empty_cache()
        extra, extra_keep = extra_workloads(sgf, W, dev, min(args.ws_gib, 64.0), 1000, only=only, models=models)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(wl, args.cpu_seconds)
        if extra:
            for name, a in check_extra(extra_keep).items():
                if name.endswith("_mixed"):
                    extra[name[:-len("_mixed")]]["mixed"]["accuracy_vs_oracle"] = a
                else:
                    extra[name]["accuracy_vs_oracle"] = a
        if fewer:
            fewer["rho_vs_f_H_L"] = check_fermi(fewer_keep)
        ref13 = None
        for name, (G, rho, st) in samples.items():
            r = ref
            if name.endswith("tol1e-13"):
                if ref13 is None:
                    import oracle
                    ref13 = oracle.solve_workload(wl, cols=wl.columns[check_cols], tol=1e-13,
                                                  threads=cpu["cores"])
                r = ref13
            variants.setdefault(name, {})["accuracy_vs_oracle"] = accuracy(wl, check_cols, r, G, rho, st)

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
        "roofline": roofline_line(fig, seed_ms, shift_ms, launches, traffic_seed, traffic_shift, hbm_counted),
        "cpu_baseline": cpu,
        "hbm_stream": hbm,
        "after_rho": post,
        "other_workloads": extra,
        "fewer_shifts": fewer,
        "autotune": {"choice": launch, "timings_ms": tuned["timings_ms"], "sample_columns": TUNE_SAMPLE},
        "variants": variants,
        "scheduler": train_info,
        "converged_solves": converged,
        "columns_not_converged": int(np.sum(status != 0)),
        "iters_mean": float(iters.mean()),
    }
    print(json.dumps(line), flush=True)
    return 0


def baseline_sample(wl):
    """Seeded random order of the workload's columns (indices into wl.columns)."""
    return np.random.default_rng(1603).permutation(wl.columns.size)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds):
    """The FP64 oracle on a seeded sample of the same columns: a sample sized
    to about seconds/3 of oracle time, run three times (median rate).  Also
    returns the oracle's results for the first 1024 columns of the sample,
    against which the GPU variants' outputs are checked."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    b = oracle.system_for(wl)
    order = baseline_sample(wl)
    t0 = time.perf_counter()
    first = oracle.solve_workload(wl, b, cols=wl.columns[order[:1024]], threads=threads)
    per_col = (time.perf_counter() - t0) / 1024
    n = int(min(order.size, max(1024, seconds / 3.0 / per_col)))
    pick = wl.columns[order[:n]]
    rates, walls = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        r = oracle.solve_workload(wl, b, cols=pick, threads=threads)
        dt = time.perf_counter() - t0
        walls.append(dt)
        rates.append(int(np.sum(r.resid <= wl.tol)) / dt)
    log(f"[bench] oracle: {n} columns x 3 runs, {np.median(walls):.1f} s median wall on {threads} threads")
    return ({"value": float(np.median(rates)), "unit": "solves/s", "cores": threads, "kind": "oracle",
             "cpu_model": cpu_model(), "runs": 3, "rates": rates,
             "sample": f"{n} seeded random columns of the same workload (all {wl.z.size} shifts), run 3 times, "
                       f"median of {np.median(walls):.1f} s wall; value = median rate"},
            first)


def accuracy(wl, cols, ref, G, rho, status):
    """Errors of one variant's outputs on the checked columns against the
    oracle: all projection rows of G (max |dG| / max |G| per column), the
    diagonal G_jj (same, over its shifts; and the worst single shift,
    relative) and rho (max |drho| / max |rho| per column, and its diagonal)."""
    e_all = e_jj = e_jj_shift = e_rho = e_rho_jj = 0.0
    for i, c in enumerate(cols):
        a, b = ref.proj_ptr[i], ref.proj_ptr[i + 1]
        d = a + int(np.nonzero(ref.proj_row[a:b] == wl.columns[c])[0][0])
        scale = np.abs(ref.G[a:b]).max()
        e_all = max(e_all, np.abs(G[a:b] - ref.G[a:b]).max() / scale)
        e_jj = max(e_jj, np.abs(G[d] - ref.G[d]).max() / np.abs(ref.G[d]).max())
        e_jj_shift = max(e_jj_shift, float((np.abs(G[d] - ref.G[d]) / np.abs(ref.G[d])).max()))
        rs = max(np.abs(ref.rho[a:b]).max(), 1e-300)
        e_rho = max(e_rho, np.abs(rho[a:b] - ref.rho[a:b]).max() / rs)
        e_rho_jj = max(e_rho_jj, abs(rho[d] - ref.rho[d]) / rs)
    return {"columns": int(len(cols)), "G_rows_normwise": e_all, "G_jj_normwise": e_jj,
            "G_jj_worst_shift": e_jj_shift, "rho_normwise": e_rho, "rho_jj": e_rho_jj,
            "not_converged": int(np.sum(status != 0))}


if __name__ == "__main__":
    sys.exit(main())
