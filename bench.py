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


CSRC = os.path.join(ROOT, "paper_1603_09616_amd", "csrc")


def kernel_fingerprint(kind):
    """sha256 over the source a kernel is built from: its own function text
    (for the solver passes) or file, and the shared device helpers.  Counter
    figures recorded in profiles/ apply only while this matches."""
    import hashlib
    import re
    common = open(os.path.join(CSRC, "common.hpp")).read()
    if kind == "apply":
        text = open(os.path.join(CSRC, "apply.hip")).read()
    else:
        src = open(os.path.join(CSRC, "scocg.hip")).read()
        head = {"seed": r"template <int M, int BMAX>\n__global__ __launch_bounds__\(SEED_T\) void k_seed_r1",
                "shift": r"template <int NPA, int MS>\n__global__ __launch_bounds__\(512\)[^\n]* void k_shift"}[kind]
        m = re.search(head, src)
        if m is None:
            return None
        end = src.find("\n}\n", m.start())
        text = src[m.start():end + 3]
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
            name = {1: f"k_bsr_apply<{dtn}, 1, false>"}.get(k, f"k_bsr_apply_br<{dtn}, {k}, false>")
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


def extra_workloads(sgf, W, dev, ws_gib, check_n):
    """The other two workloads, one timed solve each after a warm-up:
    the overlap bundle (S != I, per-column radius U[0.6, 1.4] nm, 256 shifts,
    all 473,200 columns) and the 1,000,300-atom share (256 shifts, all
    4,001,200 columns, density matrix only: G alone would be 328 GB), both
    FP64 in workspace-sized launches.  Returns the timings and, per workload,
    the outputs of `check_n` seeded columns for the oracle comparison."""
    import torch
    out, keep = {}, {}
    for name, wl, g_out in (("bundle_overlap_uneven", W.config_bundle_overlap(), True),
                            ("large_share", W.config_large(), False)):
        s = sgf.system_for(wl)
        prep = sgf.prepare(s, wl.columns, radius=wl.radius, radius_per_col=wl.radius_per_col, prune=True)
        ns = wl.z.size
        batch = sgf.batch_limit(prep, ns, int(ws_gib * (1 << 30)))
        buf = None
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=g_out, batch_cols=batch, out=buf,
                                     profile=rep == 1)
            prof = sgf.solve_profile() if rep == 1 else None
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            buf = res._out
        st = res.status.cpu().numpy()
        conv = int(np.sum(res.resid.cpu().numpy() <= wl.tol))
        t = prep.plan.totals
        out[name] = {"workload": wl.name + (" (S != I, radius per column U[0.6, 1.4] nm)" if wl.tb.overlap else
                                            " (1,000,300 atoms)"),
                     "atoms": int(s.n_atoms), "columns": int(wl.columns.size), "shifts": int(ns), "tol": wl.tol,
                     "outputs": "G and rho" if g_out else "rho only", "ms": ms, "solves_per_s": conv / (ms * 1e-3),
                     "seed_ms": prof[0], "shift_ms": prof[1], "launches": prof[2], "batch_cols": int(batch),
                     "columns_not_converged": int(np.sum(st != 0)),
                     "iters_mean": float(res.iters.float().mean()), "max_loc_atoms": int(t.max_loc_atoms)}
        log(f"[bench] {name}: {wl.columns.size} columns x {ns} shifts in {ms:.1f} ms "
            f"({conv / (ms * 1e-3):.3g} solves/s, {prof[2]} launches)")
        if wl.tb.overlap:
            out[name]["after_rho"] = overlap_forces(sgf, prep, res, wl)
        pick = np.sort(np.random.default_rng(1603).choice(wl.columns.size, check_n, replace=False))
        off = prep.proj_off.cpu().numpy()
        rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in pick])
        idx = torch.as_tensor(rows, device=dev)
        keep[name] = (wl, pick, None if res.G is None else res.G[idx].cpu().numpy(), res.rho[idx].cpu().numpy(),
                      st[pick])
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
    for name, (wl, pick, G, rho, st) in keep.items():
        b = oracle.system_for(wl)
        t0 = time.perf_counter()
        rpc = None if wl.radius_per_col is None else wl.radius_per_col[pick]
        ref = oracle.shifted_solve(b, wl.xyz, wl.columns[pick], wl.z, wl.w, tol=wl.tol, radius=wl.radius,
                                   radius_per_col=rpc, prune=True, threads=threads)
        dt = time.perf_counter() - t0
        a = {"columns": int(pick.size), "oracle_s": dt, "oracle_threads": threads}
        e_rho = e_g = 0.0
        for i in range(pick.size):
            lo, hi = ref.proj_ptr[i], ref.proj_ptr[i + 1]
            e_rho = max(e_rho, np.abs(rho[lo:hi] - ref.rho[lo:hi]).max() / max(np.abs(ref.rho[lo:hi]).max(), 1e-300))
            if G is not None:
                e_g = max(e_g, np.abs(G[lo:hi] - ref.G[lo:hi]).max() / np.abs(ref.G[lo:hi]).max())
        a["rho_normwise"] = e_rho
        if G is not None:
            a["G_rows_normwise"] = e_g
        a["not_converged"] = int(np.sum(st != 0))
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
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-bound operator-apply measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the overlap and 1M-atom workloads")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library default launch (for profiler runs, which distort the tuner's timings)")
    ap.add_argument("--spmv-only", action="store_true",
                    help="only the operator-apply measurement and a 1 GiB copy (for counter passes)")
    ap.add_argument("--wp-only", action="store_true", help="only the wavepacket-propagation measurement")
    ap.add_argument("--extra-only", action="store_true",
                    help="only the overlap and 1,000,300-atom workloads (one timed solve each)")
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
    if args.spmv_only:
        print(json.dumps({"hbm_stream": hbm_stream(sgf, W, dev), "copy": copy_reference(dev)}), flush=True)
        return 0
    if args.wp_only:
        print(json.dumps({"wavepacket": wp_stream(sgf, W, dev)}), flush=True)
        return 0
    if args.extra_only:
        extra, _ = extra_workloads(sgf, W, dev, min(args.ws_gib, 64.0), 1)
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
        tuned = autotune.tune(p_probe, wl.z, wl.w, wl.tol, use_cache=False, log=log)
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
                pred = model.predict(sgf.features(prep))
                order = sgf.order_by_prediction(pred, 0.0, float(np.log(4096.0)))
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
                                         "order": "learned", "tol": wl.tol, "launch": launch}}
    keep_sample("fp64_batched_learned", prep, res)
    post = None
    if res.G is not None:
        post = after_rho(sgf, prep, res, wl)
        log(f"[bench] after rho: traces in {post['ms']:.2f} ms ({post['GBps']:.0f} GB/s), "
            f"mu(half filling) = {post['mu_half_filling_eV']:.4f} eV")
    if not args.no_variants:
        rho_ref = res.rho.clone()
        del res, prep, s
        mixed_batch = args.batch or sgf.batch_limit(p_probe, ns, int(args.ws_gib * (1 << 30)), precision="mixed")
        specs = [("fp64_batched", "natural", batch, "fp64", wl.tol, launch),
                 ("fp64_plain", "natural", args.plain_batch, "fp64", wl.tol, None),
                 ("mixed_batched_learned", "learned", mixed_batch, "mixed", 1e-5, None),
                 ("fp64_batched_learned_tol1e-8", "learned", batch, "fp64", 1e-8, launch),
                 ("fp64_plain_tol1e-8", "natural", args.plain_batch, "fp64", 1e-8, None)]
        for name, mode, b, prec, tol, lopts in specs:
            torch.cuda.empty_cache()
            ms_v, sd_v, sh_v, l_v, (_, p_v, r_v) = timed(make_step(mode, b, prec, tol, lopts),
                                                          max(2, args.steps // 2), 1, name)
            conv_v = int(np.sum(r_v.status.cpu().numpy() == sgf.CONVERGED)) * ns
            variants[name] = {"ms_per_step": ms_v, "solves_per_s": conv_v / (ms_v * 1e-3), "seed_ms": sd_v,
                              "shift_ms": sh_v, "launches": l_v, "batch_cols": b, "order": mode, "tol": tol,
                              "precision": prec, "launch": lopts or "library defaults"}
            if prec == "mixed":
                variants[name]["fp64_fallback_columns"] = int(getattr(r_v, "n_fallback", 0))
            if tol == wl.tol:
                variants[name]["rho_bitwise_equal"] = bool(torch.equal(r_v.rho, rho_ref))
            keep_sample(name, p_v, r_v)
            del r_v, p_v
        plain_eq = variants["fp64_plain_tol1e-8"]["ms_per_step"]
        variants["speedup_vs_fp64_plain"] = variants["fp64_plain"]["ms_per_step"] / ms_step
        variants["learned_gain_vs_natural_order"] = variants["fp64_batched"]["ms_per_step"] / ms_step
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
    if not args.no_extra:
        torch.cuda.empty_cache()
        extra, extra_keep = extra_workloads(sgf, W, dev, min(args.ws_gib, 64.0), 1000)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(wl, args.cpu_seconds)
        if extra:
            for name, a in check_extra(extra_keep).items():
                extra[name]["accuracy_vs_oracle"] = a
        for name, (G, rho, st) in samples.items():
            variants.setdefault(name, {})["accuracy_vs_oracle"] = accuracy(wl, check_cols, ref, G, rho, st)

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
            "traffic": recorded_traffic("k_seed_r1<2, 5>" if dominant == "k_seed" else "k_shift<5, 1>",
                                        "seed" if dominant == "k_seed" else "shift"),
            "launches_per_step": launches,
            "passes": {
                "k_seed": {"ms_per_step": seed_ms, "tflop_per_step": f_seed / 1e12, "tflops": seed_tf},
                "k_shift": {"ms_per_step": shift_ms, "tflop_per_step": f_shift / 1e12, "tflops": shift_tf},
            },
        },
        "cpu_baseline": cpu,
        "hbm_stream": hbm,
        "after_rho": post,
        "other_workloads": extra,
        "autotune": {"choice": launch, "timings_ms": tuned["timings_ms"], "sample_columns": 32768},
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


def cpu_baseline(wl, seconds):
    """The FP64 oracle on a seeded sample of the same columns, for ~`seconds`.
    Also returns the oracle's results for the first chunk (1024 columns),
    against which the GPU variants' outputs are checked."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    b = oracle.system_for(wl)
    order = baseline_sample(wl)
    done = conv = 0
    chunk = 1024
    first = None
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < order.size:
        pick = order[done:done + chunk]
        r = oracle.solve_workload(wl, b, cols=wl.columns[pick], threads=threads)
        if first is None:
            first = r
        conv += int(np.sum(r.resid <= wl.tol))
        done += pick.size
    dt = time.perf_counter() - t0
    log(f"[bench] oracle: {done} columns in {dt:.1f} s on {threads} threads")
    return ({"value": conv / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
             "sample": f"{done} seeded random columns of the same workload (all 128 shifts), {dt:.1f} s wall"},
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
