"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances.  Both sides run the same FP64 shifted COCG; they differ only by
rounding order.  The bar for Green's-function elements is the FP64 target of
1e-10 relative per result, with G compared per shift and normwise over the
projection rows of a column (|dG| / max|G|); density-matrix entries compare
against the largest entry of their column.  Bond patterns, plan sizes and
projection rows are integer results and must agree exactly.  Iteration
counts are not pinned (they depend on rounding order near the tolerance); their
means are compared.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FP64_RTOL = 1e-10


@pytest.fixture(scope="module")
def sgf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_09616_amd as sgf
    sgf.lib()
    return sgf


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.build(force=False)
    return oracle


def col_rel_err(got, ref):
    """max over columns of max|dG| / max|G| on that column."""
    worst = 0.0
    for c in range(ref.proj_ptr.size - 1):
        a, b = ref.proj_ptr[c], ref.proj_ptr[c + 1]
        worst = max(worst, np.abs(got.G[a:b] - ref.G[a:b]).max() / np.abs(ref.G[a:b]).max())
    return worst


def rho_rel_err(got, ref):
    worst = 0.0
    for c in range(ref.proj_ptr.size - 1):
        a, b = ref.proj_ptr[c], ref.proj_ptr[c + 1]
        scale = max(np.abs(ref.rho[a:b]).max(), 1e-300)
        worst = max(worst, np.abs(got.rho[a:b] - ref.rho[a:b]).max() / scale)
    return worst


def compare(got, ref, rtol=FP64_RTOL, check_iters=True, tol=None, eta=0.01):
    """Integer layout exact; G and rho within rtol (relative, per column).
    With tol given, also the a-priori bound: each side's G is within
    tol*||b||/eta of the exact restricted solve (S = I), so the two differ
    by at most 2 tol/eta per element."""
    np.testing.assert_array_equal(got.proj_off, ref.proj_ptr)
    np.testing.assert_array_equal(got.proj_row, ref.proj_row)
    np.testing.assert_array_equal(got.status, ref.status)
    e, r = col_rel_err(got, ref), rho_rel_err(got, ref)
    print(f"  G rel err {e:.2e}  rho rel err {r:.2e}  iters {got.iters.min()}..{got.iters.max()}", flush=True)
    if tol is not None:
        assert np.abs(got.G - ref.G).max() <= 2 * tol / eta
    assert e < rtol and r < rtol
    if check_iters:
        # Iteration counts are not pinned: once a shift's residual stagnates
        # near the tolerance, the freeze iteration depends on rounding order.
        # Their distributions must agree (means within 10%).
        gm, rm = float(np.mean(got.iters)), float(np.mean(ref.iters))
        assert abs(gm - rm) <= 0.1 * rm + 2, (gm, rm)


# ---------------------------------------------------------------------------
# Setup steps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("overlap", [False, True])
def test_build_hamiltonian(sgf, O, overlap):
    wl = W.bundle_workload(4, 3, 120, overlap=overlap, config_no=70)
    sysg = sgf.system_for(wl)
    ref = O.tb_build(wl.xyz, wl.tb)
    np.testing.assert_array_equal(sysg.row_ptr.cpu().numpy(), ref.row_ptr)
    np.testing.assert_array_equal(sysg.col.cpu().numpy(), ref.col)
    h = sysg.h.cpu().numpy()
    assert np.abs(h - ref.h).max() <= 1e-14 * np.abs(ref.h).max()
    if overlap:
        assert np.abs(sysg.s.cpu().numpy() - ref.s).max() <= 1e-14


def test_build_full_bundle_pattern(sgf, O):
    wl = W.config_bundle()
    sysg = sgf.system_for(wl)
    ref = O.tb_build(wl.xyz, wl.tb)
    assert sysg.nnzb == ref.nnzb
    np.testing.assert_array_equal(sysg.col.cpu().numpy(), ref.col)
    assert np.abs(sysg.h.cpu().numpy() - ref.h).max() <= 1e-14 * np.abs(ref.h).max()


def test_build_chain(sgf, O):
    for n in (4, 8, 2000):
        wl = W.chain_workload(n, 1, 4, config_no=71)
        g = sgf.system_for(wl)
        r = O.chain_build(wl.onsite, wl.hopping)
        np.testing.assert_array_equal(g.row_ptr.cpu().numpy(), r.row_ptr)
        np.testing.assert_array_equal(g.col.cpu().numpy(), r.col)
        np.testing.assert_array_equal(g.h.cpu().numpy(), r.h)


@pytest.mark.parametrize("prune", [False, True])
def test_plan_sizes(sgf, O, prune):
    wl = W.bundle_workload(5, 5, 80, config_no=72, radius_range=(0.4, 1.4))
    sysg = sgf.system_for(wl)
    ref = O.tb_build(wl.xyz, wl.tb)
    cols = wl.columns[::7]
    rpc = wl.radius_per_col[::7]
    prep = sgf.prepare(sysg, cols, radius_per_col=rpc, prune=prune)
    n_loc, n_proj = O.plan_sizes(ref, wl.xyz, cols, 0.0, rpc, prune)
    ao = prep.plan.atom_off.cpu().numpy()
    cp = prep.col_plan.cpu().numpy()
    np.testing.assert_array_equal(np.diff(ao)[cp], n_loc)
    np.testing.assert_array_equal(np.diff(prep.proj_off.cpu().numpy()), n_proj)
    # local atom lists equal the oracle's for a few columns
    la = prep.plan.loc_atom.cpu().numpy()
    for i in range(0, cols.size, max(1, cols.size // 6)):
        full = O.solve_full(ref, wl.xyz, int(cols[i]), wl.z[:1], radius=float(rpc[i]), prune=prune, max_iter=1)
        p = cp[i]
        np.testing.assert_array_equal(la[ao[p]:ao[p + 1]], full.loc_atoms)


# ---------------------------------------------------------------------------
# Shifted solve, FP64
# ---------------------------------------------------------------------------

def test_chain_full_system(sgf, O):
    """Plain method: 2000-site chain, 64 shifts, 16 columns, whole system."""
    wl = W.config_chain()
    got = sgf.solve_workload(wl).numpy()
    ref = O.solve_workload(wl, threads=8)
    compare(got, ref)


@pytest.mark.parametrize("prune", [True, False])
@pytest.mark.parametrize("n_shifts", [128, 100])
def test_bundle_small(sgf, O, prune, n_shifts):
    """Several tiles of columns and a ragged shift count.  Each side is within
    tol/eta of the exact restricted solve, so parity at 1e-10 is guaranteed
    for tol <= 1e-10 * eta / 2 = 5e-13; the unpruned subspaces (~500
    orbitals) use that tolerance, the pruned ones keep the workload's 1e-12
    (measured margin: errors ~1e-11)."""
    wl = W.bundle_workload(3, 3, 60, n_shifts=n_shifts, config_no=73, tol=1e-12 if prune else 5e-13)
    cols = wl.columns[::3]
    got = sgf.solve_workload(wl, cols=cols, prune=prune).numpy()
    ref = O.solve_workload(wl, cols=cols, prune=prune, threads=8)
    compare(got, ref)


def test_bundle_at_looser_tol(sgf, O):
    """At tol 1e-10 the two sides may freeze a shift one iteration apart; the
    difference stays inside the a-priori bound 2 tol/eta and shrinks with tol."""
    wl = W.bundle_workload(3, 3, 60, n_shifts=128, config_no=73, tol=1e-10)
    cols = wl.columns[::3]
    got = sgf.solve_workload(wl, cols=cols).numpy()
    ref = O.solve_workload(wl, cols=cols, threads=8)
    compare(got, ref, rtol=1e-8, tol=wl.tol)


@pytest.mark.parametrize("stage", [-1, 0, 1, 3, 5])
@pytest.mark.parametrize("batch", [0, 7])
def test_launch_shapes_agree(sgf, O, stage, batch):
    """Each seed-pass variant (four columns per wavefront, LDS-staged
    operator, operator from global memory, one column per wavefront with its
    rows in registers, two columns per wavefront) gives the oracle's result,
    and history batching (with a ragged last batch) does not change a single
    bit."""
    wl = W.bundle_workload(2, 2, 50, n_shifts=128, config_no=74)
    cols = wl.columns[::2]
    got = sgf.solve_workload(wl, cols=cols, batch_cols=batch, stage_lds=stage).numpy()
    ref = O.solve_workload(wl, cols=cols, threads=8)
    compare(got, ref)
    base = sgf.solve_workload(wl, cols=cols, stage_lds=stage).numpy()
    np.testing.assert_array_equal(got.G, base.G)
    np.testing.assert_array_equal(got.rho, base.rho)


@pytest.mark.parametrize("n_shifts", [256, 200])
def test_two_columns_per_wavefront(sgf, O, n_shifts):
    """Above 128 shifts the default seed pass runs two columns of a plan per
    wavefront (32 lanes per column, two rows per lane, up to eight shifts per
    lane): against the oracle, against one column per wavefront
    (stage_lds 3) within the parity bar, bitwise under a ragged batching and
    a repeat."""
    wl = W.bundle_workload(3, 2, 60, n_shifts=n_shifts, config_no=76)
    cols = wl.columns[::3]
    got = sgf.solve_workload(wl, cols=cols).numpy()
    ref = O.solve_workload(wl, cols=cols, threads=8)
    compare(got, ref)
    again = sgf.solve_workload(wl, cols=cols, batch_cols=7).numpy()
    np.testing.assert_array_equal(got.G, again.G)
    np.testing.assert_array_equal(got.rho, again.rho)
    r1 = sgf.solve_workload(wl, cols=cols, stage_lds=3).numpy()
    r1.proj_ptr = r1.proj_off
    e_g, e_r = col_rel_err(got, r1), rho_rel_err(got, r1)
    print(f"  two columns vs one column per wavefront: G {e_g:.2e}, rho {e_r:.2e}", flush=True)
    assert e_g < FP64_RTOL and e_r < FP64_RTOL


@pytest.mark.parametrize("spl", [1, 2])
def test_shift_lanes_agree(sgf, O, spl):
    """One or two shifts per lane in the shift pass: oracle parity."""
    wl = W.bundle_workload(3, 2, 60, n_shifts=128, config_no=79)
    cols = wl.columns[::3]
    got = sgf.solve_workload(wl, cols=cols, shifts_per_lane=spl).numpy()
    ref = O.solve_workload(wl, cols=cols, threads=8)
    compare(got, ref)


def test_order_and_repeat_are_bitwise(sgf):
    wl = W.bundle_workload(2, 2, 50, n_shifts=64, config_no=75)
    s = sgf.system_for(wl)
    a = sgf.solve_workload(wl, s).numpy()
    b = sgf.solve_workload(wl, s).numpy()
    perm = np.random.default_rng(0).permutation(wl.columns.size)
    c = sgf.solve_workload(wl, s, order=perm).numpy()
    for x in (b, c):
        np.testing.assert_array_equal(a.G, x.G)
        np.testing.assert_array_equal(a.rho, x.rho)
        np.testing.assert_array_equal(a.iters, x.iters)


def test_edge_cases(sgf, O):
    wl = W.bundle_workload(2, 1, 30, n_shifts=64, config_no=76)
    s = sgf.system_for(wl)
    b = O.system_for(wl)
    # one shift; seed at either end
    for ns, seed in ((1, -1), (64, 0), (64, 63)):
        z = wl.z[:ns]
        got = sgf.shifted_solve(s, wl.columns[:9], z, wl.w[:ns], tol=1e-12, radius=1.0, seed_index=seed).numpy()
        ref = O.shifted_solve(b, wl.xyz, wl.columns[:9], z, wl.w[:ns], tol=1e-12, radius=1.0, prune=True,
                              seed_index=seed)
        compare(got, ref)
    # max_iter exhaustion
    got = sgf.shifted_solve(s, wl.columns[:5], wl.z, wl.w, tol=1e-12, radius=1.0, max_iter=3).numpy()
    ref = O.shifted_solve(b, wl.xyz, wl.columns[:5], wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, max_iter=3)
    assert np.all(got.status == sgf.MAXITER) and np.all(got.iters == 3)
    compare(got, ref)
    # isolated atom (single projection atom)
    xyz = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [3.0, 0.0, 0.15]])
    s1 = sgf.build_hamiltonian(xyz, W.BUNDLE_TB)
    b1 = O.tb_build(xyz, W.BUNDLE_TB)
    got = sgf.shifted_solve(s1, np.arange(12), wl.z, wl.w, tol=1e-12, radius=1.0).numpy()
    ref = O.shifted_solve(b1, xyz, np.arange(12), wl.z, wl.w, tol=1e-12, radius=1.0, prune=True)
    compare(got, ref)
    # empty column list
    got = sgf.shifted_solve(s, np.zeros(0, np.int64), wl.z, wl.w, radius=1.0)
    assert got.iters.numel() == 0


def test_nonfinite_column_only(sgf, O):
    """A NaN block poisons only the columns whose subspace holds it."""
    wl = W.bundle_workload(2, 1, 30, n_shifts=32, config_no=77)
    s = sgf.system_for(wl)
    s.h[int(s.row_ptr[1])] = float("nan")
    got = sgf.shifted_solve(s, np.array([0, 4, 100, 150]), wl.z, wl.w, radius=0.6).numpy()
    assert list(got.status) == [sgf.NONFINITE, sgf.NONFINITE, sgf.CONVERGED, sgf.CONVERGED]


@pytest.mark.parametrize("explicit_s", [False, True])
@pytest.mark.parametrize("stage", [-1, 0, 1, 3])
def test_breakdown_status(sgf, O, stage, explicit_s):
    """The crafted input of workloads.breakdown_block makes mu vanish exactly
    in the second iteration (worked by hand beside the oracle's pin of the
    same case).  Every seed kernel ends the column with SGF_BREAKDOWN after
    two iterations, and the one completed step gives x^k = e_0 / z_k on every
    shift, as on the oracle."""
    import torch
    if explicit_s and stage == 3:
        pytest.skip("stage_lds 3 is an S = I launch shape")
    row_ptr, col, h, z = W.breakdown_block()
    s = np.eye(4)[None].copy() if explicit_s else None
    xyz = np.zeros((1, 3))
    d = lambda a: None if a is None else torch.as_tensor(a, device="cuda")
    system = sgf.system_from_bsr(d(row_ptr), d(col), d(h), s=d(s), xyz=d(xyz))
    got = sgf.shifted_solve(system, np.array([0]), z, tol=1e-12, radius=1.0, seed_index=1, stage_lds=stage).numpy()
    ref = O.shifted_solve(O.BSR(row_ptr, col, h, s), xyz, np.array([0]), z, None, tol=1e-12, radius=1.0,
                          prune=True, seed_index=1)
    assert got.status[0] == sgf.BREAKDOWN == ref.status[0]
    assert got.iters[0] == 2 == ref.iters[0]
    np.testing.assert_array_equal(got.proj_row, ref.proj_row)
    G = got.G.reshape(4, z.size)
    np.testing.assert_allclose(G[0], 1.0 / z, rtol=1e-15, atol=0)
    assert np.all(G[1:] == 0)
    np.testing.assert_allclose(got.G, ref.G, rtol=1e-15, atol=0)


def test_invalid_arguments(sgf):
    wl = W.bundle_workload(1, 1, 10, n_shifts=8, config_no=78)
    s = sgf.system_for(wl)
    with pytest.raises(sgf.SgfError) as e:
        sgf.shifted_solve(s, wl.columns[:2], wl.z.real.astype(complex), None, radius=1.0)
    assert e.value.code == sgf.SGF_EINVAL
    with pytest.raises(sgf.SgfError) as e:
        sgf.shifted_solve(s, wl.columns[:2], wl.z, None, tol=0.0, radius=1.0)
    assert e.value.code == sgf.SGF_EINVAL


def test_bundle_full_size_sampled(sgf, O):
    """The full 118,300-atom bundle (all 473,200 columns, 128 shifts), in the
    launch configuration the benchmark times (one batch of as many columns
    as a 112 GiB workspace holds, a permuted column order); 160 sampled
    columns are recomputed by the oracle."""
    import torch
    torch.cuda.empty_cache()
    wl = W.config_bundle()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    batch = sgf.batch_limit(prep, wl.z.size, 112 << 30)
    order = np.random.default_rng(7).permutation(wl.columns.size).astype(np.int32)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, batch_cols=batch, order=order)
    torch.cuda.synchronize()
    st = res.status.cpu().numpy()
    assert np.all(st == sgf.CONVERGED)
    sample = np.sort(np.random.default_rng(1603).choice(wl.columns.size, 160, replace=False))
    ref = O.solve_workload(wl, cols=wl.columns[sample], threads=8)
    off = res.proj_off.cpu().numpy()
    rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in sample])
    idx = torch.as_tensor(rows, device=res.rho.device)

    class Sub:
        pass
    got = Sub()
    got.proj_off = np.concatenate([[0], np.cumsum(off[sample + 1] - off[sample])])
    got.proj_row = res.proj_row[idx].cpu().numpy()
    got.G = res.G[idx].cpu().numpy()
    got.rho = res.rho[idx].cpu().numpy()
    got.status = st[sample]
    got.iters = res.iters.cpu().numpy()[sample]
    compare(got, ref)


# ---------------------------------------------------------------------------
# Generalized equation (S != I)
# ---------------------------------------------------------------------------

def test_overlap_small(sgf, O):
    """(zS - H)x = e_j with the non-orthogonal overlap: GPU vs oracle."""
    wl = W.bundle_workload(2, 2, 40, overlap=True, n_shifts=64, config_no=83)
    cols = wl.columns[::3]
    got = sgf.solve_workload(wl, cols=cols).numpy()
    ref = O.solve_workload(wl, cols=cols, threads=8)
    compare(got, ref)


def test_overlap_workload_sampled(sgf, O):
    """The overlap workload (full bundle geometry, per-column radius drawn from
    U[0.6, 1.4] nm, 256 shifts): 2048 seeded columns on the GPU, 48 of them
    recomputed by the oracle."""
    wl = W.config_bundle_overlap(n_columns=2048)
    got = sgf.solve_workload(wl).numpy()
    assert np.all(got.status == sgf.CONVERGED)
    pick = np.sort(np.random.default_rng(3).choice(wl.columns.size, 48, replace=False))
    ref = O.solve_workload(wl, cols=wl.columns[pick], threads=8)

    class Sub:
        pass
    sub = Sub()
    rows = np.concatenate([np.arange(got.proj_off[c], got.proj_off[c + 1]) for c in pick])
    sub.proj_off = np.concatenate([[0], np.cumsum(got.proj_off[pick + 1] - got.proj_off[pick])])
    sub.proj_row, sub.G, sub.rho = got.proj_row[rows], got.G[rows], got.rho[rows]
    sub.status, sub.iters = got.status[pick], got.iters[pick]
    compare(sub, ref)


def test_overlap_size_classes_bitwise(sgf):
    """S != I, general S: the default seed pass runs subspaces of <= 16 atoms in a launch
    with the dense overlap inverse, and the larger ones in a second launch with
    its packed triangle, both with two wavefronts per column.  stage_lds 2
    makes the same split with one wavefront per column; each of its classes
    gives the same bits as one launch with that class's layout (stage_lds 0:
    dense, 1: packed).  The two-wavefront kernels form the same inverses but
    sum in another order, and agree with those within the parity bar, as do
    the two layouts (two exact inverses of the same S_L).  Repeated default
    solves are bitwise equal."""
    wl = W.config_bundle_overlap(n_columns=4096)
    s = sgf.system_for(wl)
    s.s_orbital_diagonal = False  # treated as a general S: the orbital-level inverse
    prep = sgf.prepare(s, wl.columns, radius_per_col=wl.radius_per_col)
    n_loc = np.diff(prep.plan.atom_off.cpu().numpy())[prep.col_plan.cpu().numpy()]
    assert n_loc.min() <= 16 < n_loc.max()
    auto = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    auto2 = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    split1 = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=2).numpy()
    dense = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=0).numpy()
    packed = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=1).numpy()
    for r in (auto, auto2, split1, dense, packed):
        assert np.all(r.status == sgf.CONVERGED)
    np.testing.assert_array_equal(auto.G, auto2.G)
    np.testing.assert_array_equal(auto.rho, auto2.rho)
    off = auto.proj_off
    worst = worst2 = 0.0
    for c in range(wl.columns.size):
        rows = slice(off[c], off[c + 1])
        ref = dense if n_loc[c] <= 16 else packed
        np.testing.assert_array_equal(split1.G[rows], ref.G[rows])
        np.testing.assert_array_equal(split1.rho[rows], ref.rho[rows])
        assert split1.iters[c] == ref.iters[c]
        worst2 = max(worst2, np.abs(auto.G[rows] - ref.G[rows]).max() / np.abs(ref.G[rows]).max(),
                     np.abs(auto.rho[rows] - ref.rho[rows]).max() / np.abs(ref.rho[rows]).max())
        if c % 5 == 0:
            worst = max(worst, np.abs(dense.G[rows] - packed.G[rows]).max() / np.abs(dense.G[rows]).max())
    print(f"  dense vs packed inverse: G {worst:.2e}; two wavefronts vs one: {worst2:.2e}, "
          f"iterations {auto.iters.mean():.1f} vs {split1.iters.mean():.1f}", flush=True)
    assert worst < 1e-10 and worst2 < 1e-10
    assert abs(auto.iters.mean() - split1.iters.mean()) <= 0.1 * split1.iters.mean() + 2


@pytest.mark.parametrize("n_shifts", [64, 320])
def test_overlap_two_wavefront_shift_counts(sgf, O, n_shifts):
    """The two-wavefront S != I seed passes hold one shift per thread at 64
    shifts and three (of four slots) at 320: both against the oracle on
    sampled columns of both size classes, and against the one-wavefront split
    (stage_lds 2) within the parity bar."""
    wl = W.config_bundle_overlap(n_columns=1536, n_shifts=n_shifts, config_no=31)
    s = sgf.system_for(wl)
    s.s_orbital_diagonal = False  # treated as a general S: the orbital-level inverse
    prep = sgf.prepare(s, wl.columns, radius_per_col=wl.radius_per_col)
    n_loc = np.diff(prep.plan.atom_off.cpu().numpy())[prep.col_plan.cpu().numpy()]
    assert n_loc.min() <= 16 < n_loc.max()
    got = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    one = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=2).numpy()
    assert np.all(got.status == sgf.CONVERGED) and np.all(one.status == sgf.CONVERGED)
    one.proj_ptr = one.proj_off
    e_g, e_r = col_rel_err(got, one), rho_rel_err(got, one)
    print(f"  {n_shifts} shifts: two wavefronts vs one: G {e_g:.2e}, rho {e_r:.2e}", flush=True)
    assert e_g < FP64_RTOL and e_r < FP64_RTOL
    small, big = np.nonzero(n_loc <= 16)[0][:12], np.nonzero(n_loc > 16)[0][:12]
    pick = np.sort(np.concatenate([small, big]))
    ref = O.solve_workload(wl, cols=wl.columns[pick], threads=8)

    class Sub:
        pass
    sub = Sub()
    rows = np.concatenate([np.arange(got.proj_off[c], got.proj_off[c + 1]) for c in pick])
    sub.proj_off = np.concatenate([[0], np.cumsum(got.proj_off[pick + 1] - got.proj_off[pick])])
    sub.proj_row, sub.G, sub.rho = got.proj_row[rows], got.G[rows], got.rho[rows]
    sub.status, sub.iters = got.status[pick], got.iters[pick]
    compare(sub, ref)


def _sub(res, pick):
    """The outputs of columns `pick` of a solve, in the oracle's layout."""
    class Sub:
        pass
    sub = Sub()
    rows = np.concatenate([np.arange(res.proj_off[c], res.proj_off[c + 1]) for c in pick])
    sub.proj_off = np.concatenate([[0], np.cumsum(res.proj_off[pick + 1] - res.proj_off[pick])])
    sub.proj_row, sub.G, sub.rho = res.proj_row[rows], res.G[rows], res.rho[rows]
    sub.status, sub.iters = res.status[pick], res.iters[pick]
    return sub


@pytest.mark.parametrize("n_shifts", [64, 256])
def test_overlap_per_atom_inverse(sgf, O, n_shifts):
    """The builder's overlap has blocks s(r) I4, so the default S != I seed
    pass inverts S_a (one number per atom pair) instead of the orbital-level
    S_L: a launch for <= 16 atoms (one wavefront per column, one row per
    lane) and one for 17-32 (two wavefronts per column, a row per thread; or
    one wavefront with two rows per lane, stage_lds 4).  Against the
    orbital-level dense inverse (stage_lds 0) within the parity bar on every
    column, the two forms of the larger class against each other, against
    the oracle on sampled columns of both classes, and bitwise on a repeat."""
    wl = W.config_bundle_overlap(n_columns=2048, n_shifts=n_shifts, config_no=32)
    s = sgf.system_for(wl)
    assert s.s_orbital_diagonal
    prep = sgf.prepare(s, wl.columns, radius_per_col=wl.radius_per_col)
    n_loc = np.diff(prep.plan.atom_off.cpu().numpy())[prep.col_plan.cpu().numpy()]
    assert n_loc.min() <= 16 < n_loc.max()
    got = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    again = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    one_wave = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=4).numpy()
    dense = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=0).numpy()
    assert np.all(got.status == sgf.CONVERGED) and np.all(dense.status == sgf.CONVERGED)
    assert np.all(one_wave.status == sgf.CONVERGED)
    np.testing.assert_array_equal(got.G, again.G)
    np.testing.assert_array_equal(got.rho, again.rho)
    # the classes of <= 16 atoms run the same kernel in both
    small = n_loc <= 16
    for c in np.nonzero(small)[0][:64]:
        rows = slice(got.proj_off[c], got.proj_off[c + 1])
        np.testing.assert_array_equal(got.G[rows], one_wave.G[rows])
    dense.proj_ptr = dense.proj_off
    one_wave.proj_ptr = one_wave.proj_off
    e_g, e_r = col_rel_err(got, dense), rho_rel_err(got, dense)
    e_g1, e_r1 = col_rel_err(got, one_wave), rho_rel_err(got, one_wave)
    print(f"  {n_shifts} shifts: per-atom vs orbital inverse: G {e_g:.2e}, rho {e_r:.2e}; two vs one wavefront "
          f"per column: G {e_g1:.2e}, rho {e_r1:.2e}; iterations {got.iters.mean():.1f} vs "
          f"{dense.iters.mean():.1f}", flush=True)
    assert e_g < FP64_RTOL and e_r < FP64_RTOL
    assert e_g1 < FP64_RTOL and e_r1 < FP64_RTOL
    assert abs(got.iters.mean() - dense.iters.mean()) <= 0.1 * dense.iters.mean() + 2
    small, big = np.nonzero(n_loc <= 16)[0][:12], np.nonzero(n_loc > 16)[0][:12]
    pick = np.sort(np.concatenate([small, big]))
    ref = O.solve_workload(wl, cols=wl.columns[pick], threads=8)
    compare(_sub(got, pick), ref)


def test_overlap_per_atom_inverse_one_class(sgf, O):
    """Every subspace at most 16 atoms (R = 0.8 nm): the per-atom seed pass
    runs one launch, against the oracle."""
    wl = W.bundle_workload(3, 2, 60, overlap=True, n_shifts=128, config_no=33)
    s = sgf.system_for(wl)
    cols = wl.columns[::3]
    got = sgf.shifted_solve(s, cols, wl.z, wl.w, tol=wl.tol, radius=0.8).numpy()
    ref = O.shifted_solve(O.system_for(wl), wl.xyz, cols, wl.z, wl.w, tol=wl.tol, radius=0.8, prune=True,
                          threads=8)
    assert np.diff(ref.proj_ptr).size == cols.size
    compare(got, ref)


def test_overlap_block_not_orbital_diagonal_is_refused(sgf):
    """A system that states s_orbital_diagonal while one off-diagonal block of
    S carries an orbital coupling: every column whose subspace holds that
    block ends BADCOLUMN, the others are bitwise those of the unmodified
    system; stated as a general S, every column converges."""
    import torch
    wl = W.bundle_workload(2, 1, 30, overlap=True, n_shifts=64, config_no=34)
    base = sgf.system_for(wl)
    s2 = base.s.clone()
    rp = base.row_ptr.cpu().numpy()
    cl = base.col.cpu().numpy()
    t = next(t for t in range(rp[10], rp[11]) if cl[t] == 11)   # block (10, 11)
    u = next(u for u in range(rp[11], rp[12]) if cl[u] == 10)   # and its transpose
    s2[t, 0, 1] = s2[t, 1, 0] = 1e-3
    s2[u, 0, 1] = s2[u, 1, 0] = 1e-3
    cols = np.arange(4 * 30)
    kw = dict(tol=1e-12, radius=0.6)
    ref = sgf.shifted_solve(base, cols, wl.z, wl.w, **kw).numpy()
    stated = sgf.system_from_bsr(base.row_ptr, base.col, base.h, s=s2, xyz=base.xyz, s_orbital_diagonal=True)
    got = sgf.shifted_solve(stated, cols, wl.z, wl.w, **kw).numpy()
    hit = got.status == sgf.BADCOLUMN
    assert hit.any() and np.all(got.status[~hit] == sgf.CONVERGED)
    for c in np.nonzero(~hit)[0]:
        rows = slice(got.proj_off[c], got.proj_off[c + 1])
        np.testing.assert_array_equal(got.G[rows], ref.G[rows])
    general = sgf.system_from_bsr(base.row_ptr, base.col, base.h, s=s2, xyz=base.xyz)
    res = sgf.shifted_solve(general, cols, wl.z, wl.w, **kw).numpy()
    assert np.all(res.status == sgf.CONVERGED)
    print(f"  {int(hit.sum())} of {cols.size} columns refused", flush=True)
    del torch


@pytest.mark.skip(reason="the register-tile S != I seed pass did not finish on the GPU (small overlap bundle, "
                         "one wavefront per column); its cause was not found, and the kernel was removed from the "
                         "library: every S != I solve takes the LDS seed passes")
def test_overlap_register_tiles_match_dense_inverse(sgf):
    """S != I seed pass with the overlap inverse in register tiles (one
    wavefront up to 16 local atoms, two for 17 to 22) against the variant
    that keeps the dense inverse in LDS, on columns of both sizes: same
    layout and status, G and rho within 1e-10 per column (two inverses of the
    same well-conditioned S_L, each iteration converged to 1e-12)."""
    wl = W.config_bundle_overlap(n_columns=4096)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius_per_col=wl.radius_per_col)
    n_loc = np.diff(prep.plan.atom_off.cpu().numpy())[prep.col_plan.cpu().numpy()]
    print(f"  local atoms {n_loc.min()}..{n_loc.max()}: {int((n_loc <= 16).sum())} columns <= 16, "
          f"{int((n_loc > 16).sum())} above", flush=True)
    assert n_loc.min() <= 16 < n_loc.max() <= 22 and np.any(n_loc == 16) and np.any(n_loc == 17)
    a = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    b = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, stage_lds=0).numpy()
    np.testing.assert_array_equal(a.status, b.status)
    assert np.all(a.status == sgf.CONVERGED)
    err_g = err_r = 0.0
    for c in range(0, wl.columns.size, 7):
        r0, r1 = a.proj_off[c], a.proj_off[c + 1]
        err_g = max(err_g, np.abs(a.G[r0:r1] - b.G[r0:r1]).max() / np.abs(b.G[r0:r1]).max())
        err_r = max(err_r, np.abs(a.rho[r0:r1] - b.rho[r0:r1]).max() / np.abs(b.rho[r0:r1]).max())
    print(f"  tiles vs dense: G {err_g:.2e}  rho {err_r:.2e}; iterations {a.iters.mean():.1f} vs "
          f"{b.iters.mean():.1f}", flush=True)
    assert err_g < 1e-10 and err_r < 1e-10
    assert abs(a.iters.mean() - b.iters.mean()) <= 0.02 * b.iters.mean()
