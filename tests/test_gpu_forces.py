"""GPU tests of the band forces F = -dE_band/dR at fixed rho (S = I) and,
with an overlap, of the energy-density matrix and its term in the forces.

Bar: the forces sum rho- (and eps-) weighted block gradients, so the GPU and
oracle forces differ by the rho and eps differences of the two solves
(<= 1e-10 relative per column) propagated through those sums: 1e-9 relative
to the largest force.  The energy-density matrix is compared per column,
1e-9 relative to the column's largest entry; from the GPU's own G it must
match the oracle's quadrature to rounding (1e-13).  At full size, an atom's force depends only on its own columns and
those of the atoms sharing a block with it, so the oracle solves just those
for a few sampled atoms.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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
    from oracle import forces
    return oracle, forces


def test_forces_vs_oracle_small(sgf, O):
    O, fo = O
    wl = W.bundle_workload(2, 1, 14, config_no=120)
    cols = np.arange(wl.n_orb)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, cols, radius=1.0, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    F = sgf.band_forces(prep, res, wl.tb).cpu().numpy()
    ref = O.shifted_solve(O.system_for(wl), wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    Fr = fo.band_forces(wl.xyz, wl.tb, ref, cols, wl.n_atoms)
    err = np.abs(F - Fr).max() / np.abs(Fr).max()
    print(f"  max |F| {np.abs(Fr).max():.3f} eV/nm, rel err {err:.2e}, sum {np.abs(F.sum(0)).max():.2e}")
    assert err < 1e-9
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()


def test_forces_full_bundle_sampled(sgf, O):
    import torch
    O, fo = O
    wl = W.config_bundle()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=False)
    F = sgf.band_forces(prep, res, wl.tb)
    F2 = sgf.band_forces(prep, res, wl.tb)
    F, F2 = F.cpu().numpy(), F2.cpu().numpy()
    scale = np.abs(F).max()
    print(f"  {wl.n_atoms} atoms: max |F| {scale:.3f} eV/nm, |sum F| {np.abs(F.sum(0)).max():.2e}, "
          f"repeat {np.abs(F - F2).max():.2e}", flush=True)
    assert np.abs(F.sum(axis=0)).max() <= 1e-11 * np.abs(F).sum()
    assert np.abs(F - F2).max() <= 1e-13 * scale
    b = O.system_for(wl)
    for A in np.random.default_rng(11).choice(wl.n_atoms, 3, replace=False):
        nbr = b.col[b.row_ptr[A]:b.row_ptr[A + 1]]          # A and the atoms sharing a block with it
        cols = (4 * nbr[:, None] + np.arange(4)[None, :]).ravel().astype(np.int64)
        ref = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=wl.tol, radius=wl.radius, prune=True, threads=8)
        Fr = fo.band_forces(wl.xyz, wl.tb, ref, cols, wl.n_atoms)[A]
        print(f"  atom {A}: {F[A]} vs {Fr}")
        assert np.abs(F[A] - Fr).max() <= 1e-9 * scale
    del res
    torch.cuda.empty_cache()


def overlap_case(sgf):
    wl = W.bundle_workload(2, 1, 14, overlap=True, config_no=120)
    cols = np.arange(wl.n_orb)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, cols, radius=1.0, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    return wl, cols, prep, res


def col_rel(a, b, off):
    return max(np.abs(a[off[c]:off[c + 1]] - b[off[c]:off[c + 1]]).max() / np.abs(b[off[c]:off[c + 1]]).max()
               for c in range(off.size - 1))


def test_energy_density_vs_oracle_small(sgf, O):
    O, fo = O
    wl, cols, prep, res = overlap_case(sgf)
    eps = sgf.energy_density(res, wl.z, wl.w)
    eps2 = sgf.energy_density(res, wl.z, wl.w)
    got = res.numpy()
    e, e2 = eps.cpu().numpy(), eps2.cpu().numpy()
    np.testing.assert_array_equal(e, e2)  # fixed summation order
    own = fo.energy_density(got, wl.z, wl.w)  # the oracle's quadrature of the GPU's G
    ref = O.shifted_solve(O.system_for(wl), wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    eref = fo.energy_density(ref, wl.z, wl.w)
    off = got.proj_off
    np.testing.assert_array_equal(off, ref.proj_ptr)
    np.testing.assert_array_equal(got.proj_row, ref.proj_row)
    r_own, r_ref = col_rel(e, own, off), col_rel(e, eref, off)
    print(f"  eps vs own G {r_own:.2e}, vs oracle solve {r_ref:.2e}", flush=True)
    assert r_own < 1e-13 and r_ref < 1e-9
    # sum_{i in P(j)} eps_ij S_ji = sum_{i in P(j)} rho_ij H_ji (real weights)
    b = O.system_for(wl)
    H, S = b.dense("h"), b.dense("s")
    for c, j in enumerate(cols):
        rows = got.proj_row[off[c]:off[c + 1]]
        assert abs(e[off[c]:off[c + 1]] @ S[j, rows] - got.rho[off[c]:off[c + 1]] @ H[j, rows]) < 1e-10


def test_overlap_forces_vs_oracle_small(sgf, O):
    O, fo = O
    wl, cols, prep, res = overlap_case(sgf)
    eps = sgf.energy_density(res, wl.z, wl.w)
    F = sgf.band_forces(prep, res, wl.tb, eps=eps).cpu().numpy()
    ref = O.shifted_solve(O.system_for(wl), wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    Fr = fo.band_forces(wl.xyz, wl.tb, ref, cols, wl.n_atoms, eps=fo.energy_density(ref, wl.z, wl.w))
    F0 = fo.band_forces(wl.xyz, wl.tb, ref, cols, wl.n_atoms, eps=np.zeros(ref.rho.size))
    err = np.abs(F - Fr).max() / np.abs(Fr).max()
    print(f"  max |F| {np.abs(Fr).max():.3f} eV/nm, eps term {np.abs(Fr - F0).max():.3f}, rel err {err:.2e}")
    assert err < 1e-9
    assert np.abs(Fr - F0).max() > 1e-3 * np.abs(Fr).max()  # the eps term is there
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()


def test_energy_density_from_the_shift_pass(sgf, O):
    """The shift pass's eps output (no G needed) against the stream over the
    kept G (same quadrature, other summation order: 1e-13) and the oracle;
    the forces from it without G match those from the stream."""
    O, fo = O
    wl, cols, prep, res = overlap_case(sgf)
    eps_g = sgf.energy_density(res, wl.z, wl.w).cpu().numpy()
    r2 = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, g_out=False, eps_out=True)
    e2 = r2.eps.cpu().numpy()
    np.testing.assert_array_equal(r2.rho.cpu().numpy(), res.rho.cpu().numpy())
    off = res.proj_off.cpu().numpy()
    ref = O.shifted_solve(O.system_for(wl), wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    r_g, r_o = col_rel(e2, eps_g, off), col_rel(e2, fo.energy_density(ref, wl.z, wl.w), off)
    print(f"  shift-pass eps vs G stream {r_g:.2e}, vs oracle {r_o:.2e}", flush=True)
    assert r_g < 1e-13 and r_o < 1e-9
    F1 = sgf.band_forces(prep, res, wl.tb, eps=sgf.energy_density(res, wl.z, wl.w)).cpu().numpy()
    F2 = sgf.band_forces(prep, r2, wl.tb, eps=r2.eps).cpu().numpy()
    assert np.abs(F1 - F2).max() <= 1e-12 * np.abs(F1).max()
    with pytest.raises(sgf.SgfError):
        sgf.solve_prepared(prep, wl.z, None, tol=1e-12, eps_out=True)  # needs weights
    with pytest.raises(sgf.SgfError):
        sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, precision="mixed", eps_out=True, fallback=False)


def test_energy_density_output_under_batching(sgf):
    """The shift pass writes eps at each column's own output rows: small
    launches (37 columns) and a learned-order-like permutation give the same
    bits as one launch in natural order."""
    wl, cols, prep, res = overlap_case(sgf)
    one = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, g_out=False, eps_out=True)
    many = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, g_out=False, eps_out=True, batch_cols=37)
    perm = np.random.default_rng(4).permutation(cols.size).astype(np.int32)
    perm_res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, g_out=False, eps_out=True, order=perm)
    e1 = one.eps.cpu().numpy()
    np.testing.assert_array_equal(many.eps.cpu().numpy(), e1)
    np.testing.assert_array_equal(perm_res.eps.cpu().numpy(), e1)
    np.testing.assert_array_equal(perm_res.rho.cpu().numpy(), one.rho.cpu().numpy())


def test_overlap_forces_argument_errors(sgf):
    import dataclasses
    wl, cols, prep, res = overlap_case(sgf)
    with pytest.raises(sgf.SgfError):
        sgf.band_forces(prep, res, wl.tb)  # no eps with an overlap
    eps = sgf.energy_density(res, wl.z, wl.w)
    with pytest.raises(sgf.SgfError):
        sgf.band_forces(prep, res, dataclasses.replace(wl.tb, overlap=0), eps=eps)  # flag does not match
    with pytest.raises(ValueError):
        sgf.energy_density(res, wl.z[:-1], wl.w[:-1])


def test_overlap_forces_full_bundle_sampled(sgf, O):
    """The overlap bundle (118,300 atoms, per-column radius U[0.6, 1.4] nm,
    256 shifts): eps from the kept G, forces with the eps term; three
    sampled atoms against the oracle, which solves only their own and their
    neighbours' columns."""
    import torch
    O, fo = O
    wl = W.config_bundle_overlap()
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius_per_col=wl.radius_per_col)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol)
    eps = sgf.energy_density(res, wl.z, wl.w)
    F = sgf.band_forces(prep, res, wl.tb, eps=eps).cpu().numpy()
    st = res.status.cpu().numpy()
    scale = np.abs(F).max()
    print(f"  {wl.n_atoms} atoms: max |F| {scale:.3f} eV/nm, |sum F| {np.abs(F.sum(0)).max():.2e}", flush=True)
    assert np.all(st == sgf.CONVERGED)
    assert np.abs(F.sum(axis=0)).max() <= 1e-11 * np.abs(F).sum()
    b = O.system_for(wl)
    for A in np.random.default_rng(12).choice(wl.n_atoms, 3, replace=False):
        nbr = b.col[b.row_ptr[A]:b.row_ptr[A + 1]]
        cols = (4 * nbr[:, None] + np.arange(4)[None, :]).ravel().astype(np.int64)
        ref = O.solve_workload(wl, bsr=b, cols=cols, threads=8)
        Fr = fo.band_forces(wl.xyz, wl.tb, ref, cols, wl.n_atoms, eps=fo.energy_density(ref, wl.z, wl.w))[A]
        print(f"  atom {A}: {F[A]} vs {Fr}", flush=True)
        assert np.abs(F[A] - Fr).max() <= 1e-9 * scale
    del res, eps
    torch.cuda.empty_cache()


def test_forces_skip_unconverged_columns(sgf, O):
    """With a small max_iter some columns stop at SGF_MAXITER.  The default
    status filter leaves them out: the forces equal the oracle's over the
    columns the GPU solve converged (the oracle's fully converged rho on
    those; which columns converge within max_iter is decided by the
    residual, and the two sides may freeze a column an iteration apart, so
    the mask is the GPU's).  Without the filter the stopped columns count
    too: the difference of the two force arrays is the oracle's force sum
    over the stopped columns, taken on the GPU's rho of those columns (an
    unconverged iterate near a resonance depends on rounding, so its rho is
    the GPU's own)."""
    O, fo = O
    wl = W.bundle_workload(2, 1, 14, config_no=121)
    cols = np.arange(wl.n_orb)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, cols, radius=1.0, prune=True)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12, max_iter=52)
    st = res.status.cpu().numpy()
    n_bad = int(np.sum(st != sgf.CONVERGED))
    print(f"  {n_bad} of {cols.size} columns stopped at max_iter", flush=True)
    assert 0 < n_bad < cols.size and np.all((st == sgf.CONVERGED) | (st == sgf.MAXITER))
    F = sgf.band_forces(prep, res, wl.tb).cpu().numpy()
    F_all = sgf.band_forces(prep, res, wl.tb, converged_only=False).cpu().numpy()
    b = O.system_for(wl)
    ref = O.shifted_solve(b, wl.xyz, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
    assert np.all(ref.status == 0)
    off = res.proj_off.cpu().numpy()
    np.testing.assert_array_equal(off, ref.proj_ptr)

    class Part:
        pass

    def part_of(sel, rho):
        p = Part()
        rows = np.concatenate([np.arange(off[c], off[c + 1]) for c in sel])
        p.proj_ptr = np.concatenate([[0], np.cumsum(off[sel + 1] - off[sel])])
        p.proj_row, p.rho = ref.proj_row[rows], rho[rows]
        return p

    ok, bad = np.nonzero(st == sgf.CONVERGED)[0], np.nonzero(st != sgf.CONVERGED)[0]
    Fr = fo.band_forces(wl.xyz, wl.tb, part_of(ok, ref.rho), cols[ok], wl.n_atoms)
    Fr_bad = fo.band_forces(wl.xyz, wl.tb, part_of(bad, res.rho.cpu().numpy()), cols[bad], wl.n_atoms)
    scale = np.abs(F_all).max()
    e = np.abs(F - Fr).max() / np.abs(Fr).max()
    e_all = np.abs((F_all - F) - Fr_bad).max() / scale
    print(f"  converged only: rel err {e:.2e}; stopped columns' share: {e_all:.2e}", flush=True)
    assert e < 1e-9 and e_all < 1e-12
    assert np.abs(Fr_bad).max() > 1e-3 * scale
