"""GPU tests of the band forces F = -dE_band/dR at fixed rho (S = I).

Bar: the forces sum rho-weighted block gradients, so the GPU and oracle
forces differ by the rho difference of the two solves (<= 1e-10 relative
per column) propagated through those sums: 1e-9 relative to the largest
force.  At full size, an atom's force depends only on its own columns and
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


def test_forces_need_an_orthogonal_basis(sgf):
    wl = W.bundle_workload(2, 1, 14, overlap=True, config_no=120)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns[:8], radius=1.0)
    res = sgf.solve_prepared(prep, wl.z, wl.w, tol=1e-12)
    with pytest.raises(sgf.SgfError):
        sgf.band_forces(prep, res, wl.tb)
