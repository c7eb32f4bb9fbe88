"""GPU tests of the quantum-MD time step: the velocity-Verlet kernels against
the oracle's update, and whole steps (new H and S at the moved positions,
local subspaces, the shifted solve of every column, band forces, Verlet)
against the same steps taken by the oracle.

Bar: the kick and the drift are one multiply-add per coordinate, so they
agree with the oracle to a rounding (1e-15 relative).  Over whole steps the
positions and velocities inherit the force differences of the two solves
(1e-9 relative to the largest force), scaled by h^2/m and h/m."""
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
    from oracle import forces, md
    return oracle, forces, md


def test_kick_and_drift_vs_oracle(sgf, O):
    import torch
    _, _, md = O
    rng = np.random.default_rng(150)
    n = 1000
    x, v = rng.normal(size=(n, 3)), rng.normal(size=(n, 3)) * 1e-3
    F, m = rng.normal(size=(n, 3)) * 100, rng.uniform(1, 30, size=n)
    dx, dv = torch.as_tensor(x, device="cuda"), torch.as_tensor(v, device="cuda")
    sgf.md_kick(torch.as_tensor(F, device="cuda"), torch.as_tensor(m, device="cuda"), 0.8, dv)
    v_half = v + 0.5 * 0.8 * md.accel(F, m)
    np.testing.assert_allclose(dv.cpu().numpy(), v_half, rtol=1e-15, atol=1e-18)
    sgf.md_drift(dv, 0.8, dx)
    np.testing.assert_allclose(dx.cpu().numpy(), x + 0.8 * v_half, rtol=1e-15, atol=1e-16)
    with pytest.raises(sgf.SgfError):
        sgf.md_drift(dv, float("nan"), dx)


@pytest.mark.parametrize("overlap", [False, True])
def test_qmd_steps_vs_oracle(sgf, O, overlap):
    """Two 1 fs steps of a 28-atom bundle (two chains of 14 atoms), every
    column solved on its R = 1.0 nm pruned subspace at 128 shifts."""
    oracle, fo, md = O
    wl = W.bundle_workload(2, 1, 14, overlap=overlap, config_no=151)
    n = wl.n_atoms
    mass = np.full(n, 12.011)
    vel = np.random.default_rng(152).normal(size=(n, 3)) * 5e-4
    run = sgf.QMD(wl.xyz, vel, mass, wl.tb, wl.z, wl.w, tol=1e-12, radius=1.0)
    cols = np.arange(4 * n)

    def force_at(x):
        b = oracle.tb_build(x, wl.tb)
        r = oracle.shifted_solve(b, x, cols, wl.z, wl.w, tol=1e-12, radius=1.0, prune=True, threads=8)
        eps = fo.energy_density(r, wl.z, wl.w) if overlap else None
        return fo.band_forces(x, wl.tb, r, cols, n, eps=eps)

    x, v = wl.xyz.copy(), vel.copy()
    f = force_at(x)
    F0 = run.force.cpu().numpy()
    scale = np.abs(f).max()
    assert np.abs(F0 - f).max() <= 1e-9 * scale
    for step in range(2):
        run.step(1.0)
        x, v, f = md.verlet_step(x, v, f, mass, 1.0, force_at)
        gx, gv, gf = run.xyz.cpu().numpy(), run.vel.cpu().numpy(), run.force.cpu().numpy()
        ex, ev = np.abs(gx - x).max(), np.abs(gv - v).max() / np.abs(v).max()
        ef = np.abs(gf - f).max() / np.abs(f).max()
        print(f"  step {step + 1}: max |dx| {ex:.2e} nm, dv {ev:.2e}, dF {ef:.2e} (moved up to "
              f"{np.abs(x - wl.xyz).max():.2e} nm)", flush=True)
        assert ex <= 1e-12 and ev <= 1e-9 and ef <= 1e-9
    assert np.all(run.last[1].status.cpu().numpy() == sgf.CONVERGED)
