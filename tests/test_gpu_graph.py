"""GPU tests of the solve captured into a HIP graph.

Every replay is checked against the eager solve bit for bit (the kernels are
deterministic and the graph holds only kernel launches), with the program's
own eager work and synchronisations between replays and the outputs
overwritten before each one, so that a replay that did not run, or ran on
stale memory, cannot pass.
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


@pytest.mark.parametrize("batch", [0, 50])
def test_graph_replays_match_eager(sgf, batch):
    import torch
    wl = W.bundle_workload(3, 2, 40, n_shifts=128, config_no=120)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    ref = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, batch_cols=batch).numpy()
    order = torch.as_tensor(np.random.default_rng(2).permutation(wl.columns.size).astype(np.int32), device="cuda")
    g = sgf.SolveGraph(prep, wl.z, wl.w, tol=wl.tol, batch_cols=batch, order=order)
    for i in range(4):
        # eager work of the program between replays, and poisoned outputs
        e = sgf.solve_prepared(prep, wl.z[:64], wl.w[:64], tol=1e-8)
        torch.cuda.synchronize()
        g.result.G.fill_(float("nan"))
        g.result.rho.fill_(float("nan"))
        g.result.iters.fill_(-1)
        torch.cuda.synchronize()
        got = g.replay()
        torch.cuda.synchronize()
        r = got.numpy()
        np.testing.assert_array_equal(r.G, ref.G)
        np.testing.assert_array_equal(r.rho, ref.rho)
        np.testing.assert_array_equal(r.iters, ref.iters)
        np.testing.assert_array_equal(r.status, ref.status)
        del e


def test_graph_follows_new_hamiltonian_values(sgf):
    """Same bond pattern, new values written into H in place between
    replays (as in successive steps of a dynamics run): each replay equals
    an eager solve with the new values."""
    import torch
    wl = W.bundle_workload(2, 2, 40, n_shifts=64, config_no=121)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    g = sgf.SolveGraph(prep, wl.z, wl.w, tol=wl.tol)
    h0 = s.h.clone()
    for scale in (1.01, 0.97, 1.0):
        s.h.copy_(h0 * scale)
        torch.cuda.synchronize()
        got = g.replay()
        torch.cuda.synchronize()
        r = got.numpy()
        ref = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
        np.testing.assert_array_equal(r.G, ref.G)
        np.testing.assert_array_equal(r.rho, ref.rho)
    s.h.copy_(h0)
