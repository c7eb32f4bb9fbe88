"""GPU tests of the planning pass at its capacity edges.

The count pass first runs with a 256-atom LDS capacity and counts a batch
again at the caller's capacity when a subspace is larger; the fill is sized
from the largest counted subspace.  Chains of 255 to 600 four-site blocks,
pruned with no radius (the subspace is the whole connected chain), put the
subspace on both sides of that first capacity; the plans must equal the
oracle's exactly and the solve must match it to the FP64 bar.
"""
import ctypes

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
    return oracle


@pytest.mark.parametrize("n_atoms", [255, 256, 257, 600])
def test_whole_chain_plans(sgf, O, n_atoms):
    wl = W.chain_workload(4 * n_atoms, n_columns=6, n_shifts=16, config_no=130 + n_atoms)
    s = sgf.system_for(wl)
    b = O.system_for(wl)
    print(f"  chain of {n_atoms} blocks, pruned, no radius", flush=True)
    prep = sgf.prepare(s, wl.columns, radius=0.0, prune=True)
    t = prep.plan.totals
    assert t.max_loc_atoms == n_atoms
    n_loc, n_proj = O.plan_sizes(b, None, wl.columns, 0.0, None, True)
    cp = prep.col_plan.cpu().numpy()
    ao = prep.plan.atom_off.cpu().numpy()
    np.testing.assert_array_equal(np.diff(ao)[cp], n_loc)
    np.testing.assert_array_equal(np.diff(prep.proj_off.cpu().numpy()), n_proj)
    la = prep.plan.loc_atom.cpu().numpy()
    for p in range(prep.plan.n_plans):
        np.testing.assert_array_equal(la[ao[p]:ao[p + 1]], np.arange(n_atoms))
    # local block rows: the chain's stored blocks, in row order
    bo = prep.plan.blk_off.cpu().numpy()
    lrow = prep.plan.lrow.cpu().numpy()
    lblk = prep.plan.lblk.cpu().numpy().reshape(-1, 2)
    for p in range(prep.plan.n_plans):
        blk = lblk[bo[p]:bo[p + 1]]
        np.testing.assert_array_equal(blk[:, 1], np.arange(b.row_ptr[-1]))
        np.testing.assert_array_equal(blk[:, 0], b.col)
        np.testing.assert_array_equal(lrow[ao[p]:ao[p + 1]], b.row_ptr[:-1])
    got = sgf.shifted_solve(s, wl.columns, wl.z, wl.w, tol=wl.tol, radius=0.0, prune=True).numpy()
    ref = O.shifted_solve(b, None, wl.columns, wl.z, wl.w, tol=wl.tol, radius=0.0, prune=True, threads=8)
    np.testing.assert_array_equal(got.proj_off, ref.proj_ptr)
    np.testing.assert_array_equal(got.proj_row, ref.proj_row)
    np.testing.assert_array_equal(got.status, ref.status)
    # per column, relative to the column's largest entry (the parity bar)
    eg = er = 0.0
    for c in range(ref.proj_ptr.size - 1):
        a, e = ref.proj_ptr[c], ref.proj_ptr[c + 1]
        eg = max(eg, np.abs(got.G[a:e] - ref.G[a:e]).max() / np.abs(ref.G[a:e]).max())
        er = max(er, np.abs(got.rho[a:e] - ref.rho[a:e]).max() / max(np.abs(ref.rho[a:e]).max(), 1e-300))
    print(f"  G rel err {eg:.2e}  rho rel err {er:.2e}", flush=True)
    assert eg < 1e-10 and er < 1e-10


def test_capacity_limits(sgf):
    """A subspace one atom larger than max_loc_atoms is refused by the count,
    also when the LDS capacity (a power of two) would hold it; a fill with
    less than the counted maximum is refused as well."""
    wl = W.chain_workload(4 * 200, n_columns=2, n_shifts=4, config_no=140)
    s = sgf.system_for(wl)
    with pytest.raises(sgf.SgfError) as e:
        sgf.make_plan(s, [0], [0.0], prune=True, max_loc_atoms=199)
    assert e.value.code == sgf.SGF_EUNSUPPORTED
    plan = sgf.make_plan(s, [0, 10], [0.0, 0.0], prune=True, max_loc_atoms=200)
    assert plan.totals.max_loc_atoms == 200
    ws = ctypes.c_size_t()
    sc = s.c()
    sgf._call("sgf_plan_workspace", ctypes.byref(sc), plan.n_plans, 200, ctypes.byref(ws))
    d_ws = sgf._bytes(ws.value, s.row_ptr.device)
    pc = plan.c()
    bws = s.build_ws
    nb = 0 if bws is None else bws.numel()
    with pytest.raises(sgf.SgfError) as e:
        sgf._call("sgf_plan_build", ctypes.byref(sc), ctypes.byref(pc), 199, sgf._ptr(bws), nb, sgf._ptr(d_ws),
                  ws.value, None)
    assert e.value.code == sgf.SGF_EUNSUPPORTED


@pytest.mark.parametrize("n_cols", [0, 1, 2047, 2048, 2049, 4096, 4097, 6145])
def test_projection_layout_many_tiles(sgf, n_cols):
    """Output offsets and projection rows, recomputed on the host from the
    plans: all 43,200 columns (n_cols 0; the offsets' scan spans 22 tiles of
    2048 and a ragged tail) and column counts at the tile edges (one tile,
    exactly one or two full tiles, a full tile and one more)."""
    wl = W.bundle_workload(6, 6, 300, n_shifts=4, config_no=141)
    s = sgf.system_for(wl)
    cols = wl.columns if n_cols == 0 else wl.columns[:n_cols]
    print(f"  {cols.size} columns", flush=True)
    prep = sgf.prepare(s, cols, radius=wl.radius, prune=True)
    cp = prep.col_plan.cpu().numpy()
    pa_off = prep.plan.pa_off.cpu().numpy()
    ao = prep.plan.atom_off.cpu().numpy()
    la = prep.plan.loc_atom.cpu().numpy()
    pa_loc = prep.plan.pa_loc.cpu().numpy()
    npa = np.diff(pa_off)[cp]
    off = np.concatenate([[0], np.cumsum(4 * npa)])
    np.testing.assert_array_equal(prep.proj_off.cpu().numpy(), off)
    rows = np.empty(off[-1], np.int64)
    for c in range(cols.size):
        p = cp[c]
        atoms = la[ao[p] + pa_loc[pa_off[p]:pa_off[p + 1]]]
        rows[off[c]:off[c + 1]] = (4 * atoms[:, None] + np.arange(4)[None, :]).reshape(-1)
    np.testing.assert_array_equal(prep.proj_row.cpu().numpy(), rows)
