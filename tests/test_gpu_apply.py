"""GPU tests of the global operator apply y = (z S - H) x against the oracle.

Bar: FP64 within 1e-13 of the oracle normwise (max |dy| / max |y|; both
sides sum at most a handful of blocks per row, so they differ only by
rounding order); FP32 (operator and vectors rounded to FP32) within 2e-6.
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
    return oracle


def seeded_x(n, k, seed):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))
    return x[:, 0] if k == 1 else x


@pytest.mark.parametrize("overlap", [False, True])
@pytest.mark.parametrize("n_rhs", [1, 2, 4, 8])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_vs_oracle(sgf, O, overlap, n_rhs, precision):
    import torch
    wl = W.bundle_workload(3, 2, 50, overlap=overlap, n_shifts=8, config_no=110)
    b = O.system_for(wl)
    s = sgf.system_for(wl)
    z = complex(wl.z[3])
    x = seeded_x(4 * b.n_atoms, n_rhs, 7 + n_rhs)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    y = sgf.bsr_apply(s, z, torch.as_tensor(x, dtype=dt, device="cuda").contiguous(), precision).cpu().numpy()
    ref = O.apply(b, z, x)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"  {precision} n_rhs {n_rhs} overlap {overlap}: normwise err {err:.2e}")
    assert err < (1e-13 if precision == "fp64" else 2e-6)


def test_apply_large_share_sampled_rows(sgf, O):
    """The 1,000,300-atom share (4,001,200 orbitals), 8 right-hand sides,
    FP64: 256 seeded rows recomputed by the oracle."""
    import torch
    wl = W.config_large(n_columns=16)
    s = sgf.system_for(wl)
    n = 4 * s.n_atoms
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.complex(torch.randn((n, 8), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((n, 8), dtype=torch.float64, device="cuda", generator=g)).contiguous()
    z = complex(wl.z[100])
    y = sgf.bsr_apply(s, z, x)
    rows = np.sort(np.random.default_rng(11).choice(n, 256, replace=False))
    # the oracle's block rows touch only neighbour atoms: copy the inputs it reads
    b = O.system_for(wl)
    need = set()
    for i in rows:
        a = int(i) // 4
        for t in range(b.row_ptr[a], b.row_ptr[a + 1]):
            need.update(range(4 * int(b.col[t]), 4 * int(b.col[t]) + 4))
        need.add(int(i))
    need = np.array(sorted(need))
    xh = np.zeros((n, 8), np.complex128)
    xh[need] = x[torch.as_tensor(need, device="cuda")].cpu().numpy()
    ref = O.apply(b, z, xh, rows=rows)
    got = y[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  large share: {s.n_atoms} atoms, {s.nnzb} blocks; sampled-row err {err:.2e}")
    assert err < 1e-13


def test_apply_argument_errors(sgf):
    import torch
    wl = W.bundle_workload(1, 1, 10, n_shifts=4, config_no=111)
    s = sgf.system_for(wl)
    x = torch.zeros((4 * s.n_atoms, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(sgf.SgfError) as e:
        sgf.bsr_apply(s, 1j, x)
    assert e.value.code == sgf.SGF_EINVAL
