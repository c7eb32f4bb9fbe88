"""GPU tests of the wavepacket propagation (Chebyshev steps of
exp(-i H h / hbar)) against the oracle.

Bar: both sides evaluate the same truncated series in FP64, and they differ
by rounding only: 1e-12 in max |dPsi| for unit-norm packets after 30 steps.
Against the exact propagation (eigen-decomposition), 1e-11 (series cut at
tol 1e-14 per step).  At full size (1,000,300 atoms) the oracle is too slow,
so the properties the exact propagator has are checked instead: norm and
energy conservation and time reversal.
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
    from oracle import wp
    return oracle, wp


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("make", ["bundle", "chain"])
def test_bounds_match_oracle(sgf, O, make):
    O, wp = O
    wl = W.bundle_workload(3, 2, 40, config_no=160) if make == "bundle" else W.chain_workload(400, 1, 4, config_no=161)
    lo, hi = sgf.wp_bounds(sgf.system_for(wl))
    rlo, rhi = wp.gershgorin_bounds(O.system_for(wl))
    print(f"  bounds {lo:.6f} {hi:.6f}")
    assert abs(lo - rlo) <= 1e-12 * abs(rlo) and abs(hi - rhi) <= 1e-12 * abs(rhi)


@pytest.mark.parametrize("n_rhs", [1, 2, 4, 8])
def test_propagation_vs_oracle(sgf, O, n_rhs):
    O, wp = O
    wl = W.bundle_workload(2, 1, 20, config_no=97)
    b = O.system_for(wl)
    psi0 = W.wavepacket(wl, n_rhs)
    lo, hi = wp.gershgorin_bounds(b)
    K = wp.chebyshev_terms(0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS, 1e-14)
    ref = wp.chebyshev_propagate(b, psi0, 0.1, 30, lo, hi, K)
    exact = wp.exact_propagate(b, psi0, 3.0)
    psi = dev(psi0 if n_rhs > 1 else psi0[:, 0])
    sgf.wp_propagate(sgf.system_for(wl), psi, 0.1, 30, lo, hi, K)
    got = psi.cpu().numpy().reshape(ref.shape)
    e1, e2 = np.abs(got - ref).max(), np.abs(got - exact).max()
    print(f"  n_rhs {n_rhs}: K {K}, vs oracle series {e1:.2e}, vs exact {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-11


def test_batches_agree_bitwise(sgf):
    """Eight packets at once give each packet's single-packet result bit for bit."""
    wl = W.bundle_workload(3, 3, 60, config_no=162)
    s = sgf.system_for(wl)
    lo, hi = sgf.wp_bounds(s)
    K = sgf.wp_terms(0.5 * (hi - lo) * 0.1 / sgf.HBAR_EV_FS, 1e-13)
    psi0 = W.wavepacket(wl, 8)
    many = dev(psi0)
    sgf.wp_propagate(s, many, 0.1, 7, lo, hi, K)
    for p in range(8):
        one = dev(psi0[:, p])
        sgf.wp_propagate(s, one, 0.1, 7, lo, hi, K)
        np.testing.assert_array_equal(one.cpu().numpy(), many[:, p].cpu().numpy())


def test_zero_steps_and_unsupported(sgf):
    import torch
    wl = W.bundle_workload(2, 1, 20, config_no=97)
    s = sgf.system_for(wl)
    psi0 = W.wavepacket(wl, 1)[:, 0]
    psi = dev(psi0)
    sgf.wp_propagate(s, psi, 0.1, 0, -10.0, 10.0, 5)
    np.testing.assert_array_equal(psi.cpu().numpy(), psi0)
    wlo = W.bundle_workload(2, 1, 20, overlap=True, config_no=97)
    with pytest.raises(sgf.SgfError):
        sgf.wp_propagate(sgf.system_for(wlo), dev(psi0), 0.1, 1, -10.0, 10.0, 5)
    torch.cuda.synchronize()


def test_large_share_conservation_and_reversal(sgf):
    """1,000,300 atoms, 8 packets, 20 steps of 0.1 fs forward and 20 back:
    norms and energies conserved, and the packets return to the start."""
    import torch
    wl = W.config_large(n_columns=16)
    s = sgf.system_for(wl)
    lo, hi = sgf.wp_bounds(s)
    K = sgf.wp_terms(0.5 * (hi - lo) * 0.1 / sgf.HBAR_EV_FS, 1e-14)
    psi0 = dev(W.wavepacket(wl, 8))
    psi = psi0.clone()

    def energy(v):
        hv = torch.empty_like(v)
        sgf.bsr_apply(s, 0.0, v, out=hv)   # (0 S - H) v = -H v
        return -(v.conj() * hv).sum(0).real

    e0 = energy(psi0)
    sgf.wp_propagate(s, psi, 0.1, 20, lo, hi, K)
    norms = torch.linalg.vector_norm(psi, dim=0).cpu().numpy()
    moved = (psi - psi0).abs().max().item()
    e1 = energy(psi)
    sgf.wp_propagate(s, psi, -0.1, 20, lo, hi, K)
    back = (psi - psi0).abs().max().item()
    print(f"  K {K}; moved {moved:.2e}; norm drift {np.abs(norms - 1).max():.2e}; "
          f"energy drift {(e1 - e0).abs().max().item():.2e}; return {back:.2e}", flush=True)
    assert moved > 1e-2
    assert np.abs(norms - 1).max() < 1e-12
    assert (e1 - e0).abs().max().item() < 1e-10 * max(abs(lo), abs(hi))
    assert back < 1e-11
    del psi, psi0
    torch.cuda.empty_cache()
