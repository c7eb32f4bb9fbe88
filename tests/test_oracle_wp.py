"""Pins for the wavepacket-propagation oracle (oracle/wp.py), each against
something other than its own series code:

* the scalar series: sum_k c_k T_k(x) = exp(-i a tau x) on [-1, 1];
* the uniform chain's closed-form eigenpairs;
* the dense eigen-decomposition (the definition exp(-i H t / hbar));
* invariants: norm and energy conservation, time reversal;
* Gershgorin bounds by brute force on the dense matrix;
* a truncated series fails the bar (the cut is where it matters).
"""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def wp(oracle_lib):
    from oracle import wp
    return wp


def small_bundle():
    return W.bundle_workload(2, 1, 20, config_no=97)


def test_series_reproduces_the_scalar_exponential(wp):
    for a_tau in (0.3, 4.56, 17.0):
        K = wp.chebyshev_terms(a_tau, 1e-15)
        c = wp.chebyshev_coefficients(a_tau, K)
        x = np.linspace(-1.0, 1.0, 81)
        T = np.cos(np.outer(np.arccos(x), np.arange(K)))  # T_k(x) = cos(k arccos x)
        got = T @ c
        assert np.abs(got - np.exp(-1j * a_tau * x)).max() < 1e-14, a_tau
        assert K > a_tau


def test_gershgorin_by_brute_force(wp, oracle_lib):
    O = oracle_lib
    wl = small_bundle()
    b = O.system_for(wl)
    H = b.dense("h")
    off = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
    lo, hi = wp.gershgorin_bounds(b)
    assert abs(lo - (np.diag(H) - off).min()) < 1e-12 and abs(hi - (np.diag(H) + off).max()) < 1e-12
    lam = np.linalg.eigvalsh(H)
    assert lo <= lam.min() and lam.max() <= hi


def test_chebyshev_equals_eigen_propagation(wp, oracle_lib):
    """30 steps of 0.1 fs on a 160-orbital bundle, two packets."""
    O = oracle_lib
    wl = small_bundle()
    b = O.system_for(wl)
    psi0 = W.wavepacket(wl, 2)
    lo, hi = wp.gershgorin_bounds(b)
    a_tau = 0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS
    K = wp.chebyshev_terms(a_tau, 1e-14)
    got = wp.chebyshev_propagate(b, psi0, 0.1, 30, lo, hi, K)
    ref = wp.exact_propagate(b, psi0, 3.0)
    err = np.abs(got - ref).max()
    print(f"  K = {K}, a tau = {a_tau:.2f}, max |dPsi| = {err:.2e}")
    assert err < 1e-11


def test_uniform_chain_closed_form(wp, oracle_lib):
    """Uniform chain (on-site 0, hopping t): lambda_m = 2 t cos(m pi / (N+1)),
    v_m(j) = sqrt(2/(N+1)) sin(j m pi / (N+1)); exp(-i H t/hbar) psi from
    those, not from a numerical eigen-solver."""
    O = oracle_lib
    N, t = 64, -1.0
    wl = W.chain_workload(N, 1, 4, disorder=0.0, hopping=t, config_no=98)
    b = O.chain_build(np.zeros(N), t)
    psi0 = W.wavepacket(wl, 1, width=3.0, k_z=0.7)[:, 0]
    m = np.arange(1, N + 1)
    lam = 2 * t * np.cos(m * np.pi / (N + 1))
    V = np.sqrt(2 / (N + 1)) * np.sin(np.outer(np.arange(1, N + 1), m) * np.pi / (N + 1))
    T_fs = 2.5
    ref = V @ (np.exp(-1j * lam * T_fs / wp.HBAR_EV_FS) * (V.T @ psi0))
    lo, hi = wp.gershgorin_bounds(b)
    K = wp.chebyshev_terms(0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS, 1e-14)
    got = wp.chebyshev_propagate(b, psi0, 0.1, 25, lo, hi, K)
    assert np.abs(got - ref).max() < 1e-12


def test_norm_and_energy_are_conserved(wp, oracle_lib):
    O = oracle_lib
    wl = small_bundle()
    b = O.system_for(wl)
    H = b.dense("h")
    psi0 = W.wavepacket(wl, 1)[:, 0]
    lo, hi = wp.gershgorin_bounds(b)
    K = wp.chebyshev_terms(0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS, 1e-14)
    psi = wp.chebyshev_propagate(b, psi0, 0.1, 200, lo, hi, K)
    e0 = np.vdot(psi0, H @ psi0).real
    e1 = np.vdot(psi, H @ psi).real
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    assert abs(e1 - e0) < 1e-10 * max(abs(lo), abs(hi))


def test_time_reversal(wp, oracle_lib):
    O = oracle_lib
    wl = small_bundle()
    b = O.system_for(wl)
    psi0 = W.wavepacket(wl, 1)[:, 0]
    lo, hi = wp.gershgorin_bounds(b)
    K = wp.chebyshev_terms(0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS, 1e-14)
    fwd = wp.chebyshev_propagate(b, psi0, 0.1, 40, lo, hi, K)
    back = wp.chebyshev_propagate(b, fwd, -0.1, 40, lo, hi, K)
    assert np.abs(back - psi0).max() < 1e-12


def test_truncated_series_fails(wp, oracle_lib):
    """The rule's cut meets the bar; ten terms fewer misses it by far (the
    error grows about 30x per two terms dropped at a tau = 8.3)."""
    O = oracle_lib
    wl = small_bundle()
    b = O.system_for(wl)
    psi0 = W.wavepacket(wl, 1)[:, 0]
    lo, hi = wp.gershgorin_bounds(b)
    K = wp.chebyshev_terms(0.5 * (hi - lo) * 0.1 / wp.HBAR_EV_FS, 1e-14)
    ref = wp.exact_propagate(b, psi0, 0.5)
    good = wp.chebyshev_propagate(b, psi0, 0.1, 5, lo, hi, K)
    bad = wp.chebyshev_propagate(b, psi0, 0.1, 5, lo, hi, K - 10)
    assert np.abs(good - ref).max() < 1e-13
    assert np.abs(bad - ref).max() > 1e-7
