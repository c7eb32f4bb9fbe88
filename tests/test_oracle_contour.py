"""Pins of the Fermi-Dirac pole expansion (oracle/contour.py): the poles
tend to the Matsubara frequencies (2p - 1) pi with unit residues, the
expansion reproduces the Fermi function to rounding over the range a local
spectrum covers, and the density matrix from the shifts and weights (with
the exact resolvent) equals f(H) from the eigen-decomposition, for S = I and
S != I, and gives the electron count sum f(lambda)."""
import numpy as np

from oracle import contour as C


def test_poles_tend_to_matsubara_frequencies():
    z, R = C.cf_poles(60)
    np.testing.assert_allclose(z[:5], (2 * np.arange(1, 6) - 1) * np.pi, rtol=1e-13)
    np.testing.assert_allclose(R[:5], 1.0, rtol=1e-12)
    assert np.all(np.diff(z) > 0) and np.all(R > 0)


def test_expansion_reproduces_fermi_function():
    for n, ymax, bar in ((20, 100, 1e-13), (40, 500, 1e-9), (60, 1000, 1e-12)):
        z, R = C.cf_poles(n)
        y = np.linspace(-ymax, ymax, 40001)
        assert np.abs(C.fermi_approx(y, z, R) - C.fermi(y)).max() <= bar
    # a truncated expansion tends to 1/2 far out, not to 0 or 1: it only holds
    # over a finite range, which is why the number of poles is chosen from it
    z, R = C.cf_poles(10)
    assert abs(C.fermi_approx(1e6, z, R) - 0.5) < 1e-3


def _resolvent_rho(H, S, z, w):
    rho = np.zeros_like(H)
    for zk, wk in zip(z, w):
        rho += -(wk * np.linalg.inv(zk * S - H)).imag / np.pi
    return rho


def test_shifts_give_the_fermi_density_matrix():
    rng = np.random.default_rng(5)
    n = 40
    A = rng.normal(size=(n, n))
    H = 8.0 * (A + A.T) / np.sqrt(n)
    B = rng.normal(size=(n, n)) * 0.05
    for S in (np.eye(n), np.eye(n) + (B + B.T) / 2):
        lam = np.linalg.eigvals(np.linalg.solve(S, H)).real
        kT, mu = 0.1, 0.3
        assert np.abs(lam - mu).max() / kT < 600
        z, w = C.fermi_shifts(48, kT, mu)
        rho = _resolvent_rho(H, S, z, w)
        want = C.fermi_rho_dense(H, S, kT, mu)
        err = np.abs(rho - want).max() / np.abs(want).max()
        assert err < 1e-10, err
        # electron count tr(rho S) = sum_lambda f(lambda)
        assert abs(np.trace(rho @ S) - C.fermi((lam - mu) / kT).sum()) < 1e-9


def test_low_temperature_limit_is_the_spectral_projector():
    """Below kT ~ gap / 40 the Fermi matrix is the projector on the states
    below mu, where mu sits in a gap."""
    rng = np.random.default_rng(6)
    lam = np.concatenate([rng.uniform(-20, -1, 15), rng.uniform(1, 20, 15)])
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    H = (Q * lam) @ Q.T
    z, w = C.fermi_shifts(60, 0.02, 0.0)
    rho = _resolvent_rho(H, np.eye(30), z, w)
    P = (Q[:, lam < 0]) @ Q[:, lam < 0].T
    assert np.abs(rho - P).max() < 1e-10
