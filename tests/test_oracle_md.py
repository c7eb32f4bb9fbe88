"""Pins of the velocity-Verlet oracle against closed forms: a constant force
(Verlet is exact for constant acceleration), the one-step map of a harmonic
oscillator, energy behaviour and time reversibility."""
import numpy as np

from oracle import md


def test_unit_of_acceleration():
    # 1 eV/nm on 1 amu: (1.602176634e-19 / 1e-9 N) / 1.66053906660e-27 kg in m/s^2, then nm/fs^2
    a_si = (1.602176634e-19 / 1e-9) / 1.66053906660e-27
    assert abs(md.ACCEL - a_si * 1e9 / 1e30) <= 1e-15 * md.ACCEL
    assert abs(md.ACCEL - 9.6485332157e-5) < 1e-14


def test_constant_force_is_exact():
    rng = np.random.default_rng(0)
    x0, v0 = rng.normal(size=(5, 3)), rng.normal(size=(5, 3)) * 0.01
    F = rng.normal(size=(5, 3)) * 10
    m = rng.uniform(1, 20, size=5)
    a = md.accel(F, m)
    x, v, f = x0, v0, F
    h = 0.7
    for n in range(1, 11):
        x, v, f = md.verlet_step(x, v, f, m, h, lambda y: F)
        t = n * h
        np.testing.assert_allclose(x, x0 + v0 * t + 0.5 * a * t * t, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(v, v0 + a * t, rtol=1e-13, atol=1e-13)


def test_harmonic_oscillator_one_step_map():
    """F = -k x: one step maps (x, v) by the matrix
    [[1 - w^2 h^2 / 2, h], [-w^2 h (1 - w^2 h^2 / 4), 1 - w^2 h^2 / 2]],
    w^2 = k ACCEL / m."""
    k, m, h = 50.0, 12.0, 1.0
    w2 = k * md.ACCEL / m
    A = np.array([[1 - w2 * h * h / 2, h], [-w2 * h * (1 - w2 * h * h / 4), 1 - w2 * h * h / 2]])
    x, v = np.array([[0.01, -0.02, 0.03]]), np.array([[0.001, 0.002, -0.0005]])
    xn, vn, _ = md.verlet_step(x, v, -k * x, np.array([m]), h, lambda y: -k * y)
    for d in range(3):
        want = A @ np.array([x[0, d], v[0, d]])
        assert abs(xn[0, d] - want[0]) <= 1e-15 and abs(vn[0, d] - want[1]) <= 1e-15
    # the map has determinant 1 (symplectic)
    assert abs(np.linalg.det(A) - 1) < 1e-14


def test_harmonic_energy_and_reversal():
    k, m, h = 50.0, 12.0, 1.0
    w2 = k * md.ACCEL / m
    x0, v0 = np.array([[0.01, 0.0, 0.0]]), np.array([[0.0, 0.001, 0.0]])
    force = lambda y: -k * y
    x, v, f = x0, v0, force(x0)

    def energy(x, v):
        return 0.5 * m * (v ** 2).sum() / md.ACCEL + 0.5 * k * (x ** 2).sum()
    e0 = energy(x0, v0)
    worst = 0.0
    for _ in range(2000):
        x, v, f = md.verlet_step(x, v, f, np.array([m]), h, force)
        worst = max(worst, abs(energy(x, v) - e0))
    # Verlet keeps the energy within O((w h)^2) of its start, with no drift
    assert worst <= 0.5 * w2 * h * h * e0
    for _ in range(2000):
        x, v, f = md.verlet_step(x, v, f, np.array([m]), -h, force)
    np.testing.assert_allclose(x, x0, atol=1e-13)
    np.testing.assert_allclose(v, v0, atol=1e-14)
