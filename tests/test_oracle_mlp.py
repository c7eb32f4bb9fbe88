"""Pins of the FP64 iteration-count network: backward pass against central
finite differences, Adam against its closed form on a quadratic."""
import numpy as np

import oracle.mlp as M
import workloads as W


def test_gradient_matches_central_differences():
    p = W.mlp_init(seed=5)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(40, M.NF)) * 3 + 5
    p[0:M.NF] = x.mean(0)
    p[M.NF:2 * M.NF] = 1 / x.std(0)
    t = rng.normal(size=40) + 4
    loss, g = M.loss_and_grad(p, x, t)
    h = 1e-5
    idx = np.concatenate([rng.choice(np.arange(M.OFF_W1, M.NPARAM), 60, replace=False), [M.OFF_B3, M.OFF_B1]])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss_and_grad(p + e, x, t)[0] - M.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert np.all(g[:M.OFF_W1] == 0)
    assert abs(loss - np.mean((M.forward(p, x) - t) ** 2)) < 1e-12


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected moments are g and g^2,
    so Adam moves each weight by exactly -lr g / (|g| + eps)."""
    p = W.mlp_init(seed=2)
    g = np.zeros_like(p)
    g[M.OFF_W1:] = np.linspace(-1, 1, M.NPARAM - M.OFF_W1) + 0.01
    q, m, v = M.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, 1, 1e-3)
    gg = g[M.OFF_W1:]
    np.testing.assert_allclose(q[M.OFF_W1:] - p[M.OFF_W1:], -1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-9)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(512, M.NF))
    t = np.sin(3 * x[:, 0]) + x[:, 1] ** 2
    p = W.mlp_init(seed=9)
    p[0:M.NF] = x.mean(0)
    p[M.NF:2 * M.NF] = 1 / x.std(0)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss_and_grad(p, x, t)[0]
    for step in range(1, 301):
        b = rng.choice(512, 64, replace=False)
        _, g = M.loss_and_grad(p, x[b], t[b])
        p, m, v = M.adam_step(p, m, v, g, step, 3e-3)
    assert M.loss_and_grad(p, x, t)[0] < 0.1 * l0


# --- features, pinned against hand-computed cases -------------------------------
# The Slater-Koster block of a bond along +z at distance r (direction cosines
# (0, 0, 1)) has, with f = (r0/r)^2: row s = (Vss, 0, 0, Vsp) f,
# rows px, py = Vpp_pi f on their own diagonal, row pz = (-Vsp, 0, 0, Vpp_sigma) f.
# So the row norms ||H_cb[o, :]||_2 are closed forms, and a Frobenius norm of
# the whole block (sqrt(Vss^2 + 2 Vsp^2 + Vpps^2 + 2 Vppp^2) f) differs from
# every one of them.

def _row_norms_along_z(tb, r):
    f = (tb.r0 / r) ** tb.power
    return np.array([np.hypot(tb.v_sss, tb.v_sps), abs(tb.v_ppp), abs(tb.v_ppp), np.hypot(tb.v_sps, tb.v_pps)]) * f


def test_features_isolated_atom():
    import oracle
    b = oracle.tb_build(np.zeros((1, 3)), W.BUNDLE_TB)
    for o in range(4):
        f = M.features(b, np.array([0]), o)
        np.testing.assert_array_equal(f, [0.0, 0.0, 0.0, 0.0, 4.0])


def test_features_dimer_along_z():
    import oracle
    tb = W.BUNDLE_TB
    r = 0.15
    b = oracle.tb_build(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]]), tb)
    want = _row_norms_along_z(tb, r)
    frob = np.sqrt(tb.v_sss ** 2 + 2 * tb.v_sps ** 2 + tb.v_pps ** 2 + 2 * tb.v_ppp ** 2) * (tb.r0 / r) ** 2
    for atom in (0, 1):
        for o in range(4):
            f = M.features(b, np.array([0, 1]), 4 * atom + o)
            assert f[0] == 1.0                      # one off-diagonal block; the diagonal one is not counted
            assert abs(f[1] - want[o]) <= 1e-13 * want[o]
            assert f[2] == f[1]                     # one block: mean == max
            assert abs(f[1] - frob) > 1e-3 * frob   # the row norm, not the block's Frobenius norm
            assert f[3] == 0.0                      # both atoms carry the same on-site energies
            assert f[4] == 8.0
    # the same column on a subspace that leaves the partner out sees no block
    np.testing.assert_array_equal(M.features(b, np.array([0]), 2), [0.0, 0.0, 0.0, 0.0, 4.0])


def test_features_three_atom_chain_with_onsite_energies():
    """Atoms on the z axis at 0, r1 and r1 + r2 (both bonds within the cutoff,
    the end pair beyond it), with on-site energies set per orbital."""
    import oracle
    tb = W.BUNDLE_TB
    r1, r2 = 0.14, 0.16
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r1], [0.0, 0.0, r1 + r2]])
    onsite = np.array([[-8.0, 0.1, 0.2, 0.3],
                       [-7.0, 0.5, -0.4, 0.9],
                       [-8.6, -0.3, 0.8, 0.0]])
    b = oracle.tb_build(xyz, tb, onsite=onsite.reshape(-1))
    n1, n2 = _row_norms_along_z(tb, r1), _row_norms_along_z(tb, r2)
    loc = np.array([0, 1, 2])
    for o in range(4):
        f = M.features(b, loc, 4 + o)   # the middle atom: two off-diagonal blocks
        assert f[0] == 2.0
        assert abs(f[1] - 0.5 * (n1[o] + n2[o])) <= 1e-13 * n1[o]
        assert abs(f[2] - max(n1[o], n2[o])) <= 1e-13 * n1[o]
        # |H_jj - mean of the same orbital type over the three atoms|
        assert abs(f[3] - abs(onsite[1, o] - onsite[:, o].mean())) <= 1e-14
        assert f[4] == 12.0
        f_end = M.features(b, loc, 8 + o)   # the last atom: one block (bond r2)
        assert f_end[0] == 1.0
        assert abs(f_end[1] - n2[o]) <= 1e-13 * n2[o]
        assert abs(f_end[3] - abs(onsite[2, o] - onsite[:, o].mean())) <= 1e-14
    # the type mean runs over orbitals of the column's own type only: a mean over
    # all orbitals of the subspace would give a different value here
    wrong = abs(onsite[1, 1] - onsite.mean())
    assert abs(M.features(b, loc, 5)[3] - wrong) > 0.1
