"""GPU tests of the learned scheduler: features, the network's forward pass,
gradient and Adam step against the FP64 oracle, training on logged solves,
and the order it produces leaving every result unchanged."""
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


def synthetic_batch(n, seed):
    """Seeded feature rows shaped like the bundle's and smooth targets."""
    g = np.random.default_rng(seed)
    x = np.column_stack([g.integers(1, 5, n), g.uniform(1, 20, n), g.uniform(1.5, 50, n), g.uniform(0, 0.5, n),
                         4 * g.integers(7, 16, n)]).astype(np.float64)
    t = np.log(60 + 8 * x[:, 0] + 2 * x[:, 1] + g.normal(0, 3, n))
    p = W.mlp_init(seed)
    p[0:5] = x.mean(0)
    p[5:10] = 1 / x.std(0)
    return x, t, p


@pytest.mark.parametrize("kind", ["bundle", "chain"])
def test_features_vs_oracle(sgf, O, kind):
    import oracle.mlp as M
    if kind == "bundle":
        wl = W.bundle_workload(3, 2, 40, n_shifts=16, config_no=84)
        cols = wl.columns[::5]
    else:
        wl = W.chain_workload(200, 12, 16, config_no=85)
        cols = wl.columns
    b = O.system_for(wl)
    prep = sgf.prepare(sgf.system_for(wl), cols, radius=wl.radius, prune=True)
    got = sgf.features(prep).cpu().numpy()
    for i, j in enumerate(cols):
        full = O.solve_full(b, wl.xyz, int(j), wl.z[:1], radius=wl.radius, prune=True, max_iter=1)
        ref = M.features(b, full.loc_atoms, int(j))
        np.testing.assert_allclose(got[i], ref, rtol=2e-6, atol=1e-6)


def test_forward_gradient_adam_vs_oracle(sgf):
    import torch
    import oracle.mlp as M
    x, t, p = synthetic_batch(128, 11)
    model = sgf.IterationModel(p)
    dx = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    dt = torch.as_tensor(t, dtype=torch.float32, device="cuda")
    # FP32 GPU vs FP64 oracle on the FP32-rounded inputs
    p32 = p.astype(np.float32).astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    y = model.predict(dx).cpu().numpy()
    yr = M.forward(p32, x32)
    assert np.abs(y - yr).max() / np.abs(yr).max() < 1e-5
    g, loss = model.gradient(dx, dt)
    lr_, gr = M.loss_and_grad(p32, x32, t32)
    g = g.cpu().numpy()
    err = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"  gradient normwise rel err {err:.2e}")
    assert err < 1e-4
    assert abs(float(loss.cpu()) - lr_) / lr_ < 1e-5
    model.train_step(dx, dt, lr=1e-3)
    # the Adam arithmetic is checked on the GPU's own gradient: a first step
    # moves each weight by lr * g / (|g| + eps), so entries whose gradient is
    # rounding noise would otherwise flip sign between FP32 and FP64
    q, _, _ = M.adam_step(p32, np.zeros_like(p32), np.zeros_like(p32), g.astype(np.float64), 1, 1e-3)
    got = model.params.cpu().numpy()
    assert np.abs(got - q).max() < 1e-6


def test_training_step_is_bitwise_reproducible(sgf):
    import torch
    x, t, p = synthetic_batch(100, 12)
    dx = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    dt = torch.as_tensor(t, dtype=torch.float32, device="cuda")
    runs = []
    for _ in range(2):
        m = sgf.IterationModel(p)
        for _ in range(5):
            m.train_step(dx, dt)
        runs.append(m.params.cpu().numpy())
    np.testing.assert_array_equal(runs[0], runs[1])


def test_train_on_logged_solves_and_schedule(sgf):
    """Train on iteration counts logged by GPU solves of one bundle, predict
    another (different seed), and check that the learned order is a
    permutation that leaves G and rho bit for bit unchanged."""
    import torch
    train_wl = W.bundle_workload(4, 4, 300, n_shifts=128, config_no=20)
    s_tr = sgf.system_for(train_wl)
    prep = sgf.prepare(s_tr, train_wl.columns, radius=train_wl.radius, prune=True)
    res = sgf.solve_prepared(prep, train_wl.z, train_wl.w, tol=train_wl.tol, g_out=False)
    feat = sgf.features(prep)
    target = torch.log(res.iters.to(torch.float32))
    model = sgf.IterationModel(W.mlp_init(3))
    hist, test_mse = model.fit(feat, target, epochs=15, lr=1e-3, seed=4)
    var = float(target.var())
    print(f"  train loss {hist[0]:.4f} -> {hist[-1]:.4f}; held-out MSE {test_mse:.4f} vs variance {var:.4f}")
    assert hist[-1] < hist[0]
    assert test_mse < 0.8 * var

    wl = W.bundle_workload(4, 4, 300, n_shifts=128, config_no=21)
    s = sgf.system_for(wl)
    prep2 = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    pred = model.predict(sgf.features(prep2))
    order = sgf.order_by_prediction(pred, 0.0, float(np.log(10 * 4 * 16)))
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(wl.columns.size))
    po = pred.cpu().numpy()[o]
    # longest predicted first, up to the bucket width
    assert np.all(np.diff(po) <= np.log(640) / 4096 + 1e-6)
    a = sgf.solve_prepared(prep2, wl.z, wl.w, tol=wl.tol).numpy()
    b = sgf.solve_prepared(prep2, wl.z, wl.w, tol=wl.tol, order=o).numpy()
    np.testing.assert_array_equal(a.G, b.G)
    np.testing.assert_array_equal(a.rho, b.rho)
    np.testing.assert_array_equal(a.iters, b.iters)


def test_order_many_chunks_crowded_buckets(sgf):
    """The counting sort over several 8192-prediction chunks and a ragged
    tail, with most predictions in a handful of buckets (as a trained
    scheduler gives) and some outside [y_lo, y_hi] (clamped)."""
    import torch
    g = np.random.default_rng(9)
    n = 3 * 8192 + 517
    pred = np.where(g.random(n) < 0.8, g.choice([1.0, 1.5, 2.0], n), g.uniform(-0.5, 3.5, n)).astype(np.float32)
    order = sgf.order_by_prediction(torch.as_tensor(pred, device="cuda"), 0.0, 3.0)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(n))
    po = np.clip(pred[o], 0.0, 3.0)
    assert np.all(np.diff(po) <= 3.0 / 4096 + 1e-6)


def test_grouped_order_keeps_plans_together(sgf):
    """sgf_order_groups_by_prediction: a permutation in which the columns of
    each plan are contiguous and the plans come by their largest prediction
    (bucket resolution), with columns of an out-of-range plan last; a solve
    in that order gives the natural order's bits."""
    import torch
    wl = W.bundle_workload(3, 3, 40, n_shifts=64, config_no=170)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius)
    pred = torch.as_tensor(np.random.default_rng(5).uniform(3.0, 6.0, wl.columns.size).astype(np.float32),
                           device="cuda")
    n_plans = prep.plan.n_plans
    order = sgf.order_groups_by_prediction(pred, prep.col_plan, n_plans, 0.0, float(np.log(4096.0))).cpu().numpy()
    assert sorted(order.tolist()) == list(range(wl.columns.size))
    cp = prep.col_plan.cpu().numpy()[order]
    runs = np.concatenate([[0], np.nonzero(np.diff(cp))[0] + 1])
    assert len(runs) == n_plans                       # one run per plan
    pk = np.full(n_plans, -1.0)
    np.maximum.at(pk, prep.col_plan.cpu().numpy(), pred.cpu().numpy())
    b = np.floor((np.log(4096.0) - pk[cp[runs]]) / np.log(4096.0) * 4096)
    assert np.all(np.diff(b) >= -1)                   # largest first (to a bucket: FP32 keys)
    # an out-of-range plan index goes last
    bad = prep.col_plan.clone()
    bad[7] = n_plans + 3
    o2 = sgf.order_groups_by_prediction(pred, bad, n_plans, 0.0, float(np.log(4096.0))).cpu().numpy()
    assert o2[-1] == 7 and sorted(o2.tolist()) == list(range(wl.columns.size))
    a = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    g = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, order=torch.as_tensor(order, device="cuda")).numpy()
    np.testing.assert_array_equal(a.G, g.G)
    np.testing.assert_array_equal(a.rho, g.rho)


def test_learned_order_balances_plain_launches(sgf):
    """What the trained network gains over the natural order: the network is
    trained on solves of one bundle and orders the columns of another into
    fixed launches of 2048 columns.  A launch this small gives each
    wavefront at most one column group, so it lasts as long as its slowest
    column; the sum over launches of the largest iteration count is the
    modelled cost.  The learned order must cost less than the natural one
    (and no less than the order by the true counts); the measured times of
    the two launch sequences are printed beside it."""
    import time
    import torch
    train_wl = W.bundle_workload(6, 6, 400, n_shifts=128, config_no=20)
    s_tr = sgf.system_for(train_wl)
    prep_tr = sgf.prepare(s_tr, train_wl.columns, radius=train_wl.radius, prune=True)
    res_tr = sgf.solve_prepared(prep_tr, train_wl.z, train_wl.w, tol=train_wl.tol, g_out=False)
    feat = sgf.features(prep_tr)
    target = torch.log(res_tr.iters.to(torch.float32))
    model = sgf.IterationModel(W.mlp_init(3))
    hist, test_mse = model.fit(feat, target, epochs=20, lr=1e-3, seed=4)
    var = float(target.var())
    del prep_tr, res_tr, s_tr

    wl = W.bundle_workload(6, 6, 400, n_shifts=128, config_no=21)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    nat = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=False)
    it = nat.iters.cpu().numpy()
    pred = model.predict(sgf.features(prep)).cpu().numpy()
    heldout_r2 = 1.0 - np.mean((pred - np.log(it)) ** 2) / np.var(np.log(it))
    learned = sgf.learned_order(prep, model).cpu().numpy()
    # the order by the true counts, plans together (the bound for any order)
    cp = prep.col_plan.cpu().numpy()
    pk = np.zeros(prep.plan.n_plans)
    np.maximum.at(pk, cp, it)
    best = np.lexsort((cp, -pk[cp]))
    B = 2048

    def cost(order):
        o = np.arange(it.size) if order is None else order
        return sum(int(it[o[i:i + B]].max()) for i in range(0, o.size, B))

    c_nat, c_lrn, c_best = cost(None), cost(learned), cost(best)

    def timed(order):
        ts = []
        od = None if order is None else torch.as_tensor(order.astype(np.int32), device="cuda")
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, g_out=False, batch_cols=B, order=od)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts[1:])), r

    t_nat, r_nat = timed(None)
    t_lrn, r_lrn = timed(learned)
    print(f"  held-out MSE {test_mse:.4f} vs variance {var:.4f} (training geometry); other geometry R^2 "
          f"{heldout_r2:.3f}; modelled launch cost natural {c_nat}, learned {c_lrn}, by true counts {c_best} "
          f"(gain {c_nat / c_lrn:.3f}, bound {c_nat / c_best:.3f}); measured {t_nat * 1e3:.1f} ms natural, "
          f"{t_lrn * 1e3:.1f} ms learned (gain {t_nat / t_lrn:.3f})", flush=True)
    np.testing.assert_array_equal(r_nat.rho.cpu().numpy(), r_lrn.rho.cpu().numpy())
    assert test_mse < 0.8 * var
    assert c_best <= c_lrn < c_nat
