"""GPU test of the autotuner: a valid choice, cached, and every candidate
agreeing with the default launch (they differ only in rounding order)."""
import json

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


def test_tune_and_cache(sgf, tmp_path):
    from paper_1603_09616_amd import autotune as AT
    wl = W.bundle_workload(3, 3, 60, n_shifts=128, config_no=130)
    s = sgf.system_for(wl)
    prep = sgf.prepare(s, wl.columns, radius=wl.radius, prune=True)
    path = str(tmp_path / "tune.json")
    r = AT.tune(prep, wl.z, wl.w, wl.tol, sample=2048, reps=1, path=path)
    cands = AT.candidates(prep.plan.totals, "fp64", False)
    assert r["choice"] in cands and not r["cached"]
    assert set(r["timings_ms"]) == {json.dumps(c, sort_keys=True) for c in cands}
    r2 = AT.tune(prep, wl.z, wl.w, wl.tol, sample=2048, reps=1, path=path)
    assert r2["cached"] and r2["choice"] == r["choice"]
    base = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol).numpy()
    scale = np.abs(base.G).max()
    for c in cands:
        got = sgf.solve_prepared(prep, wl.z, wl.w, tol=wl.tol, **c).numpy()
        assert np.all(got.status == base.status)
        assert np.abs(got.G - base.G).max() / scale < 1e-10, c
