"""Host logic of the autotuner: candidate sets and the JSON cache."""
import types

from paper_1603_09616_amd import autotune as AT


def totals(atoms=15, row_blocks=5, proj=5):
    return types.SimpleNamespace(max_loc_atoms=atoms, max_row_blocks=row_blocks, max_proj_atoms=proj)


def test_candidates_follow_the_workload_shape():
    c = AT.candidates(totals(), "fp64", False)
    assert {x["stage_lds"] for x in c} == {-1, 0, 1, 3, 5}
    assert {x["shifts_per_lane"] for x in c} == {1, 2}
    # large subspaces: no register variant; wide projections: one shift per lane
    c = AT.candidates(totals(atoms=60, proj=7), "fp64", False)
    assert {x["stage_lds"] for x in c} == {-1, 0} and {x["shifts_per_lane"] for x in c} == {1}
    # mixed precision has a single seed variant, and so has S != I when no
    # subspace is larger than 16 atoms; above, one and two wavefronts per
    # column (per-atom inverse: 4, orbital-level inverse: 2)
    assert {x["stage_lds"] for x in AT.candidates(totals(), "mixed", False)} == {-1}
    assert {x["stage_lds"] for x in AT.candidates(totals(), "fp64", True)} == {-1}
    assert {x["stage_lds"] for x in AT.candidates(totals(atoms=21), "fp64", True, True)} == {-1, 4}
    assert {x["stage_lds"] for x in AT.candidates(totals(atoms=21), "fp64", True)} == {-1, 2}


def test_signature_separates_shapes():
    a = AT.signature(totals(), 128, "fp64", False, "dev")
    assert a != AT.signature(totals(), 256, "fp64", False, "dev")
    assert a != AT.signature(totals(atoms=14), 128, "fp64", False, "dev")
    assert a != AT.signature(totals(), 128, "mixed", False, "dev")
    assert a != AT.signature(totals(), 128, "fp64", True, "dev")


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert AT._load(p) == {}
    AT._store(p, {"k": {"choice": {"grid": 0}}})
    assert AT._load(p)["k"]["choice"] == {"grid": 0}
