"""The library's host-side electron count, band energy and Fermi level
(C functions in libsgf.so, no GPU involved) against the oracle's."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def sgf():
    import paper_1603_09616_amd as sgf
    sgf.lib()
    return sgf


def synthetic(n, seed):
    g = np.random.default_rng(seed)
    T = g.standard_normal(n) - (np.abs(g.standard_normal(n)) + 0.05) * 1j
    U = g.standard_normal(n) + 1j * g.standard_normal(n)
    return T, U


def test_occupation_matches_oracle(sgf, oracle_lib):
    O = oracle_lib
    z = W.shift_grid(-30, 30, 128, 0.01)
    T, U = synthetic(128, 1)
    for mu in (-31.0, -5.0, 0.0, 12.5, 31.0):
        w = W.occupied_weights(z, mu)
        got = sgf.occupation(T, U, w)
        ref = O.occupation(T, U, w)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 7, 128])
def test_fermi_level_matches_oracle(sgf, oracle_lib, n):
    O = oracle_lib
    z = W.shift_grid(-6, 6, n, 0.05)
    T, U = synthetic(n, 2 + n)
    top = O.occupation(T, U, W.occupied_weights(z, 7.0))[0]
    for frac in (0.05, 0.33, 0.5, 0.71, 0.999):
        mu, ne, eb = sgf.fermi_level(z, T, U, frac * top)
        rmu, rne, reb = O.fermi_level(z, T, U, frac * top)
        assert mu == rmu
        assert abs(ne - rne) <= 1e-12 * top and abs(eb - reb) <= 1e-12 * max(1.0, abs(reb))


def test_fermi_level_errors(sgf):
    z = W.shift_grid(-6, 6, 16, 0.05)
    T, U = synthetic(16, 9)
    with pytest.raises(sgf.SgfError) as e:
        sgf.fermi_level(z, T, U, 1e9)
    assert e.value.code == sgf.SGF_EUNSUPPORTED
    with pytest.raises(sgf.SgfError) as e:
        sgf.fermi_level(z[::-1], T, U, 0.1)
    assert e.value.code == sgf.SGF_EINVAL
