"""Host logic of the wavepacket propagation (no GPU): the library's rule for
the number of Chebyshev terms, checked against Bessel values from scipy,
and its argument errors."""
import ctypes

import numpy as np
import pytest
from scipy.special import jv


@pytest.fixture(scope="module")
def sgf():
    import paper_1603_09616_amd as sgf
    sgf.lib()
    return sgf


@pytest.mark.parametrize("a_tau", [0.05, 1.0, 4.56, 8.3, 25.0, -8.3])
@pytest.mark.parametrize("tol", [1e-10, 1e-13])
def test_terms_rule(sgf, a_tau, tol):
    K = sgf.wp_terms(a_tau, tol)
    x = abs(a_tau)
    assert K >= 3 and K > x
    # the cut: both J_K and J_{K+1} below tol; one term earlier is not
    assert abs(jv(K, x)) <= tol * (1 + 1e-9) and abs(jv(K + 1, x)) <= tol * (1 + 1e-9)
    if K - 1 > x and K > 3:
        assert not (abs(jv(K - 1, x)) <= tol and abs(jv(K, x)) <= tol)


def test_terms_rule_matches_the_oracle(sgf, oracle_lib):
    from oracle import wp
    for a_tau in np.linspace(0.5, 30.0, 25):
        assert abs(sgf.wp_terms(a_tau, 1e-13) - max(3, wp.chebyshev_terms(a_tau, 1e-13))) <= 1


def test_argument_errors(sgf):
    k = ctypes.c_int32()
    L = sgf.lib()
    assert L.sgf_wp_terms(1.0, 0.0, ctypes.byref(k)) == sgf.SGF_EINVAL
    assert L.sgf_wp_terms(float("nan"), 1e-13, ctypes.byref(k)) == sgf.SGF_EINVAL
    ws = ctypes.c_size_t()
    assert L.sgf_wp_workspace(100, 3, ctypes.byref(ws)) == sgf.SGF_EINVAL
    assert L.sgf_wp_workspace(100, 8, ctypes.byref(ws)) == sgf.SGF_OK
    assert ws.value >= 2 * 400 * 8 * 16
