"""The library's Fermi-Dirac shifts (a host call: Sturm bisection and a
characteristic-polynomial recurrence) against the oracle's (numpy eigh of the
same tridiagonal matrix), and its argument checks.  No GPU is touched."""
import numpy as np
import pytest

from oracle import contour as C


@pytest.mark.parametrize("n_poles", [1, 10, 48, 100, 256])
def test_shifts_match_oracle(n_poles):
    import paper_1603_09616_amd as sgf
    z, w = sgf.fermi_shifts(n_poles, 0.1, -0.3, 1e8)
    zo, wo = C.fermi_shifts(n_poles, 0.1, -0.3, 1e8)
    assert z.size == w.size == n_poles + 1
    np.testing.assert_allclose(z, zo, rtol=1e-13)
    np.testing.assert_allclose(w, wo, rtol=1e-12)
    assert np.argmin(z.imag) == 0


def test_argument_errors():
    import paper_1603_09616_amd as sgf
    for args in ((0, 0.1, 0.0), (512, 0.1, 0.0), (10, 0.0, 0.0), (10, 0.1, float("nan"))):
        with pytest.raises(sgf.SgfError) as e:
            sgf.fermi_shifts(*args)
        assert e.value.code == sgf.SGF_EINVAL
