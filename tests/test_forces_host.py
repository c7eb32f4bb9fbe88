"""Argument checks of the energy-density and band-force entry points (no
GPU): each case below is rejected before anything is launched, so the
pointers handed over are never dereferenced."""
import ctypes

import pytest

import workloads as W


@pytest.fixture(scope="module")
def sgf():
    import paper_1603_09616_amd as sgf
    sgf.lib()
    return sgf


FAKE = 1 << 20  # a stand-in device address; none of these calls reach a launch


def test_energy_density_arguments(sgf):
    L = sgf.lib()
    P = ctypes.c_void_p
    f = L.sgf_energy_density
    assert f(10, 0, P(FAKE), P(FAKE), P(FAKE), P(FAKE), None) == sgf.SGF_EINVAL          # no shifts
    assert f(-1, 8, P(FAKE), P(FAKE), P(FAKE), P(FAKE), None) == sgf.SGF_EINVAL          # negative rows
    assert f(10, 513, P(FAKE), P(FAKE), P(FAKE), P(FAKE), None) == sgf.SGF_EUNSUPPORTED  # above 512 shifts
    assert f(10, 8, None, P(FAKE), P(FAKE), P(FAKE), None) == sgf.SGF_EINVAL             # z missing
    assert f(10, 8, P(FAKE), P(FAKE), P(FAKE), None, None) == sgf.SGF_EINVAL             # output missing
    assert f(0, 8, None, None, None, None, None) == sgf.SGF_OK                           # nothing to do
    assert b"energy_density" in L.sgf_last_error()


def test_band_forces_arguments(sgf):
    L = sgf.lib()
    P = ctypes.c_void_p
    tb = sgf._tb_c(W.BUNDLE_TB)
    tbo = sgf._tb_c(W.BUNDLE_TB_OVERLAP)
    ortho = sgf.SystemC(100, 300, FAKE, FAKE, FAKE, None, None, None, FAKE)
    ovl = sgf.SystemC(100, 300, FAKE, FAKE, FAKE, FAKE, None, None, FAKE)

    def call(sys, p, n_cols=8, eps=FAKE, force=FAKE, xyz=FAKE):
        return L.sgf_band_forces(None if sys is None else ctypes.byref(sys), P(xyz), ctypes.byref(p), n_cols,
                                 P(FAKE), P(FAKE), P(FAKE), None, P(FAKE), None if eps is None else P(eps),
                                 None if force is None else P(force), None)

    assert call(None, tb) == sgf.SGF_EINVAL
    assert call(ortho, tb, force=None) == sgf.SGF_EINVAL
    assert call(ortho, tb, n_cols=-1) == sgf.SGF_EINVAL
    assert call(ortho, tbo) == sgf.SGF_EINVAL          # overlap parameters, orthogonal system
    assert call(ovl, tb) == sgf.SGF_EINVAL             # overlap system, orthogonal parameters
    assert call(ovl, tbo, eps=None) == sgf.SGF_EINVAL  # an overlap needs eps
    assert b"energy-density" in L.sgf_last_error()
    bad = sgf._tb_c(W.BUNDLE_TB)
    bad.r0 = 0.0
    assert call(ortho, bad) == sgf.SGF_EINVAL
