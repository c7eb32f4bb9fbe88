"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgf.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libsgf():
    import paper_1603_09616_amd as sgf
    if not os.path.exists(sgf.LIB_PATH):
        pytest.fail("libsgf.so is not built (run __graft_entry__.build())")
    return sgf.lib()


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("sgf_build_hamiltonian", "sgf_shifted_solve", "sgf_last_error"):
        assert s in syms


def test_every_declared_symbol_is_exported(libsgf):
    missing = [s for s in declared_symbols() if not hasattr(libsgf, s)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_1603_09616_amd as sgf
    assert sorted(sgf.EXPORTED) == declared_symbols()


def test_version_and_error_text(libsgf):
    assert libsgf.sgf_version() >= 10000
    # an argument error is reported without touching the GPU
    ws = ctypes.c_size_t()
    rc = libsgf.sgf_build_workspace(ctypes.c_int64(0), ctypes.byref(ws))
    assert rc == -1
    assert b"n_atoms" in libsgf.sgf_last_error()


def test_struct_layouts_match_header():
    """ctypes mirrors of the C structs have the sizes the header implies."""
    import paper_1603_09616_amd as sgf
    assert ctypes.sizeof(sgf.TBParamsC) == 12 * 8
    assert ctypes.sizeof(sgf.SystemC) == 10 * 8
    assert ctypes.sizeof(sgf.PlanC) == 12 * 8
    assert ctypes.sizeof(sgf.PlanTotalsC) == 3 * 8 + 4 * 4
    assert ctypes.sizeof(sgf.SolveOptsC) == 96
    assert ctypes.sizeof(sgf.BsrC) == 9 * 8


def test_product_path_has_no_oracle_dependency():
    """The library package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1603_09616_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("the oracle", ""), f


def test_system_from_bsr_host_checks(libsgf):
    """sgf_system_from_bsr fills a host descriptor from the caller's
    (device) arrays without touching them, and refuses inconsistent sizes."""
    import paper_1603_09616_amd as sgf
    fake = [0x1000 * (i + 1) for i in range(6)]   # never dereferenced by this call
    m = sgf.BsrC(10, 28, fake[0], fake[1], fake[2], None, fake[3], None)
    out = ctypes.c_void_p()
    assert libsgf.sgf_system_from_bsr(ctypes.byref(m), ctypes.c_void_p(fake[4]), ctypes.byref(out)) == 0
    c = sgf.SystemC.from_address(out.value)
    assert (c.n_atoms, c.nnzb, c.row_ptr, c.col, c.h, c.s, c.h32, c.s32, c.xyz) == \
        (10, 28, fake[0], fake[1], fake[2], None, fake[3], None, fake[4])
    assert c.s_orbital_diagonal == 0
    libsgf.sgf_system_destroy(out)
    # the per-atom overlap flag is kept with an overlap and dropped without one
    for s_ptr, flag in ((fake[5], 1), (None, 0)):
        m = sgf.BsrC(10, 28, fake[0], fake[1], fake[2], s_ptr, None, None, 1)
        assert libsgf.sgf_system_from_bsr(ctypes.byref(m), None, ctypes.byref(out)) == 0
        assert sgf.SystemC.from_address(out.value).s_orbital_diagonal == flag
        libsgf.sgf_system_destroy(out)
    libsgf.sgf_system_destroy(None)
    for bad in (sgf.BsrC(0, 1, fake[0], fake[1], fake[2], None, None, None),    # no rows
                sgf.BsrC(10, 28, fake[0], fake[1], fake[2], fake[5], None, None, 2),  # flag neither 0 nor 1
                sgf.BsrC(10, 9, fake[0], fake[1], fake[2], None, None, None),   # fewer blocks than diagonal blocks
                sgf.BsrC(10, 28, fake[0], None, fake[2], None, None, None),     # no column indices
                sgf.BsrC(10, 28, fake[0], fake[1], fake[2], None, None, fake[5])):  # FP32 S without S
        assert libsgf.sgf_system_from_bsr(ctypes.byref(bad), None, ctypes.byref(out)) == -1
