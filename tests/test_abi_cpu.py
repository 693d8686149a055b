"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/hfmm.h declares (no compute call is made without a GPU), and
the binding refuses to run without the library rather than falling back."""
import ctypes
import os

import pytest

from paper_1608_02461_amd import hfmm


def test_header_declares_the_boundary():
    names = hfmm.header_functions()
    for required in ["hfmm_build_tree", "hfmm_fmm_apply", "hfmm_fd_helmholtz_matvec", "hfmm_fgmres_solve",
                     "hfmm_solver_create", "hfmm_fgmres_solve_batched", "hfmm_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(hfmm.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(hfmm.LIB_PATH)
    missing = [n for n in hfmm.header_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(hfmm._SIGS) == set(hfmm.header_functions())


@pytest.mark.skipif(not os.path.exists(hfmm.LIB_PATH), reason="library not built")
def test_version_and_error_string():
    assert hfmm.hfmm_version() >= 100
    assert isinstance(hfmm.hfmm_last_error(), str)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(hfmm, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(hfmm, "_lib", None)
    with pytest.raises(RuntimeError):
        hfmm.lib()


def test_product_path_does_not_import_oracle():
    pkg = os.path.dirname(hfmm.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(root, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


@pytest.mark.skipif(not os.path.exists(hfmm.LIB_PATH), reason="library not built")
def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache (host only) reads lines with and without the M2L
    class-group column (files written before that choice existed load with
    class groups allowed) and writes all four columns; an invalid lane count
    or a short line is an argument error."""
    hfmm.hfmm_tune_cache_clear()
    f = tmp_path / "t.txt"
    f.write_text("# hfmm tuning cache\nkeyA:c1 2 0\nkeyB:c1 4 1 0\n")
    assert hfmm.hfmm_tune_cache_load(str(f)) == 2
    assert hfmm.hfmm_tune_cache_size() == 2
    out = tmp_path / "o.txt"
    hfmm.hfmm_tune_cache_save(str(out))
    rows = sorted(ln.split() for ln in out.read_text().splitlines() if not ln.startswith("#"))
    assert rows == [["keyA:c1", "2", "0", "1"], ["keyB:c1", "4", "1", "0"]]
    for bad in ("keyC:c1 3 0 1\n", "keyD:c1\n"):
        g = tmp_path / "bad.txt"
        g.write_text(bad)
        with pytest.raises(hfmm.HFMMError):
            hfmm.hfmm_tune_cache_load(str(g))
    hfmm.hfmm_tune_cache_clear()
    assert hfmm.hfmm_tune_cache_size() == 0


@pytest.mark.skipif(not os.path.exists(hfmm.LIB_PATH), reason="library not built")
def test_3d_entry_points_reject_bad_arguments_before_any_device_call():
    """The oct-tree entry points validate their host arguments first, so
    these calls return HFMM_ERR_ARG (with a message) without touching a GPU."""
    L = hfmm.lib()
    out = ctypes.c_void_p()
    vp = ctypes.c_void_p

    def st(code):
        assert code == hfmm.HFMM_ERR_ARG
        return hfmm.hfmm_last_error()

    assert "out is NULL" in st(L.hfmm3_build_tree(vp(1), 10, 0.0, 0.0, 0.0, 1.0, 8, None, None))
    assert "n must be >= 1" in st(L.hfmm3_build_tree(vp(1), 0, 0.0, 0.0, 0.0, 1.0, 8, None, ctypes.byref(out)))
    assert "side" in st(L.hfmm3_build_tree(vp(1), 10, 0.0, 0.0, 0.0, -1.0, 8, None, ctypes.byref(out)))
    assert "leaf_size" in st(L.hfmm3_build_tree(vp(1), 10, 0.0, 0.0, 0.0, 1.0, 0, None, ctypes.byref(out)))
    assert "d_xyz is NULL" in st(L.hfmm3_build_tree(None, 10, 0.0, 0.0, 0.0, 1.0, 8, None, ctypes.byref(out)))
    assert "corner" in st(L.hfmm3_build_tree(vp(1), 10, float("nan"), 0.0, 0.0, 1.0, 8, None, ctypes.byref(out)))
    assert out.value is None
    assert "NULL tree" in st(L.hfmm3_fmm_apply(None, 10.0, 6, hfmm.FP64, vp(1), vp(1), None))
    assert "NULL tree" in st(L.hfmm3_fmm_apply_timed(None, 10.0, 6, hfmm.FP32, vp(1), vp(1), None, None))
    assert "NULL tree" in st(L.hfmm3_tree_info(None, None, None, None, None))
    assert "NULL tree" in st(L.hfmm3_fmm_orders(None, 10.0, 6, None))
    assert L.hfmm3_tree_destroy(None) == hfmm.HFMM_OK
