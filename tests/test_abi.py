"""The C-ABI library builds for gfx950 and exports every entry point that
include/ibb.h declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ibb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("ibb_solve", "ibb_solve_async", "ibb_workspace_size", "ibb_ctx_create", "ibb_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1802_00330_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1802_00330_amd import build
        build.build()
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(P.EXPORTS) == set(_declared())


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1802_00330_amd as P
    saved = P._lib
    P._lib = None
    try:
        with pytest.raises(RuntimeError):
            P.load_library(str(tmp_path / "missing.so"))
    finally:
        P._lib = saved


def test_build_rejects_scratch_in_search_kernels():
    """The build refuses search kernels that spill to scratch memory."""
    from paper_1802_00330_amd.build import check_no_scratch
    ok = ("k.hip:1:1: remark: Function Name: _ZN3ibb12solve_kernelILi8ELb0EEEvNS_9SolveArgsE\n"
          "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 0\n"
          "k.hip:1:1: remark: Function Name: _ZN3ibb14selftest_kernelEi\n"
          "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 16\n")
    check_no_scratch(ok)
    bad = ok.replace("ScratchSize [bytes/lane]: 0", "ScratchSize [bytes/lane]: 196")
    with pytest.raises(RuntimeError):
        check_no_scratch(bad)
