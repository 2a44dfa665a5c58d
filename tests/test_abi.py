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


def test_build_rejects_scratch_in_queue_kernel():
    """The work-queue search kernel is held to the same no-scratch rule."""
    from paper_1802_00330_amd.build import check_no_scratch
    ok = ("k.hip:1:1: remark: Function Name: _ZN3ibb12queue_kernelILi16EEEvNS_9SolveArgsE\n"
          "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 0\n")
    check_no_scratch(ok)
    with pytest.raises(RuntimeError):
        check_no_scratch(ok.replace("ScratchSize [bytes/lane]: 0", "ScratchSize [bytes/lane]: 8"))


_ASM = """\
_ZN3ibb12solve_kernelILi8ELb0EEEvNS_9SolveArgsE:
\t;;#ASMSTART
\ts_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2
\t;;#ASMEND
\t;;#ASMSTART
\tv_add_f64 v[0:1], v[2:3], v[4:5]
\t;;#ASMEND
\tv_cvt_f64_f32_e32 v[6:7], v8
\tv_rcp_f64_e32 v[6:7], v[6:7]
\tv_max_f64 v[0:1], v[0:1], v[2:3]
\ts_endpgm
_ZN3ibb11sort_kernelEPKd:
\tv_add_f64 v[0:1], v[2:3], v[4:5]
\ts_endpgm
"""


def test_isa_check_accepts_directed_kernels():
    """One MODE write at entry, FP64 arithmetic only in the one-instruction
    statements; kernels without a rounding-mode change are not restricted."""
    from paper_1802_00330_amd.build import check_isa
    check_isa(_ASM)


@pytest.mark.parametrize("planted", [
    "\tv_add_f64 v[0:1], v[2:3], v[4:5]\n",          # compiler FP64 add in round-down code
    "\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[6:7]\n",  # compiler FP64 fma
    "\ts_round_mode 0x0\n",                         # a second MODE write
    "\ts_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 4), 0\n",
    "\tv_pk_mul_f32 v[0:1], v[2:3], v[4:5]\n",       # packed FP32
])
def test_isa_check_rejects(planted):
    from paper_1802_00330_amd.build import check_isa
    at = _ASM.index("\tv_cvt_f64_f32_e32")
    with pytest.raises(RuntimeError):
        check_isa(_ASM[:at] + planted + _ASM[at:])


def test_built_library_passed_the_isa_check():
    """The device assembly kept by the last build satisfies check_isa."""
    from paper_1802_00330_amd import build
    s = os.path.join(build.HERE, "_build", "kernels-hip-amdgcn-amd-amdhsa-gfx950.s")
    if not os.path.exists(s):
        pytest.skip("library not built in this tree")
    build.check_isa(open(s).read())
