"""The DPP hazard check over the generated assembly (check_dpp.py): pinned on
synthetic instruction sequences, then run on the solve kernels' source."""
import shutil

import pytest

from paper_2304_04980_amd import check_dpp as cd

DPP = "v_fmac_f32_dpp v1, v5, v2 row_newbcast:3 row_mask:0xf bank_mask:0xf"


def body(*lines):
    out = []
    for s in lines:
        out.append(("label", s[:-1]) if s.endswith(":") else ("ins", s))
    return out


def test_flags_valu_write_of_dpp_source():
    assert cd.check_func("f", body("v_mov_b32_e32 v5, v6", DPP))
    assert cd.check_func("f", body("v_add_f32_e32 v5, v6, v7", "s_nop 0", DPP))
    assert cd.check_func("f", body("v_pk_mov_b32 v[4:5], v[6:7], v[6:7]", DPP))


def test_two_instructions_apart_or_memory_writes_are_fine():
    assert not cd.check_func("f", body("v_mov_b32_e32 v5, v6", "s_nop 0", "s_nop 0", DPP))
    assert not cd.check_func("f", body("buffer_load_dword v5, v0, s[0:3], 0 offen", DPP))
    assert not cd.check_func("f", body("v_mov_b32_e32 v1, v6", DPP))  # dst only


def test_exec_write_within_five():
    assert cd.check_func("f", body("v_cmpx_gt_u32_e32 vcc, 5, v0", "s_nop 0", "s_nop 0",
                                   "s_nop 0", DPP))
    assert not cd.check_func("f", body("v_cmpx_gt_u32_e32 vcc, 5, v0", *["s_nop 0"] * 5, DPP))


def test_branch_into_window_is_followed():
    b = body("v_mov_b32_e32 v5, v6", "s_cbranch_scc1 .LBB0_2", "s_nop 0", "s_nop 0",
             ".LBB0_2:", DPP)
    assert cd.check_func("f", b)
    b = body("v_mov_b32_e32 v5, v6", "s_nop 0", "s_nop 0", "s_cbranch_scc1 .LBB0_2",
             "s_nop 0", ".LBB0_2:", DPP)
    assert not cd.check_func("f", b)


@pytest.mark.skipif(shutil.which(cd.HIPCC) is None and not __import__("os").path.exists(cd.HIPCC),
                    reason="hipcc not available")
@pytest.mark.parametrize("src", ["ops.hip", "batch.hip", "warm.hip"])
def test_kernels_have_no_dpp_hazards(src):
    """Every source whose kernels are built from the DPP-folded FMAs (the
    single-problem and the batched stencil / block-solve kernels; the network
    kernels, which use none, are scanned too)."""
    assert cd.main([src]) == 0
