"""CPU checks of the build's machine-code scan for wide-store data hazards: a vector
ALU write of a wide store's data registers fewer than two wait states after it."""
import glob
import os

import pytest

from paper_2201_09729_amd import build

HEAD = "0000000000001000 <_ZN4dlma6kernelEv>:\n"


def _scan(body):
    return build.store_data_hazards(HEAD + "\n".join("\t" + l for l in body))


def test_overwrite_right_after_the_store_is_flagged():
    h = _scan(["buffer_store_dwordx4 v[26:29], v30, s[20:23], s48 offen nt",
               "v_mov_b64_e32 v[28:29], v[16:17]"])
    assert len(h) == 1 and h[0][0] == "_ZN4dlma6kernelEv"


def test_wait_states_are_counted():
    st = "buffer_store_dwordx3 v[4:6], v1, s[12:15], 0 offen"
    assert len(_scan([st, "s_nop 0", "v_mov_b32_e32 v5, s7"])) == 1       # one wait state
    assert len(_scan([st, "s_nop 1", "v_mov_b32_e32 v5, s7"])) == 0       # two
    assert len(_scan([st, "s_add_i32 s0, s1, s2", "s_mov_b32 s3, 0", "v_mov_b32_e32 v4, 0"])) == 0


def test_other_registers_and_narrow_stores_are_not_flagged():
    assert not _scan(["global_store_dwordx4 v[0:1], v[4:7], off", "v_mov_b32_e32 v8, 0"])
    assert len(_scan(["global_store_dwordx4 v[0:1], v[4:7], off", "v_add_u32_e32 v7, 1, v7"])) == 1
    assert not _scan(["buffer_store_dwordx2 v[4:5], v1, s[12:15], 0 offen", "v_mov_b32_e32 v4, 0"])
    assert not _scan(["buffer_store_dwordx4 v[4:7], v1, s[12:15], 0 offen", "v_cmp_eq_u32_e32 vcc, v4, v5"])


def test_built_objects_are_clean():
    objs = glob.glob(os.path.join(build.BUILD, "*_hip.o"))
    if not objs or not os.path.exists(os.path.join(build.LLVM, "llvm-objdump")):
        pytest.skip("library not built here")
    for o in objs:
        assert build.check_object(o) == [], o


def test_branch_targets_are_followed():
    """A write at a branch target counts too (the branch is one wait state)."""
    body = ("0000000000001000 <_ZN4dlma6kernelEv>:\n"
            "\tbuffer_store_dwordx4 v[4:7], v1, s[12:15], 0 offen // 000000001000: E07C1000\n"
            "\ts_branch 2 // 000000001008: BF820002 <_ZN4dlma6kernelEv+0x14>\n"
            "\ts_nop 7 // 00000000100C: BF800007\n"
            "\ts_nop 7 // 000000001010: BF800007\n"
            "\tv_mov_b32_e32 v6, 0 // 000000001014: 7E0C0280\n")
    assert len(build.store_data_hazards(body)) == 1
    # the same write past two wait states on the taken path is clean
    clean = body.replace("s_branch 2 // 000000001008", "s_nop 1 // 000000001008")
    assert build.store_data_hazards(clean) == []
    # one more instruction before the branch: two wait states, clean
    two = body.replace("\ts_branch", "\ts_mov_b32 s0, 0 // 000000001004: BE800080\n\ts_branch")
    two = two.replace("offen // 000000001000", "offen // 000000000FFC")
    assert build.store_data_hazards(two) == []
    # conditional branch: both the fall-through and the target path are scanned
    cond = ("0000000000001000 <_ZN4dlma6kernelEv>:\n"
            "\tbuffer_store_dwordx4 v[4:7], v1, s[12:15], 0 offen // 000000001000: E07C1000\n"
            "\ts_cbranch_execz 1 // 000000001008: BF880001 <_ZN4dlma6kernelEv+0x10>\n"
            "\ts_nop 7 // 00000000100C: BF800007\n"
            "\tv_add_u32_e32 v7, 1, v7 // 000000001010: 680E0E81\n")
    assert len(build.store_data_hazards(cond)) == 1
