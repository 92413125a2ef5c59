"""The build's guards for the staged kernels' counted waits: the compiler's
resource-usage remarks are parsed, and a staged kernel with scratch memory
(whose spills would add vector-memory operations the waits do not count)
fails the build, as does one whose device assembly places fewer operations
after its global->LDS copies than a wait lets run on."""
import pytest

from paper_1202_4748_amd import build

REMARKS = """\
x.hip:1:1: remark: Function Name: _ZN5lbfss14k_fused_stagedIfLi64ELi4ELb1ELb0EEEvv [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     VGPRs: 131 [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark: Function Name: _ZN5lbfss9k_collideIfLb0EEEvv [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]
"""


def test_parse_and_accept():
    u = build.resource_usage(REMARKS)
    assert u["_ZN5lbfss14k_fused_stagedIfLi64ELi4ELb1ELb0EEEvv"]["VGPRs"] == "131"
    assert u["_ZN5lbfss9k_collideIfLb0EEEvv"]["ScratchSize [bytes/lane]"] == "16"
    assert build.check_counted_waits(u) == 1   # scratch elsewhere is allowed


def test_scratch_in_a_staged_kernel_fails():
    bad = REMARKS.replace("ScratchSize [bytes/lane]: 0", "ScratchSize [bytes/lane]: 8")
    with pytest.raises(RuntimeError):
        build.check_counted_waits(build.resource_usage(bad))
    with pytest.raises(RuntimeError):
        build.check_counted_waits({})


def _occ_remarks(fp32_64x8_waves):
    lines = []
    for prefix, need in build.REQUIRED_OCCUPANCY.items():
        occ = fp32_64x8_waves if prefix.endswith("IfLi64ELi8ELb1ELb0E") else need
        lines.append(f"x.hip:1:1: remark: Function Name: {prefix}EEvv [-Rpass-analysis=kernel-resource-usage]")
        lines.append(f"x.hip:1:1: remark:     Occupancy [waves/SIMD]: {occ} [-Rpass-analysis=kernel-resource-usage]")
    return "\n".join(lines) + "\n"


def test_occupancy_guard():
    """The 64 x 8 FP32 step kernel must keep four waves per SIMD (two
    512-thread workgroups per CU); one VGPR too many (three waves) fails the
    build, as does a missing remark."""
    assert build.check_occupancy(build.resource_usage(_occ_remarks(4))) == len(build.REQUIRED_OCCUPANCY)
    with pytest.raises(RuntimeError, match="below their occupancy"):
        build.check_occupancy(build.resource_usage(_occ_remarks(3)))
    with pytest.raises(RuntimeError, match="no resource-usage remark"):
        build.check_occupancy({})


def _staged_asm(stores_after_copy=19, stores_before_copy=0):
    """A staged kernel's loop as the compiler lays it out: the loop header
    holds the counted wait (taken when the last iteration stored), the body
    issues the next plane's copies, then the collision's stores."""
    body = ["\tglobal_store_dword v1, v2, s[0:1] nt"] * stores_before_copy
    body += ["\tglobal_load_lds_dwordx4 v3, s[4:5] offset:16"]
    body += ["\tglobal_store_dword v1, v2, s[0:1] nt"] * stores_after_copy
    return "\n".join([
        "_ZN5lbfss14k_fused_stagedIfLi64ELi8ELb1ELb0EEEvv:",
        "\tglobal_load_lds_dwordx4 v3, s[4:5]",
        ".LBB0_1:                                ; =>This Inner Loop Header: Depth=1",
        "\ts_cbranch_execz .LBB0_3",
        "\ts_waitcnt vmcnt(0)",
        ".LBB0_3:",
        "\ts_cbranch_execz .LBB0_4",
        "\ts_waitcnt vmcnt(19)",
        ".LBB0_4:",
        "\ts_barrier",
        *body,
        "\ts_cbranch_scc1 .LBB0_1",
        "\ts_endpgm",
        ".Lfunc_end0:",
    ]) + "\n"


def test_counted_wait_order_guard():
    """The build reads the device assembly: every vmcnt(19) wait of a staged
    kernel must follow at least 19 vector-memory operations issued after the
    last global->LDS copy (here along the loop's back edge).  Stores moved
    ahead of the copies, or fewer of them (merged), fail the build."""
    assert build.check_counted_wait_order(_staged_asm()) == 1
    with pytest.raises(RuntimeError, match="0 younger"):
        build.check_counted_wait_order(_staged_asm(stores_after_copy=0, stores_before_copy=19))
    with pytest.raises(RuntimeError, match="18 younger"):
        build.check_counted_wait_order(_staged_asm(stores_after_copy=18))
    straight = "\n".join(["_ZN5lbfss12k_meq_stagedILi64ELi8ELb0EEEvv:", "\tglobal_load_lds_dword v3, s[4:5]"]
                         + ["\tglobal_store_dword v1, v2, s[0:1] nt"] * 5 + ["\ts_waitcnt vmcnt(19)", ".Lfunc_end1:"])
    with pytest.raises(RuntimeError, match="5 younger"):
        build.check_counted_wait_order(straight)
    with pytest.raises(RuntimeError, match="no staged kernels"):
        build.check_counted_wait_order("_ZN5lbfss9k_collideIfLb0EEEvv:\n\ts_endpgm\n.Lfunc_end2:\n")


def test_counted_wait_guard_takes_any_path():
    """A path that skips the collision (no stores) reaches the loop header's
    counted wait too, but at run time it takes the full wait instead: the
    guard asks for one path from a copy with enough operations, laid out as
    the compiler does with the copies of the next plane out of line."""
    asm = "\n".join([
        "_ZN5lbfss12k_meq_stagedILi64ELi4ELb1EEEvv:",
        "\tglobal_load_lds_dwordx4 v3, s[4:5]",
        ".LBB1_1:",
        "\ts_cbranch_vccz .LBB1_4",
        "\ts_waitcnt vmcnt(19)",
        ".LBB1_4:",
        "\ts_cbranch_scc1 .LBB1_9",      # the copies, out of line
        ".LBB1_5:",                      # the collision and its stores
        *["\tglobal_store_dword v1, v2, s[0:1] nt"] * 19,
        ".LBB1_6:",
        "\ts_cbranch_scc0 .LBB1_1",
        "\ts_endpgm",
        ".LBB1_9:",
        "\tglobal_load_lds_dwordx4 v3, s[4:5] offset:16",
        "\ts_cbranch_scc0 .LBB1_5",      # on to the collision
        "\ts_branch .LBB1_6",            # or past it (no stores)
        ".Lfunc_end1:",
    ]) + "\n"
    assert build.check_counted_wait_order(asm) == 1
    with pytest.raises(RuntimeError, match="18 younger"):
        build.check_counted_wait_order(asm.replace("\tglobal_store_dword v1, v2, s[0:1] nt\n", "", 1))
