"""The build's guard for the staged kernels' counted waits: the compiler's
resource-usage remarks are parsed, and a staged kernel with scratch memory
(whose spills would add vector-memory operations the waits do not count)
fails the build."""
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
