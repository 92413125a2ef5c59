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
