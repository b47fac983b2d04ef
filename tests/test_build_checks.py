"""The build's guard against register spills in the hot kernels: it reads
the compiler's kernel-resource-usage remarks and rejects scratch memory in
the kernels listed in NO_SCRATCH."""
from paper_2402_14821_amd import build as B

REMARKS = """\
x.hip:1:1: remark: Function Name: _ZN3bpi7k_sweepILi2EEEvPKNS_10LaunchDescE [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     VGPRs: 64 [-Rpass-analysis=kernel-resource-usage]
x.hip:1:1: remark:     ScratchSize [bytes/lane]: 608 [-Rpass-analysis=kernel-resource-usage]
x.hip:2:1: remark: Function Name: _ZN3bpi12k_node_deltaEPKNS_8NodeTaskElPKiPxPyP9bp_bounds [-Rpass-analysis=kernel-resource-usage]
x.hip:2:1: remark:     ScratchSize [bytes/lane]: 64 [-Rpass-analysis=kernel-resource-usage]
x.hip:4:1: remark: Function Name: _ZN3bpi7k_sweepILi4EEEvPKNS_10LaunchDescE [-Rpass-analysis=kernel-resource-usage]
x.hip:4:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]
x.hip:3:1: remark: Function Name: _ZN3bpi10k_finalizeEPKNS_10LaunchDescE [-Rpass-analysis=kernel-resource-usage]
x.hip:3:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
"""


def test_scratch_guard_flags_only_the_listed_kernels():
    bad = B._scratch_kernels(REMARKS)
    assert bad == [("_ZN3bpi7k_sweepILi2EEEvPKNS_10LaunchDescE", 608), ("_ZN3bpi7k_sweepILi4EEEvPKNS_10LaunchDescE", 16)]
    assert B._scratch_kernels("") == []
