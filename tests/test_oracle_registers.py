"""Pin of the oracle's register-allocation rule (oracle/enumerate.py,
regs_per_block) against something outside both implementations: the
compiler's own occupancy report for every compiled instance.

On gfx950 a lane's unified register allocation is its architectural VGPRs
rounded up to 4, plus its accumulation registers (AGPRs), rounded up to the
allocation granule of 8; a SIMD holds 512 such registers per lane and at
most 8 wavefronts.  The compiler reports, per kernel, the wavefronts per
SIMD it can keep resident ("Occupancy [waves/SIMD]"), limited by registers
and by LDS (160 KiB per compute unit, workgroups of the kernel's launch
bound spread over 4 SIMDs).  If the rule is right, the occupancy it implies
equals the compiler's for every instance; the test also shows that the
plausible slips (AGPRs left out, the larger of the two files instead of
their sum, a granule of 4 or 16) contradict the compiler on some instance,
so the check can tell them apart.
"""
import pytest

import oracle.enumerate as en
from paper_1801_04348_amd import pk
from tests import machines

LDS_PER_CU = 160 * 1024
REGS_PER_LANE = 512
MAX_WAVES_PER_SIMD = 8


def _cdiv(a, b):
    return -(-a // b)


@pytest.fixture(scope="module")
def instances():
    t = pk.pk_case_table_build(0, machines.gfx950())
    return pk.pk_case_table_describe(t)["instances"]


def _occupancy(e, per_lane):
    waves = _cdiv(e["threads"], 64)
    by_regs = REGS_PER_LANE // per_lane
    lds = e["lds_compiled"]
    by_lds = MAX_WAVES_PER_SIMD if lds == 0 else _cdiv((LDS_PER_CU // lds) * waves, 4)
    return min(MAX_WAVES_PER_SIMD, by_regs, by_lds)


def test_register_rule_implies_the_compilers_occupancy(instances):
    assert len(instances) > 500
    bound_by_regs = 0
    for e in instances:
        per_lane = en.regs_per_block(e["vgpr"], e["agpr"], 64) // 64
        assert en.regs_per_block(e["vgpr"], e["agpr"], e["threads"]) == per_lane * 64 * _cdiv(e["threads"], 64)
        assert _occupancy(e, per_lane) == e["occupancy"], (e["name"], e["vgpr"], e["agpr"], e["occupancy"])
        if REGS_PER_LANE // per_lane < MAX_WAVES_PER_SIMD:
            bound_by_regs += 1
    # the check has teeth: many instances are held back by their registers
    assert bound_by_regs >= 50, bound_by_regs


@pytest.mark.parametrize("slip", ["agprs_left_out", "larger_not_sum", "granule_4", "granule_16"])
def test_plausible_slips_contradict_the_compiler(instances, slip):
    rules = {
        "agprs_left_out": lambda v, a: _cdiv(_cdiv(v, 4) * 4, 8) * 8,
        "larger_not_sum": lambda v, a: _cdiv(max(_cdiv(v, 4) * 4, a), 8) * 8,
        "granule_4": lambda v, a: _cdiv(_cdiv(v, 4) * 4 + a, 4) * 4,
        "granule_16": lambda v, a: _cdiv(_cdiv(v, 4) * 4 + a, 16) * 16,
    }
    wrong = [e["name"] for e in instances if _occupancy(e, rules[slip](e["vgpr"], e["agpr"])) != e["occupancy"]]
    assert wrong, slip
