"""The algorithmic operation count behind the benchmark's roofline
(measure/opcount.py): splitting the events over parallel shards, each told
the index of its first event, gives the same counts as one run over all of
them (the events are independent and the point stream is keyed by the
event index), and the counts are consistent with the evaluations."""
import os
import shutil
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", "measure"))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def test_sharding_leaves_the_count_unchanged():
    import opcount
    one = opcount.run(512, 2, 6, 6, jobs=1)
    three = opcount.run(512, 2, 6, 6, jobs=3)
    assert one["evaluations"] == three["evaluations"] == 6 * 2 * 2 * 512
    for p in ("fp64", "fp32"):
        for k, v in one[p].items():
            assert abs(v - three[p][k]) <= 0.011, (p, k, v, three[p][k])
    assert abs(one["flop_fp32_equivalent"] - three["flop_fp32_equivalent"]) <= 0.05
    assert one["solutions_per_eval"] == pytest.approx(three["solutions_per_eval"], abs=1e-6)
    # every evaluation maps its point and forms its weight; FP64 work dominates
    assert one["fp64"]["flop"] > one["fp32"]["flop"] > 0
    assert one["flop_fp32_equivalent"] == pytest.approx(2 * one["fp64"]["flop"] + one["fp32"]["flop"], abs=0.02)
