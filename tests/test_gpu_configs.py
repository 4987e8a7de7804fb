"""Full-size workloads, in the launch configuration bench.py times: seeded
samples of every tile checked against the oracle one pair at a time, plus
0 <= LCS <= min(|A|, |B|) over whole tiles."""
import numpy as np
import pytest

from helpers import Sampler, check_all_tiles
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def test_c2_sampled():
    b = inputs.c2()
    s = Sampler(b, per_tile=400, seed=1)
    with B.Plan.from_batch(b) as p:
        p.run(s)
    assert s.count == b.pairs()
    assert s.check() >= 3000


def test_c3_sampled_batched_and_plain_agree():
    b = inputs.c3()
    s = Sampler(b, per_tile=100, seed=2)
    with B.Plan.from_batch(b) as p:
        p.run(s)
    assert s.count == b.pairs()
    s.check()


@pytest.mark.timeout(600)
def test_c4_sampled_bench_configuration():
    b = inputs.c4()
    s = Sampler(b, per_tile=60, seed=3, bound_check_every=25)
    with B.Plan.from_batch(b, flags=B.NO_GRAPH) as p:
        p.run(s)
    assert s.ntiles == 98
    assert s.count == b.pairs()
    assert s.check() >= 5000
