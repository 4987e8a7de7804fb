"""Full-size workloads, in the launch configurations bench.py times (c2, c3,
c4, and the c5 serving jobs): seeded samples of every tile checked against
the oracle one pair at a time, plus 0 <= LCS <= min(|A|, |B|) over whole
tiles; on c2 and c3 every value of the batched kernels also equals the
plain kernel's."""
import hashlib

import numpy as np
import pytest

from helpers import Sampler, check_all_tiles
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def run_hashed(b, sampler=None, **opt):
    """Digest of every tile (and the sampler fed the same tiles)."""
    out = {}

    def fn(t):
        a = B.tile_array(t)
        out[(int(t.family), int(t.row_begin), int(t.row_end))] = hashlib.blake2b(a.tobytes(), digest_size=16).digest()
        return sampler(t) if sampler else 0

    with B.Plan.from_batch(b, **opt) as p:
        p.run(fn)
    return out


@pytest.mark.parametrize("name,seed,per_tile", [("c2", 1, 400), ("c3", 2, 100)])
def test_sampled_and_batched_equals_plain(name, seed, per_tile):
    # the batched kernels (32-bit words, masks in LDS, 64 rows per wave) and
    # the plain one (64-bit words, one pair per lane) agree on every value
    # of the workload; seeded samples of every tile also match the oracle
    b = getattr(inputs, name)()
    s = Sampler(b, per_tile=per_tile, seed=seed)
    batched = run_hashed(b, sampler=s)
    assert s.count == b.pairs()
    assert s.check() >= 3000
    plain = run_hashed(b, flags=B.PLAIN)
    assert plain.keys() == batched.keys()
    assert all(plain[key] == batched[key] for key in batched)


@pytest.mark.timeout(600)
def test_c4_sampled_bench_configuration():
    # the launch configuration bench.py times: 2^28-value steps on one
    # compute stream, direct launches, autotuned launch shape
    b = inputs.c4()
    s = Sampler(b, per_tile=60, seed=3, bound_check_every=25)
    with B.Plan.from_batch(b, flags=B.ONE_STREAM | B.NO_GRAPH, step_values=1 << 28) as p:
        p.autotune(None)
        p.run(s)
    assert s.ntiles == 98
    assert s.count == b.pairs()
    assert s.check() >= 5000


@pytest.mark.timeout(600)
def test_c4_sampled_two_streams_with_graphs():
    # graph replays alternating between two compute streams
    b = inputs.c4()
    s = Sampler(b, per_tile=20, seed=4, bound_check_every=49)
    with B.Plan.from_batch(b, flags=B.TWO_STREAMS) as p:
        p.run(s)
    assert s.ntiles == 98 and s.count == b.pairs()
    s.check()


def test_c5_jobs_sampled_in_the_serving_configuration():
    # every job of the serving workload through the server as bench.py runs
    # it (2^24-value, 2^41-cell steps, 256-row tiles), arrivals replayed at once
    from paper_1603_06958_amd import serve
    jobs = inputs.c5(seed=4, njobs=40, rate_per_s=serve.C5_RATE_PER_S)  # the bench's 40 jobs
    samplers = {}

    def on_tile(jid, t):
        if jid not in samplers:
            samplers[jid] = Sampler(jobs[r_ids[jid]].batch, per_tile=30, seed=jid, bound_check_every=7)
        local = B.Tile.from_buffer_copy(t)  # the job's own batch holds one family
        local.family = 0
        samplers[jid](local)

    r_ids = {}
    srv = serve.Server(step_values=serve.SERVE_STEP_VALUES, step_cells=serve.SERVE_STEP_CELLS,
                       tile_rows=serve.SERVE_TILE_ROWS)
    for i, j in enumerate(jobs):
        r_ids[srv.submit(j.batch.codes, j.batch.seq_off)] = i
    active = 1
    while active:
        active = srv.step(lambda t: on_tile(int(t.family), t))
    srv.close()
    assert len(samplers) == len(jobs)
    total = 0
    for jid, smp in samplers.items():
        assert smp.count == jobs[r_ids[jid]].batch.pairs()
        total += smp.check()
    assert total >= 1000
