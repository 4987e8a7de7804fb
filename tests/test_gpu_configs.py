"""Full-size workloads, in the launch configurations bench.py times (c2, c3,
c4, and the c5 serving jobs): seeded samples of every tile checked against
the oracle one pair at a time, plus 0 <= LCS <= min(|A|, |B|) over every
value of every tile; every value of the batched kernels also equals the
plain kernel's (c2, c3, c4: per-tile digests), and every c5 job's values
are the same in the serving mix as when the job runs alone; on c4 the host
SLINK consumer and the GPU spanning-tree consumer, both fed the GPU's tiles,
give the same merge heights, and every tree edge's LCS is the oracle's."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from helpers import RowStream, Sampler, check_all_tiles, digest
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def run_hashed(b, sampler=None, **opt):
    """Digest of every tile (and the sampler fed the same tiles)."""
    out = {}

    def fn(t):
        a = B.tile_array(t)
        out[(int(t.family), int(t.row_begin), int(t.row_end))] = digest(a)
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


@pytest.fixture(scope="module")
def c4_plain():
    """c4 and the plain kernel's per-tile digests (one pass, ~12 s)."""
    b = inputs.c4()
    return b, run_hashed(b, flags=B.PLAIN)


@pytest.mark.timeout(900)
def test_c4_bench_configuration_every_tile_equals_plain(c4_plain):
    # the launch configuration bench.py times: 2^28-value steps on one
    # compute stream, direct launches, autotuned launch shape; every one of
    # the 98 tiles (5.0e9 values) equals the plain kernel's by digest and is
    # within [0, min length]; 1,000 seeded values per tile (98,000 pairs,
    # 6.7e9 oracle cells) match the oracle
    b, plain = c4_plain
    s = Sampler(b, per_tile=1000, seed=3)
    batched = {}

    def fn(t):
        batched[(int(t.family), int(t.row_begin), int(t.row_end))] = digest(B.tile_array(t))
        return s(t)

    with B.Plan.from_batch(b, flags=B.ONE_STREAM | B.NO_GRAPH, step_values=1 << 28) as p:
        p.autotune(None)
        p.run(fn)
    assert s.ntiles == 98
    assert s.count == b.pairs()
    assert s.check() >= 90000
    assert plain.keys() == batched.keys() and len(plain) == 98
    bad = [key for key in batched if plain[key] != batched[key]]
    assert not bad, f"{len(bad)} tiles differ from the plain kernel, first {bad[0]}"


def _sim_key(n, d):
    return oracle.INF if d == 0 else Fraction(int(n), int(d))


@pytest.mark.timeout(900)
def test_c4_host_slink_heights_equal_gpu_tree():
    # stage II at the headline scale: the host SLINK over all 98 descending
    # host tiles and the GPU spanning-forest consumer over device tiles give
    # the same multiset of 99,999 merge similarities; the GPU tree's edges
    # carry the oracle's LCS of their pairs
    b = inputs.c4()
    k = b.nseq
    s = B.SLink(b.lengths())
    with B.Plan.from_batch(b, flags=B.DESCENDING, step_values=1 << 28) as p:
        p.run_native(B.SLink.consume_fn(), s.handle)
    pi, num, den = s.result()
    s.close()
    m = B.Mst(b.lengths())
    with B.Plan.from_batch(b, flags=B.DEVICE_TILES, step_values=1 << 28) as p:
        p.run_native(B.Mst.consume_fn(), m.handle)
    u, v, L, D = m.result()
    m.close()
    assert len(u) == k - 1
    slink_h = sorted(_sim_key(n, q) for n, q in zip(num, den) if not (n == -1 and q == 0))
    assert len(slink_h) == k - 1
    assert sorted(_sim_key(x, y) for x, y in zip(L, D)) == slink_h
    exp = oracle.lcs_pairs(b.codes, b.seq_off, u.astype(np.int64), v.astype(np.int64))
    assert np.array_equal(exp, np.asarray(L, dtype=np.int64))
    lens = b.lengths().astype(np.int64)
    d = lens[u] + lens[v] - 2 * exp
    assert np.array_equal(d * d, np.asarray(D, dtype=np.int64))


@pytest.mark.timeout(600)
def test_c4_two_streams_with_graphs_equals_plain(c4_plain):
    # graph replays alternating between two compute streams: every tile
    # equals the plain kernel's, and 200 seeded values per tile match the
    # oracle
    b, plain = c4_plain
    s = Sampler(b, per_tile=200, seed=4)
    got = run_hashed(b, sampler=s, flags=B.TWO_STREAMS)
    assert s.ntiles == 98 and s.count == b.pairs()
    s.check()
    assert got == plain


@pytest.mark.timeout(900)
def test_c5_jobs_sampled_in_the_serving_configuration():
    # every job of the serving workload (all 200 jobs of the bench's mix)
    # through the server as bench.py runs it (2^24-value, 2^41-cell steps,
    # tiles of at most 256 rows and 2^41 cells), arrivals replayed at once;
    # every job's values, row by row, equal the job's when it runs alone
    # (stream digests, whatever the tile boundaries), seeded samples match
    # the oracle, every value is within [0, min length], and no tile passes
    # the cell bound unless it is one row
    import os
    from paper_1603_06958_amd import serve
    jobs = inputs.c5(seed=4, njobs=200, rate_per_s=serve.C5_RATE_PER_S,
                     workers=min(16, len(os.sched_getaffinity(0))))
    samplers = {}
    streams = {}
    row_cells = {}  # per job: cells of each row's pairs, L_i * (L_{i+1} + ... + L_{k-1})
    over = []

    def on_tile(jid, t):
        b = jobs[r_ids[jid]].batch
        if jid not in samplers:
            samplers[jid] = Sampler(b, per_tile=4, seed=jid)
            streams[jid] = RowStream(b.nseq)
            L = b.lengths().astype(np.int64)
            after = np.concatenate([np.cumsum(L[::-1])[::-1][1:], [0]])
            row_cells[jid] = L * after
        local = B.Tile.from_buffer_copy(t)  # the job's own batch holds one family
        local.family = 0
        streams[jid].feed(t)
        samplers[jid](local)
        r0, r1 = int(t.row_begin), int(t.row_end)
        if r1 - r0 > 1 and int(row_cells[jid][r0:r1].sum()) > serve.SERVE_STEP_CELLS:
            over.append((jid, r0, r1))

    r_ids = {}
    srv = serve.Server(step_values=serve.SERVE_STEP_VALUES, step_cells=serve.SERVE_STEP_CELLS,
                       tile_rows=serve.SERVE_TILE_ROWS)
    for i, j in enumerate(jobs):
        r_ids[srv.submit(j.batch.codes, j.batch.seq_off)] = i
    active = 1
    per_step = []
    while active:
        seen = set()
        active = srv.step(lambda t: (seen.add(int(t.family)), on_tile(int(t.family), t))[1])
        per_step.append(seen)
    srv.close()
    assert max(len(x) for x in per_step) >= 2  # tiles of several jobs in one step
    assert len(samplers) == len(jobs)
    assert not over, f"tiles over the cell bound: {over[:3]}"
    # the cell bound cut some job's tiles below 256 rows
    assert any(streams[jid].tiles > (jobs[i].batch.nseq + 255) // 256 for jid, i in r_ids.items())
    total = 0
    for jid, smp in samplers.items():
        assert smp.count == jobs[r_ids[jid]].batch.pairs()
        total += smp.check()
    assert total >= 1000
    # each job alone, through a plan with 256-row tiles
    for n, (jid, i) in enumerate(r_ids.items()):
        alone = RowStream(jobs[i].batch.nseq)
        with B.Plan.from_batch(jobs[i].batch, tile_rows=serve.SERVE_TILE_ROWS,
                               step_values=serve.SERVE_STEP_VALUES) as p:
            p.run(lambda t: (alone.feed(t), 0)[1])
        assert streams[jid].digest() == alone.digest(), jid
        if n % 50 == 49:
            print(f"c5: {n + 1} jobs alone equal their values in the mix", flush=True)
