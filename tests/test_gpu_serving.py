"""Serving: every job's values are bit-exact against the oracle and identical
to the same job run alone through a plan (tiles of tile_rows rows, or fewer
under a cell bound); a budget that fits one job at a
time queues jobs instead of failing; a job that can never fit is refused."""
import numpy as np
import pytest

import oracle
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs, serve

pytestmark = pytest.mark.gpu


def small_jobs(n=9, seed=21):
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for j in range(n):
        k = int(rng.integers(2, 260))
        b = inputs.random_family(k, 0, int(rng.integers(20, 1300)), seed + j)
        jobs.append(inputs.ServeJob(t, b))
        t += float(rng.exponential(0.002))
    return jobs


def collect(jobs, **opt):
    got = {}

    def on_tile(jid, t):
        got[(jid, int(t.row_begin), int(t.row_end))] = B.tile_array(t).copy()

    r = serve.run_jobs(jobs, on_tile=on_tile, **opt)
    return got, r


@pytest.mark.parametrize("R,step_values,step_cells,realtime", [
    (64, 0, 0, True), (16, 5000, 0, True), (32, 0, 3_000_000, True),
    (64, 0, 0, False), (16, 5000, 0, False), (32, 0, 3_000_000, False)])
def test_serving_matches_oracle_and_alone(R, step_values, step_cells, realtime):
    jobs = small_jobs()
    got, r = collect(jobs, tile_rows=R, step_values=step_values, step_cells=step_cells, realtime=realtime)
    ids = r["job_ids"]
    if not realtime and step_cells == 0:
        # every job queued before the first step and steps bounded by values
        # only: steps must hold tiles of several jobs at once, so the
        # comparison below is of results computed in a mix (a 3e6-cell bound
        # lets one tile of these jobs fill a step)
        assert r["max_jobs_per_step"] >= 2
        mixed = [s for s in r["step_jobs"] if len(s) >= 2]
        assert len(set().union(*mixed)) >= 2
    for jid, i in ids.items():
        b = jobs[i].batch
        k = b.nseq
        with B.Plan.from_batch(b, tile_rows=R) as p:
            alone = p.collect()
        keys = sorted(key for key in got if key[0] == jid)
        # the job's tiles cover its rows in order; R rows each without a
        # cell bound, at most R rows and the bound's cells (or one row) with it
        assert keys[0][1] == 0 and keys[-1][2] == k and all(a[2] == c[1] for a, c in zip(keys, keys[1:]))
        L = b.lengths().astype(np.int64)
        cells = L * np.concatenate([np.cumsum(L[::-1])[::-1][1:], [0]])
        for _, r0, r1 in keys:
            assert r1 - r0 <= R
            if step_cells:
                assert r1 - r0 == 1 or int(cells[r0:r1].sum()) <= step_cells, (jid, r0, r1)
            else:
                assert r0 % R == 0
        mix = np.concatenate([got[key] for key in keys])
        whole = np.concatenate([alone[key] for key in sorted(alone)])
        assert np.array_equal(mix, whole), jid
        assert np.array_equal(mix, oracle.tile_expected(b.codes, b.seq_off, 0, k, 0, k)), jid
    if step_cells:  # the bound cut some tile below R rows
        assert any(key[2] - key[1] < R and key[2] != jobs[ids[key[0]]].batch.nseq for key in got)


def test_small_budget_queues():
    jobs = small_jobs(5, seed=3)
    # room for the step buffers and about one job
    got, r = collect(jobs, tile_rows=64, step_values=20000, hbm_budget=2 * 20000 * 4 + (64 << 20) + 1_200_000)
    assert r["jobs"] == 5
    for jid, i in r["job_ids"].items():
        b = jobs[i].batch
        k = b.nseq
        for r0 in range(0, k, 64):
            exp = oracle.tile_expected(b.codes, b.seq_off, 0, k, r0, min(k, r0 + 64))
            assert np.array_equal(got[(jid, r0, min(k, r0 + 64))], exp)


def test_job_too_large_is_refused():
    srv = serve.Server(step_values=4096, hbm_budget=2 * 4096 * 4 + (64 << 20) + 1000)
    b = inputs.random_family(3000, 500, 900, 1)
    with pytest.raises(B.FamsaError) as e:
        srv.submit(b.codes, b.seq_off)
    assert e.value.code == B.ENOMEM
    srv.close()


def test_alone_service_times():
    # each job alone on an idle server, one after the other: the server is
    # idle again after each, so every job gets a positive, finite time
    jobs = small_jobs(4, seed=8)
    t = serve.alone_ms(jobs, tile_rows=64)
    assert t.shape == (4,) and (t > 0).all() and np.isfinite(t).all()


def test_admission_passes_a_job_that_does_not_fit_yet():
    # A holds most of the budget; B fits alone but not beside A; C fits
    # beside A.  C is admitted on the first step although B is older, and B
    # once A has finished; every result still equals the oracle.
    A = inputs.random_family(200, 250, 350, 31)
    Bj = inputs.random_family(150, 250, 350, 32)
    C = inputs.random_family(20, 40, 60, 33)
    sv = 1 << 16

    def footprint(b):
        srv = serve.Server(step_values=sv, tile_rows=64)
        fixed = srv.memory()[0]
        srv.submit(b.codes, b.seq_off)
        srv.step(None)
        used = srv.memory()[0]
        while srv.step(None):
            pass
        srv.close()
        return fixed, used - fixed

    fixed, fA = footprint(A)
    _, fB = footprint(Bj)
    _, fC = footprint(C)
    assert fC + 100 < fB <= fA + fC
    srv = serve.Server(step_values=sv, tile_rows=64, hbm_budget=fixed + fA + fC + 100)
    got = {}
    ids = [srv.submit(b.codes, b.seq_off) for b in (A, Bj, C)]

    def keep(t):
        got[(int(t.family), int(t.row_begin), int(t.row_end))] = B.tile_array(t).copy()
        return 0

    active = srv.step(keep)
    assert [srv.job_state(j) for j in ids] == [1, 0, 1]
    while active:
        active = srv.step(keep)
    srv.close()
    for jid, b in zip(ids, (A, Bj, C)):
        k = b.nseq
        for r0 in range(0, k, 64):
            r1 = min(k, r0 + 64)
            assert np.array_equal(got[(jid, r0, r1)], oracle.tile_expected(b.codes, b.seq_off, 0, k, r0, r1))
