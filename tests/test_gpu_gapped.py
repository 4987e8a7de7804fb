"""The gapped representation on the GPU (famsa_gapped_*) against the oracle:
the paper's Fig. 1 example reproduced from the ungapped sequence (counters
and tree as printed), then random batches -- empty and long sequences, runs
at the first and last columns, repeated and empty runs, several rounds of
insertion -- compared value for value (counters, tree, decoded rows,
located positions) with the oracle's explicit gapped strings."""
import numpy as np
import pytest

from oracle import gapped as G
from paper_1603_06958_amd import binding as B
from test_gapped_oracle import fig1

pytestmark = pytest.mark.gpu


def batch_of(seqs):
    codes = np.concatenate([np.asarray(s, np.uint8) for s in seqs]) if seqs else np.zeros(0, np.uint8)
    off = np.concatenate([[0], np.cumsum([len(s) for s in seqs])]).astype(np.uint64)
    return codes, off


def row_of(g):
    return np.array([0xFF if c is None else c for c in g[1:]], np.uint8)


def check(gp, strings):
    w = gp.width()
    assert list(w) == [len(g) - 1 for g in strings]
    rows = gp.decode()
    for i, g in enumerate(strings):
        assert np.array_equal(rows[i, :len(g) - 1], row_of(g)), i
        gaps, dps = gp.state(i)
        assert list(gaps) == G.no_gaps(g)
        assert list(dps[1:]) == G.dps(g)[1:]


def test_fig1_on_gpu():
    alphabet, g, d = fig1()
    seq = G.symbols(g)
    codes, off = batch_of([seq])
    gp = B.Gapped(codes, off)
    ng = [int(x) for x in d["no_gaps"]]
    runs = [(i + 1, n) for i, n in enumerate(ng) if n]
    gp.insert([c for c, _ in runs], [n for _, n in runs])
    gaps, dps = gp.state(0)
    assert list(gaps) == ng
    assert list(dps[8:16]) == [int(x) for x in d["dps8_15"]]
    assert list(dps[4:8]) == [int(x) for x in d["dps4_7"]]
    assert list(dps[2:4]) == [int(x) for x in d["dps2_3"]]
    assert dps[1] == int(d["dps1"][0])
    row = gp.decode()[0]
    assert "".join("-" if c == 0xFF else alphabet[c] for c in row) == d["gapped"][0]
    gp.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_batches_match_oracle(seed):
    rng = np.random.default_rng(seed)
    lens = [0, 1, 2, 3, 15, 16, 17, 255, 256, 1000] + [int(x) for x in rng.integers(0, 400, 40)]
    seqs = [rng.integers(0, 20, n).astype(np.uint8) for n in lens]
    codes, off = batch_of(seqs)
    gp = B.Gapped(codes, off)
    strings = [G.from_symbols(s.tolist()) for s in seqs]
    check(gp, strings)
    for rnd in range(4):
        # a profile-like round: one run list for a range of sequences
        first = int(rng.integers(0, len(seqs)))
        count = int(rng.integers(1, len(seqs) - first + 1))
        width = min(len(strings[i]) for i in range(first, first + count))
        cols = sorted([1, width] + [int(x) for x in rng.integers(1, width + 1, int(rng.integers(0, 12)))])
        lens_ = [int(x) for x in rng.integers(0, 6, len(cols))]
        gp.insert(cols, lens_, first, count)
        for i in range(first, first + count):
            strings[i] = G.insert_runs(strings[i], list(zip(cols, lens_)))
        check(gp, strings)
    qs, qc, want = [], [], []
    for i, g in enumerate(strings):
        for col in {0, len(g) - 1, int(rng.integers(0, len(g)))}:
            qs.append(i)
            qc.append(col)
            want.append(G.locate(g, col))
    assert list(gp.locate(qs, qc)) == want
    gp.close()


def test_insert_rejects_bad_runs():
    codes, off = batch_of([np.arange(5, dtype=np.uint8)])
    gp = B.Gapped(codes, off)
    for cols in ([0], [7], [3, 2]):  # before the guard, past width + 1, unsorted
        with pytest.raises(B.FamsaError):
            gp.insert(cols, [1] * len(cols))
    gp.insert([6], [2])  # width + 1 appends
    assert list(gp.width()) == [7]
    with pytest.raises(B.FamsaError):
        gp.locate([0], [8])
    gp.close()
