"""Pins for the oracle of aligning one sequence to a profile (oracle.profile),
against facts other than itself:

* the gap-type rules, checked by hand on small profiles where the paper's
  six situations (Methods, "Gap types and costs determination") decide the
  cost, with gap costs of different magnitudes so every total names the
  types it holds;
* reductions to LCS: with score 1 for equal symbols, 0 otherwise and free
  gaps, a one-row profile gives LCS(A, B); with unit gaps and mismatches
  forbidden it gives -(|A| + |B| - 2 LCS), the indel distance of the LCS
  section;
* a profile of K identical rows scores K times its one-row profile;
* brute force: on tiny inputs the DP's score is the maximum of the direct
  alignment score over every alignment, and the DP's own alignment scores
  its score;
* the gap-scale formula at points where it is exact.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import profile as P

G = P.GAP
M, D, I = P.OP_M, P.OP_D, P.OP_I
COSTS = (100, 10, 1000, 1)  # To, Te, Go, Ge: any total names its gap types


def zero_S(sigma=4):
    return np.zeros((sigma, sigma), dtype=np.int64)


@pytest.mark.parametrize("rows,seq,ops,want", [
    # inside a row, no gap next to it: the inserted gap opens a series (Go)
    ([[0, 0]], [0, 0, 0], [M, I, M], -1000),
    # a gap open on the right: inserted becomes the open, the old one an extension: Ge
    ([[0, G, 0]], [0, 0, 0], [M, I, D, M], -1),
    # inside a gap series: Ge
    ([[0, G, G, 0]], [0, 0, 0], [M, D, I, D, M], -1),
    # in front of a leading (terminal) gap open: net Te
    ([[G, 0]], [0, 0], [I, D, M], -10),
    # after a leading gap: a terminal extension, Te
    ([[G, G, 0]], [0, 0], [D, I, D, M], -10),
    # before the first residue of a row that starts with one: a terminal open, To
    ([[0, 0]], [0, 0, 0], [I, M, M], -100),
    # after the last residue: To, and each further column Te
    ([[0, 0]], [0, 0, 0], [M, M, I], -100),
    ([[0, 0]], [0, 0, 0, 0, 0], [M, M, I, I, I], -120),
    # in front of a trailing gap series: net Te
    ([[0, G]], [0, 0], [M, I, D], -10),
    # three rows at one boundary: inside and opening (Go), leading region
    # next to a gap (Te), trailing region next to a gap (Te)
    ([[0, 0], [G, 0], [0, G]], [0, 0, 0], [M, I, M], -1020),
    # gaps in the sequence: weighted by the rows with a residue in the column;
    # leading and trailing ones terminal
    ([[0, 0, 0], [0, G, 0]], [0], [D, M, D], -400),
    ([[0, 0, 0], [0, G, 0]], [0], [M, D, D], -120),
    ([[0, 0, 0]], [0, 0], [M, D, M], -1000),
    ([[0, 0, 0, 0]], [0, 0], [M, D, D, M], -1001),
    # a D run and an I run back to back are two runs
    ([[0, 0, 0]], [0, 0, 0], [M, D, I, M], -2000),
])
def test_gap_rules_by_hand(rows, seq, ops, want):
    assert P.alignment_score(seq, rows, zero_S(), COSTS, ops) == want


def test_column_scores_by_hand():
    S = np.eye(4, dtype=np.int64) * 5 - 1  # 4 on the diagonal, -1 off it
    rows = [[1, 2], [1, G], [3, 2]]
    # column 1 holds 1, 1, 3 against residue 1: 4 + 4 - 1; column 2 holds 2, -, 2 against 2: 4 + 4
    assert P.alignment_score([1, 2], rows, S, (0, 0, 0, 0), [M, M]) == 15
    cost, w = P.column_costs(rows, S)
    assert cost[0].tolist() == [-3, 7, -3, 2] and w.tolist() == [3, 2]


@pytest.mark.parametrize("seed", range(4))
def test_reduces_to_lcs(seed):
    rng = np.random.default_rng(500 + seed)
    sigma = [20, 3, 2, 20][seed]
    S = np.eye(sigma, dtype=np.int64)
    for _ in range(12):
        a = rng.integers(0, sigma, rng.integers(0, 60))
        b = rng.integers(0, sigma, rng.integers(0, 60))
        score, ops = P.align(a, [b], S, (0, 0, 0, 0))
        assert score == oracle.lcs(a, b)
        assert P.alignment_score(a, [b], S, (0, 0, 0, 0), ops) == score


@pytest.mark.parametrize("seed", range(4))
def test_reduces_to_minus_indel(seed):
    rng = np.random.default_rng(600 + seed)
    sigma = [20, 3, 2, 5][seed]
    for _ in range(12):
        a = rng.integers(0, sigma, rng.integers(0, 50))
        b = rng.integers(0, sigma, rng.integers(0, 50))
        big = 4 * (a.size + b.size) + 10
        S = np.where(np.eye(sigma, dtype=bool), 0, -big).astype(np.int64)
        score, ops = P.align(a, [b], S, (1, 1, 1, 1))
        L = oracle.lcs(a, b)
        assert score == -(a.size + b.size - 2 * L)
        assert sum(1 for o in ops if o == M) == L


@pytest.mark.parametrize("seed", range(3))
def test_k_identical_rows_scale(seed):
    rng = np.random.default_rng(700 + seed)
    sigma = 6
    S = rng.integers(-4, 6, (sigma, sigma)).astype(np.int64)
    for _ in range(8):
        a = rng.integers(0, sigma, rng.integers(0, 30))
        row = rng.integers(0, sigma, rng.integers(0, 30)).astype(np.int64)
        gaps = rng.random(row.size) < 0.3
        row[gaps] = G
        costs = tuple(int(x) for x in rng.integers(0, 7, 4))
        s1, o1 = P.align(a, [row], S, costs)
        for K in (2, 5):
            sk, ok = P.align(a, [row] * K, S, costs)
            assert sk == K * s1 and ok == o1


def all_alignments(m, n):
    for k in range(min(m, n) + 1):
        base = [M] * k + [D] * (n - k) + [I] * (m - k)
        for perm in set(itertools.permutations(base)):
            yield list(perm)


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_optimum(seed):
    rng = np.random.default_rng(800 + seed)
    sigma = 3
    for _ in range(10):
        m, n = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        K = int(rng.integers(1, 4))
        rows = rng.integers(0, sigma, (K, n)).astype(np.int64)
        rows[rng.random((K, n)) < 0.35] = G
        a = rng.integers(0, sigma, m)
        S = rng.integers(-3, 5, (sigma, sigma)).astype(np.int64)
        costs = tuple(int(x) for x in rng.integers(0, 6, 4))
        score, ops = P.align(a, rows, S, costs)
        best = max(P.alignment_score(a, rows, S, costs, o) for o in all_alignments(m, n))
        assert score == best
        assert P.alignment_score(a, rows, S, costs, ops) == score


def test_empty_sides():
    S = np.eye(3, dtype=np.int64)
    assert P.align([], [[]], S, COSTS) == (0, [])
    # only gaps into the sequence: a leading (terminal) run over both columns
    assert P.align([], [[0, 1], [G, 1]], S, COSTS) == (-(1 * 100 + 2 * 10), [D, D])
    # only new columns in an empty-width profile: each row terminal, To then Te
    assert P.align([0, 1, 2], [[], []], S, COSTS) == (-2 * (100 + 2 * 10), [I, I, I])


def test_gap_runs_rebuild_the_alignment():
    from oracle import gapped as Gd
    rng = np.random.default_rng(901)
    sigma = 5
    S = rng.integers(-2, 6, (sigma, sigma)).astype(np.int64)
    for _ in range(20):
        a = rng.integers(0, sigma, rng.integers(0, 25))
        rows = rng.integers(0, sigma, (3, int(rng.integers(0, 25)))).astype(np.int64)
        rows[rng.random(rows.shape) < 0.3] = G
        score, ops = P.align(a, rows, S, (3, 1, 6, 2))
        sr, pr = P.gap_runs(ops)
        ga = Gd.insert_runs(Gd.from_symbols(a.tolist()), sr)[1:]
        assert len(ga) == len(ops)
        for s in range(rows.shape[0]):
            gr = Gd.insert_runs(Gd.from_symbols(rows[s].tolist()), pr)[1:]
            assert len(gr) == len(ops)
        # residues sit against columns exactly where the alignment says M
        for t, o in enumerate(ops):
            assert (ga[t] is not None) == (o != D)


def test_gap_scale():
    assert P.gap_scale(45) == 1.0
    assert abs(P.gap_scale(45 * math.exp(7)) - 2.0) < 1e-12
    assert abs(P.gap_scale(1) - (1 - math.log(45) / 7)) < 1e-15
    assert abs(P.gap_scale(10, gl=10, gd=3) - 1.0) < 1e-15
    # rounding of the scaled costs: half away from zero
    assert P.scaled_gap_costs(45, (1.5, -1.5, 2.4, 0)) == (2, -2, 2, 0)
    assert P.scaled_gap_costs(45 * math.exp(7), (3, 5, 7, 11)) == (6, 10, 14, 22)
