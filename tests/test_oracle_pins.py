"""Pins for the CPU oracle's LCS (DP rule) against facts other than itself.

* brute force: the largest subsequence of A that is also a subsequence of B,
  enumerated exhaustively on tiny strings;
* textbook worked examples (tests/golden/lcs_textbook.txt);
* an independent recurrence: the indel distance (insertions and deletions
  only, unit cost) computed by its own DP, and the paper's identity
  indel = |A| + |B| - 2 * LCS (Methods, "Pairwise similarities calculation");
* an independent algorithm: a big-integer bit-parallel LCS (the family of
  methods the paper cites for w-cells-at-a-time computation), written here in
  Python.
"""
import itertools
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def is_subseq(s, t):
    it = iter(t)
    return all(c in it for c in s)


def brute_lcs(a, b):
    a, b = list(a), list(b)
    for r in range(min(len(a), len(b)), 0, -1):
        for idx in itertools.combinations(range(len(a)), r):
            if is_subseq([a[i] for i in idx], b):
                return r
    return 0


def indel_dp(a, b):
    """Edit distance with only unit-cost insertions and deletions."""
    m, n = len(a), len(b)
    prev = list(range(n + 1))
    for i in range(1, m + 1):
        cur = [i] + [0] * n
        for j in range(1, n + 1):
            if a[i - 1] == b[j - 1]:
                cur[j] = prev[j - 1]
            else:
                cur[j] = 1 + min(prev[j], cur[j - 1])
        prev = cur
    return prev[n]


def bitparallel_lcs(a, b):
    """Bit-vector LCS length on Python ints (bit p of a word = position p of a)."""
    m = len(a)
    if m == 0 or len(b) == 0:
        return 0
    full = (1 << m) - 1
    pm = {}
    for p, c in enumerate(a):
        pm[c] = pm.get(c, 0) | (1 << p)
    v = full
    for c in b:
        u = v & pm.get(c, 0)
        v = ((v + u) | (v - u)) & full
    return m - bin(v).count("1")


def test_bruteforce_exhaustive_binary():
    strings = [s for n in range(0, 7) for s in itertools.product((0, 1), repeat=n)]
    for a in strings:
        for b in strings:
            if len(a) + len(b) > 11:
                continue
            assert oracle.lcs(a, b) == brute_lcs(a, b), (a, b)


def test_bruteforce_exhaustive_ternary():
    strings = [s for n in range(0, 5) for s in itertools.product((0, 1, 2), repeat=n)]
    for a in strings:
        for b in strings:
            assert oracle.lcs(a, b) == brute_lcs(a, b), (a, b)


def test_bruteforce_random_20():
    rng = np.random.default_rng(11)
    for _ in range(400):
        a = rng.integers(0, 20, rng.integers(0, 11))
        b = rng.integers(0, 20, rng.integers(0, 11))
        assert oracle.lcs(a, b) == brute_lcs(a.tolist(), b.tolist())
    for _ in range(200):  # small alphabets make long common subsequences
        a = rng.integers(0, 3, rng.integers(0, 12))
        b = rng.integers(0, 3, rng.integers(0, 12))
        assert oracle.lcs(a, b) == brute_lcs(a.tolist(), b.tolist())


def test_golden_textbook():
    n = 0
    with open(os.path.join(HERE, "golden", "lcs_textbook.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, v, _src = line.rstrip("\n").split("\t")
            enc = lambda s: [ord(c) - ord("A") for c in s]
            assert oracle.lcs(enc(a), enc(b)) == int(v), line
            assert oracle.lcs(enc(b), enc(a)) == int(v), line
            n += 1
    assert n >= 7


@pytest.mark.parametrize("seed", range(6))
def test_indel_identity(seed):
    rng = np.random.default_rng(100 + seed)
    sigma = [2, 4, 20, 20, 20, 32][seed]
    for _ in range(6):
        m, n = int(rng.integers(0, 160)), int(rng.integers(0, 160))
        a = rng.integers(0, sigma, m).tolist()
        b = rng.integers(0, sigma, n).tolist()
        L = oracle.lcs(a, b)
        assert oracle.indel(L, m, n) == indel_dp(a, b)


@pytest.mark.parametrize("seed", range(4))
def test_bitparallel_independent(seed):
    rng = np.random.default_rng(200 + seed)
    for m, n in [(1, 1), (31, 33), (63, 64), (64, 65), (257, 300), (1000, 900), (3000, 2500)]:
        sigma = [2, 5, 20, 20][seed]
        a = rng.integers(0, sigma, m).tolist()
        b = rng.integers(0, sigma, n).tolist()
        assert oracle.lcs(a, b) == bitparallel_lcs(a, b), (m, n)


def test_pairs_and_rows_layout():
    from paper_1603_06958_amd import inputs
    b = inputs.random_family(13, 0, 40, seed=5)
    k = b.nseq
    tri = oracle.tile_expected(b.codes, b.seq_off, 0, k, 0, k)
    assert tri.size == k * (k - 1) // 2
    p = 0
    for i in range(k):
        for j in range(i + 1, k):
            assert tri[p] == brute_lcs(b.seq(i).tolist(), b.seq(j).tolist()) if len(b.seq(i)) <= 12 else True
            assert tri[p] == oracle.lcs(b.seq(i), b.seq(j))
            p += 1
    part = oracle.tile_expected(b.codes, b.seq_off, 0, k, 4, 9)
    start = sum(k - 1 - i for i in range(4))
    assert np.array_equal(part, tri[start:start + part.size])
    ia = np.array([0, 3, 12]); ib = np.array([5, 3, 1])
    got = oracle.lcs_pairs(b.codes, b.seq_off, ia, ib)
    assert got.tolist() == [oracle.lcs(b.seq(x), b.seq(y)) for x, y in zip(ia, ib)]


@pytest.mark.parametrize("seed", range(3))
def test_full_matrix_pairwise(seed):
    """full_matrix (the k x k matrix the linkage pins and GPU consumer tests
    read) against one oracle.lcs call per pair: every (i, j) in both triangles,
    the symmetry and the diagonal (LCS(a, a) = |a|), on families holding empty
    and repeated sequences; on tiny families also against brute force."""
    rng = np.random.default_rng(300 + seed)
    k = [17, 23, 9][seed]
    sigma = [20, 3, 2][seed]
    hi = [40, 14, 8][seed]
    seqs = [rng.integers(0, sigma, rng.integers(0, hi)).astype(np.uint8) for _ in range(k)]
    seqs[2] = np.zeros(0, np.uint8)            # empty
    seqs[5] = seqs[1].copy()                   # repeated
    seqs[k - 1] = seqs[0][::-1].copy()         # reversal of another
    seqs.insert(3, np.zeros(0, np.uint8))      # second empty
    k += 1
    codes = np.concatenate(seqs) if sum(s.size for s in seqs) else np.zeros(0, np.uint8)
    off = np.zeros(k + 1, np.uint64)
    off[1:] = np.cumsum([s.size for s in seqs])
    # a family inside a larger batch: one leading sequence before it
    lead = rng.integers(0, sigma, 7).astype(np.uint8)
    codes2 = np.concatenate([lead, codes])
    off2 = np.concatenate([[0], off + lead.size]).astype(np.uint64)
    for cc, oo, base in ((codes, off, 0), (codes2, off2, 1)):
        M = oracle.full_matrix(cc, oo, base, k)
        assert M.shape == (k, k)
        assert np.array_equal(M, M.T)
        for i in range(k):
            assert M[i, i] == seqs[i].size
            for j in range(k):
                if i != j:
                    assert M[i, j] == oracle.lcs(seqs[i], seqs[j]), (i, j)
        if seed == 2:
            for i in range(k):
                for j in range(i + 1, k):
                    assert M[i, j] == brute_lcs(seqs[i].tolist(), seqs[j].tolist()), (i, j)
