"""The host single-linkage consumer (famsa_slink_*) against the oracle's
Kruskal single linkage on exact LCS matrices.  Tiles are built on the CPU
from the oracle's rows and fed in descending order, as the library delivers
them under FAMSA_LCS_DESCENDING.  Only tie-independent quantities are
compared: the multiset of merge similarities and the cophenetic similarity
of every pair."""
import ctypes
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs


def feed_descending(s, M, k, R):
    tiles = []
    for r0 in range(0, k, R):
        r1 = min(k, r0 + R)
        vals = np.concatenate([M[i, i + 1:] for i in range(r0, r1)]).astype(np.int32) if r1 > r0 else \
            np.zeros(0, np.int32)
        tiles.append((r0, r1, np.ascontiguousarray(vals)))
    for idx, (r0, r1, vals) in enumerate(reversed(tiles)):
        t = B.Tile()
        t.tile_index = idx
        t.family = 0
        t.k = k
        t.row_begin = r0
        t.row_end = r1
        t.count = vals.size
        t.lcs = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if vals.size else None
        assert s.feed(t) == 0


def to_sim(num, den):
    return oracle.INF if den == 0 else Fraction(int(num), int(den))


def pointer_to_linkage(pi, num, den):
    """Merge heights and cophenetic matrix from the pointer representation
    (merge each non-root point with its pointer's cluster, most similar first)."""
    k = len(pi)
    order = [i for i in range(k) if not (num[i] == -1 and den[i] == 0)]
    order.sort(key=lambda i: to_sim(num[i], den[i]), reverse=True)
    parent = list(range(k))
    members = {i: [i] for i in range(k)}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    coph = np.empty((k, k), dtype=object)
    for i in range(k):
        coph[i, i] = oracle.INF
    heights = []
    for i in order:
        a, b = find(i), find(int(pi[i]))
        assert a != b
        h = to_sim(num[i], den[i])
        for x in members[a]:
            for y in members[b]:
                coph[x, y] = coph[y, x] = h
        parent[b] = a
        members[a] += members.pop(b)
        heights.append(h)
    return heights, coph


@pytest.mark.parametrize("seed,k,lo,hi,sigma,R", [(1, 25, 0, 20, 3, 4), (2, 40, 5, 40, 20, 7), (3, 33, 1, 6, 2, 1),
                                                  (4, 60, 10, 60, 4, 64), (5, 2, 3, 3, 2, 1), (6, 1, 3, 3, 2, 1)])
def test_slink_matches_kruskal(seed, k, lo, hi, sigma, R):
    b = inputs.random_family(k, lo, hi, seed, alphabet=sigma)
    if seed == 3:  # duplicates and empties: identical pairs have similarity +inf
        seqs = [b.seq(i) for i in range(k)]
        seqs[5] = seqs[6].copy()
        seqs[7] = np.zeros(0, np.uint8)
        seqs[8] = np.zeros(0, np.uint8)
        b = inputs.from_sequences(seqs)
    M = oracle.full_matrix(b.codes, b.seq_off, 0, k)
    L = b.lengths()
    s = B.SLink(L)
    feed_descending(s, M, k, R)
    assert s.rows_done() == k
    pi, num, den = s.result()
    assert sum(1 for i in range(k) if num[i] == -1 and den[i] == 0) == 1
    h, coph = pointer_to_linkage(pi, num, den)
    h_ref, c_ref = oracle.single_linkage(M, L)
    assert sorted(h, reverse=True) == sorted(h_ref, reverse=True)
    assert (coph == c_ref).all()


def test_slink_rejects_out_of_order():
    b = inputs.random_family(10, 3, 9, 0)
    s = B.SLink(b.lengths())
    vals = np.zeros(9, np.int32)
    t = B.Tile()
    t.k, t.row_begin, t.row_end, t.count = 10, 0, 1, 9   # first row first: wrong order
    t.lcs = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert s.feed(t) != 0
    assert B.lib().famsa_slink_result(s.handle, None, None, None) == B.EINVAL
