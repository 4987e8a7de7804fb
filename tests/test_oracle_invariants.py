"""Closed forms and invariants of LCS length that pin the oracle.

LCS(a, a) = |a|; LCS(x^p, x^q) = min(p, q); LCS(a, s) = |s| for a
subsequence s of a; LCS(a.c, b.c) = LCS(a, b) + 1; disjoint alphabets give 0;
symmetry; 0 <= LCS <= min(|a|, |b|); appending one symbol raises LCS by 0 or 1;
reversal and relabelling of the alphabet leave it unchanged; the indel
distance (paper, Methods: indel = |A| + |B| - 2 LCS) is a metric.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle

seqs = st.lists(st.integers(0, 5), max_size=40)
seqs20 = st.lists(st.integers(0, 19), max_size=60)


@given(seqs20)
@settings(max_examples=150, deadline=None)
def test_self(a):
    assert oracle.lcs(a, a) == len(a)


@given(st.integers(0, 200), st.integers(0, 200), st.integers(0, 19))
@settings(max_examples=100, deadline=None)
def test_homopolymer(p, q, x):
    assert oracle.lcs([x] * p, [x] * q) == min(p, q)


@given(seqs20, st.data())
@settings(max_examples=150, deadline=None)
def test_subsequence(a, data):
    keep = data.draw(st.lists(st.booleans(), min_size=len(a), max_size=len(a)))
    s = [c for c, k in zip(a, keep) if k]
    assert oracle.lcs(a, s) == len(s)
    assert oracle.lcs(s, a) == len(s)


@given(seqs, seqs, st.integers(0, 5))
@settings(max_examples=200, deadline=None)
def test_common_suffix(a, b, c):
    assert oracle.lcs(a + [c], b + [c]) == oracle.lcs(a, b) + 1


@given(st.lists(st.integers(0, 9), max_size=50), st.lists(st.integers(10, 19), max_size=50))
@settings(max_examples=100, deadline=None)
def test_disjoint(a, b):
    assert oracle.lcs(a, b) == 0


@given(seqs, seqs)
@settings(max_examples=300, deadline=None)
def test_symmetry_bounds_reversal(a, b):
    L = oracle.lcs(a, b)
    assert L == oracle.lcs(b, a)
    assert 0 <= L <= min(len(a), len(b))
    assert L == oracle.lcs(a[::-1], b[::-1])


@given(seqs, seqs, st.integers(0, 5))
@settings(max_examples=300, deadline=None)
def test_append_step(a, b, x):
    d = oracle.lcs(a + [x], b) - oracle.lcs(a, b)
    assert d in (0, 1)


@given(seqs, seqs, st.permutations(list(range(6))))
@settings(max_examples=150, deadline=None)
def test_relabel(a, b, perm):
    assert oracle.lcs([perm[c] for c in a], [perm[c] for c in b]) == oracle.lcs(a, b)


@given(seqs, seqs, seqs)
@settings(max_examples=200, deadline=None)
def test_indel_metric(a, b, c):
    d = lambda x, y: oracle.indel(oracle.lcs(x, y), len(x), len(y))
    assert d(a, b) >= abs(len(a) - len(b))
    assert (d(a, b) == 0) == (a == b)
    assert d(a, c) <= d(a, b) + d(b, c)


def test_similarity_cases():
    from fractions import Fraction
    assert oracle.similarity(3, 3, 3) == oracle.INF          # identical: indel 0
    assert oracle.similarity(0, 0, 0) == oracle.INF          # both empty are identical
    assert oracle.similarity(0, 2, 3) == 0
    assert oracle.similarity(2, 3, 4) == Fraction(2, 9)      # indel = 3 + 4 - 4 = 3
