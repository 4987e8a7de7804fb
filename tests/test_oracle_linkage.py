"""Pins for the oracle's single linkage (paper, Methods, "Determination of
the guide tree"): Kruskal's merge heights and cophenetic similarities equal
(a) SciPy's single-linkage routine and (b) a naive agglomerative loop that
repeatedly merges the two clusters with the most similar pair of members.
Only tie-independent quantities are compared."""
import numpy as np
import pytest
from fractions import Fraction

import oracle
from paper_1603_06958_amd import inputs


def naive_single_linkage(S):
    """S: k x k similarity (object); merges by brute force, O(k^3)."""
    k = S.shape[0]
    clusters = [[i] for i in range(k)]
    heights = []
    coph = np.empty((k, k), dtype=object)
    for i in range(k):
        coph[i, i] = oracle.INF
    while len(clusters) > 1:
        best = None
        for x in range(len(clusters)):
            for y in range(x + 1, len(clusters)):
                s = max(S[i, j] for i in clusters[x] for j in clusters[y])
                if best is None or s > best[0]:
                    best = (s, x, y)
        s, x, y = best
        for i in clusters[x]:
            for j in clusters[y]:
                coph[i, j] = coph[j, i] = s
        heights.append(s)
        clusters[x] = clusters[x] + clusters[y]
        del clusters[y]
    return heights, coph


def sim_matrix(M, L):
    k = M.shape[0]
    S = np.empty((k, k), dtype=object)
    for i in range(k):
        for j in range(k):
            S[i, j] = oracle.INF if i == j else oracle.similarity(int(M[i, j]), int(L[i]), int(L[j]))
    return S


@pytest.mark.parametrize("seed,k,lo,hi,sigma", [(1, 12, 0, 12, 3), (2, 20, 5, 30, 4), (3, 30, 10, 40, 20),
                                                 (4, 16, 3, 6, 2)])
def test_kruskal_vs_naive(seed, k, lo, hi, sigma):
    b = inputs.random_family(k, lo, hi, seed, alphabet=sigma)
    M = oracle.full_matrix(b.codes, b.seq_off, 0, k)
    L = b.lengths()
    h1, c1 = oracle.single_linkage(M, L)
    h2, c2 = naive_single_linkage(sim_matrix(M, L))
    assert sorted(h1, reverse=True) == sorted(h2, reverse=True)
    assert (c1 == c2).all()


def test_kruskal_vs_scipy():
    from scipy.cluster.hierarchy import linkage, cophenet
    from scipy.spatial.distance import squareform
    b = inputs.random_family(60, 20, 80, 9, alphabet=4)
    k = b.nseq
    M = oracle.full_matrix(b.codes, b.seq_off, 0, k)
    L = b.lengths()
    S = sim_matrix(M, L)
    # distance = rank of similarity (most similar -> smallest); exact, ties kept equal
    vals = sorted({S[i, j] for i in range(k) for j in range(i + 1, k)}, reverse=True)
    rank = {v: r for r, v in enumerate(vals)}
    D = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            if i != j:
                D[i, j] = rank[S[i, j]]
    Z = linkage(squareform(D), method="single")
    h_ref = sorted(vals[int(round(x))] for x in Z[:, 2])
    h, coph = oracle.single_linkage(M, L)
    assert sorted(h) == h_ref
    cref = squareform(cophenet(Z))
    for i in range(k):
        for j in range(i + 1, k):
            assert coph[i, j] == vals[int(round(cref[i, j]))]
