"""Guide tree (single-linkage merge list).

The oracle's Kruskal merge list is pinned to a naive O(k^3) agglomeration
that applies the same rule (merge the two clusters holding the most similar
cross pair, equal similarities by the pair (i, j)) -- exact equality, ties
included -- and, on inputs without equal similarities, to SciPy's single
linkage.  The library's famsa_guide_tree (host code) must reproduce the
oracle's list from the oracle tree's edges in any order, and the host SLINK
path (famsa_slink_guide_tree) must give the same clusters where the tree is
unique and the same heights always."""
import ctypes
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs
from test_slink import feed_descending


def sim_key(s):
    return (1, 0) if s == oracle.INF else (0, s)


def naive_agglomeration(M, L):
    """Merge, k-1 times, the two clusters holding the most similar cross pair
    (i, j); equal similarities: smallest (i, j).  Cluster ids as the oracle's."""
    k = M.shape[0]
    clusters = {i: {i} for i in range(k)}
    merges = []
    while len(clusters) > 1:
        best = None
        for a in clusters:
            for b in clusters:
                if a == b:
                    continue
                for i in clusters[a]:
                    for j in clusters[b]:
                        if i >= j:
                            continue
                        s = oracle.similarity(int(M[i, j]), int(L[i]), int(L[j]))
                        key = (sim_key(s), -i, -j)
                        if best is None or key > best[0]:
                            best = (key, a, b, s)
        _, a, b, s = best
        new = k + len(merges)
        merges.append((a, b, s))
        clusters[new] = clusters.pop(a) | clusters.pop(b)
    return merges


def family_matrix(seed, k, lo, hi, sigma):
    b = inputs.random_family(k, lo, hi, seed, alphabet=sigma)
    return oracle.full_matrix(b.codes, b.seq_off, 0, k), b.lengths()


def clusters_of(merges, k):
    sets = [frozenset([i]) for i in range(k)]
    out = []
    for l, r, *_ in merges:
        sets.append(sets[int(l)] | sets[int(r)])
        out.append(sets[-1])
    return out


@pytest.mark.parametrize("seed,k,lo,hi,sigma", [(1, 12, 0, 12, 2), (2, 18, 3, 40, 4), (3, 25, 20, 60, 20),
                                                (4, 9, 0, 3, 2), (5, 1, 4, 4, 2), (6, 2, 5, 5, 2)])
def test_oracle_guide_tree_equals_naive_agglomeration(seed, k, lo, hi, sigma):
    M, L = family_matrix(seed, k, lo, hi, sigma)
    assert oracle.guide_tree(M, L) == naive_agglomeration(M, L)


def distinct_similarity_case(seed, k):
    """Synthetic LCS values and lengths whose k(k-1)/2 similarities are all different."""
    rng = np.random.default_rng(seed)
    while True:
        L = rng.integers(200, 400, k)
        M = np.zeros((k, k), np.int64)
        for i in range(k):
            for j in range(i + 1, k):
                M[i, j] = M[j, i] = rng.integers(0, min(L[i], L[j]) + 1)
        sims = [oracle.similarity(int(M[i, j]), int(L[i]), int(L[j])) for i in range(k) for j in range(i + 1, k)]
        if len(set(sims)) == len(sims):
            return M, L


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_guide_tree_matches_scipy_without_ties(seed):
    hierarchy = pytest.importorskip("scipy.cluster.hierarchy")
    k = 30
    M, L = distinct_similarity_case(seed, k)
    sims = {(i, j): oracle.similarity(int(M[i, j]), int(L[i]), int(L[j])) for i in range(k) for j in range(i + 1, k)}
    # distance = rank of the similarity, most similar first: same order, no rounding
    rank = {p: r for r, p in enumerate(sorted(sims, key=lambda p: sims[p], reverse=True))}
    cond = np.array([rank[(i, j)] + 1.0 for i in range(k) for j in range(i + 1, k)])
    Z = hierarchy.linkage(cond, method="single")
    got = oracle.guide_tree(M, L)
    assert clusters_of(got, k) == clusters_of([(a, b) for a, b, _, _ in Z], k)
    order = sorted(sims.values(), reverse=True)
    assert [s for _, _, s in got] == [order[int(d) - 1] for d in Z[:, 2]]


def oracle_edges(M, L):
    """The tie-broken maximum spanning tree's edges, from Kruskal as the oracle orders pairs."""
    k = M.shape[0]
    edges = sorted(((oracle.similarity(int(M[i, j]), int(L[i]), int(L[j])), i, j)
                    for i in range(k) for j in range(i + 1, k)),
                   key=lambda e: (sim_key(e[0])[0] * -1, -e[0] if e[0] != oracle.INF else 0, e[1], e[2]))
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    out = []
    for s, i, j in edges:
        a, b = find(i), find(j)
        if a != b:
            parent[a] = b
            out.append((i, j, int(M[i, j]), (int(L[i]) + int(L[j]) - 2 * int(M[i, j])) ** 2))
    return out


def to_sim(num, den):
    return oracle.INF if den == 0 else Fraction(int(num), int(den))


@pytest.mark.parametrize("seed,k,lo,hi,sigma", [(1, 12, 0, 12, 2), (3, 25, 20, 60, 20), (7, 40, 0, 30, 3),
                                                (5, 1, 4, 4, 2), (6, 2, 5, 5, 2)])
def test_library_guide_tree_from_edges(seed, k, lo, hi, sigma):
    M, L = family_matrix(seed, k, lo, hi, sigma)
    want = oracle.guide_tree(M, L)
    e = oracle_edges(M, L)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(e))
    # edges in any order and either orientation
    u = [e[p][1] if p % 2 else e[p][0] for p in perm]
    v = [e[p][0] if p % 2 else e[p][1] for p in perm]
    left, right, num, den = B.guide_tree(k, u, v, [e[p][2] for p in perm], [e[p][3] for p in perm])
    got = [(int(a), int(b), to_sim(n, d)) for a, b, n, d in zip(left, right, num, den)]
    assert got == want
    nw = B.newick(left, right, k)
    assert nw.endswith(";") and nw.count("(") == max(k - 1, 0) and all(str(i) in nw for i in range(k))


def test_library_guide_tree_errors_and_forests():
    with pytest.raises(B.FamsaError):
        B.guide_tree(3, [0, 1, 0], [1, 2, 2], [1, 1, 1], [1, 1, 1])  # more than k-1 edges
    with pytest.raises(B.FamsaError):
        B.guide_tree(4, [0, 1, 0], [1, 2, 2], [1, 1, 1], [1, 1, 1])  # a cycle
    with pytest.raises(B.FamsaError):
        B.guide_tree(3, [0], [3], [1], [1])  # out of range
    with pytest.raises(B.FamsaError):
        B.guide_tree(3, [0], [0], [1], [1])  # a loop
    with pytest.raises(B.FamsaError):
        B.guide_tree(3, [0], [1], [-1], [4])  # negative similarity
    left, right, num, den = B.guide_tree(5, [3, 0], [4, 1], [2, 5], [0, 9])  # a forest: +inf first
    assert list(left) == [3, 0] and list(right) == [4, 1] and list(den) == [0, 9]
    assert B.newick(left, right, 5) == "(2,(3,4),(0,1));"
    assert B.guide_tree(0, [], [], [], [])[0].size == 0


@pytest.mark.parametrize("seed,k,lo,hi,sigma,R", [(1, 12, 0, 12, 2, 5), (3, 25, 20, 60, 20, 7),
                                                  (8, 33, 0, 40, 3, 64)])
def test_host_slink_guide_tree(seed, k, lo, hi, sigma, R):
    M, L = family_matrix(seed, k, lo, hi, sigma)
    s = B.SLink(L)
    feed_descending(s, M, k, R)
    left, right, num, den = s.guide_tree()
    got = [(int(a), int(b), to_sim(n, d)) for a, b, n, d in zip(left, right, num, den)]
    want = oracle.guide_tree(M, L)
    assert [x for _, _, x in got] == [x for _, _, x in want]  # heights, in merge order
    # the partition after all merges of each height is the same
    for cut in sorted({x for _, _, x in want}, key=sim_key):
        def parts(ms):
            sets = {i: frozenset([i]) for i in range(k)}
            for t, (a, b, x) in enumerate(ms):
                if sim_key(x) >= sim_key(cut):
                    sets[k + t] = sets.pop(a) | sets.pop(b)
                else:
                    break
            return set(sets.values())
        assert parts(got) == parts(want)
    s.close()


def test_host_slink_guide_tree_without_ties_is_the_oracle_tree():
    k = 24
    M, L = distinct_similarity_case(5, k)
    s = B.SLink(L)
    feed_descending(s, M, k, 5)
    left, right, num, den = s.guide_tree()
    want = oracle.guide_tree(M, L)
    assert clusters_of(list(zip(left, right)), k) == clusters_of(want, k)
    s.close()


@pytest.mark.parametrize("seed,k,lo,hi,sigma", [(1, 12, 0, 12, 2), (3, 25, 20, 60, 20), (9, 1, 3, 3, 2)])
def test_leaf_order_makes_every_cluster_a_range(seed, k, lo, hi, sigma):
    M, L = family_matrix(seed, k, lo, hi, sigma)
    want = oracle.guide_tree(M, L)
    left = [a for a, _, _ in want]
    right = [b for _, b, _ in want]
    order, first, size = B.leaf_order(left, right, k)
    assert sorted(order) == list(range(k))
    members = clusters_of(want, k)
    for c in range(k + len(want)):
        leaves = {c} if c < k else members[c - k]
        assert set(order[first[c]:first[c] + size[c]]) == leaves
    for t, (a, b, _) in enumerate(want):  # merging profiles are adjacent, left first
        assert first[a] == first[k + t] and first[b] == first[a] + size[a]


def test_leaf_order_and_newick_of_a_forest_and_errors():
    left, right = [3, 0], [4, 1]
    order, first, size = B.leaf_order(left, right, 5)
    assert list(order) == [2, 3, 4, 0, 1]
    with pytest.raises(B.FamsaError):
        B.leaf_order([0, 0], [1, 2], 3)  # cluster 0 merged twice
    with pytest.raises(B.FamsaError):
        B.newick([0], [5], 3)  # no cluster 5 yet
    assert B.newick([], [], 1) == "0;"


@pytest.mark.parametrize("seed,k,lo,hi,sigma", [(1, 12, 0, 12, 2), (3, 25, 20, 60, 20), (7, 40, 0, 30, 3)])
def test_spanning_forest_of_all_pairs_and_of_merged_shards(seed, k, lo, hi, sigma):
    M, L = family_matrix(seed, k, lo, hi, sigma)
    want = oracle_edges(M, L)
    ii, jj = np.triu_indices(k, 1)
    lcs = M[ii, jj].astype(np.int64)
    d2 = (L[ii].astype(np.int64) + L[jj] - 2 * lcs) ** 2
    u, v, n, d = B.spanning_forest(k, ii, jj, lcs, d2)
    assert list(zip(u.tolist(), v.tolist(), n.tolist(), d.tolist())) == want
    # forests of disjoint shards of the pairs, merged, give the same forest
    rng = np.random.default_rng(seed)
    shard = rng.integers(0, 3, ii.size)
    parts = [B.spanning_forest(k, ii[shard == s], jj[shard == s], lcs[shard == s], d2[shard == s]) for s in range(3)]
    cat = [np.concatenate([p[x] for p in parts]) for x in range(4)]
    u2, v2, n2, d2_ = B.spanning_forest(k, *cat)
    assert list(zip(u2.tolist(), v2.tolist(), n2.tolist(), d2_.tolist())) == want


def test_spanning_forest_errors():
    with pytest.raises(B.FamsaError):
        B.spanning_forest(3, [0], [3], [1], [1])
    with pytest.raises(B.FamsaError):
        B.spanning_forest(3, [1], [1], [1], [1])
    u, v, n, d = B.spanning_forest(4, [0, 1, 0, 2], [1, 0, 1, 3], [1, 1, 1, 1], [4, 4, 4, 0])
    assert list(zip(u, v)) == [(2, 3), (0, 1)]  # +inf first; the duplicate pairs close cycles
