"""CPU oracle for the all-pairs LCS similarity stage -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_1603_06958_amd``): it neither imports it nor is imported by it.  The
only common dependency is the seeded input generator, which holds none of the
method's arithmetic.

Contents, each following the FAMSA paper (Methods):

* ``lcs`` / ``lcs_pairs`` / ``tile_expected`` -- LCS length by the textbook
  dynamic-programming rule ("Pairwise similarities calculation"), in the C
  file ``lcs_dp.c`` next to this one.
* ``indel`` and ``similarity`` -- the indel distance |A|+|B|-2*LCS and the
  similarity LCS/indel^2 (the two displayed equations of the same section),
  as exact integers and fractions.
* ``single_linkage`` -- single-linkage clustering ("Determination of the guide
  tree") by its plain definition: Kruskal's algorithm over all pairs, giving
  the merge heights and the cophenetic similarity of every pair.
* ``guide_tree`` -- the same clustering as a merge list (the guide tree).
* ``oracle.profile`` -- aligning one sequence to a profile ("Progressive
  construction of the alignment", "Gap types and costs determination"):
  column costs, gap-type rules and the affine-gap DP (``profile_dp.c``).
* ``oracle.gapped`` -- the gapped sequence representation ("Progressive
  construction of the alignment", Fig. 1) computed from explicit gapped
  strings.

Readings where the paper is silent: identical sequences (indel 0) have
similarity +infinity; an empty sequence has LCS 0 with anything.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "lcs_dp.c"), os.path.join(_HERE, "profile_dp.c")]
_LIB = os.path.join(_HERE, "liboracle_lcs.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile lcs_dp.c and profile_dp.c into liboracle_lcs.so with gcc (-O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_lcs.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64]
        lib.oracle_lcs.restype = ctypes.c_int32
        lib.oracle_lcs_pairs.argtypes = [u8p, u64p, ctypes.c_uint64, u64p, u64p, ctypes.c_uint64, i32p]
        lib.oracle_lcs_pairs.restype = ctypes.c_int
        lib.oracle_lcs_rows.argtypes = [u8p, u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, i32p]
        lib.oracle_lcs_rows.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_profile_dp.argtypes = [ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_uint32, i64p, i64p, i64p,
                                          i64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          i64p, u8p, ctypes.POINTER(ctypes.c_uint32)]
        lib.oracle_profile_dp.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def lcs(a: Sequence[int], b: Sequence[int]) -> int:
    """LCS length of two code sequences (DP rule, C implementation)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.uint8))
    # keep a valid pointer for empty inputs
    pa = a if a.size else np.zeros(1, np.uint8)
    pb = b if b.size else np.zeros(1, np.uint8)
    r = _load().oracle_lcs(_p(pa, ctypes.c_uint8), a.size, _p(pb, ctypes.c_uint8), b.size)
    if r < 0:
        raise MemoryError("oracle_lcs allocation failed")
    return int(r)


def lcs_pairs(codes: np.ndarray, seq_off: np.ndarray, ia: np.ndarray, ib: np.ndarray) -> np.ndarray:
    """LCS for pairs of sequences (global indices) of a concatenated batch."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    if codes.size == 0:
        codes = np.zeros(1, np.uint8)
    seq_off = np.ascontiguousarray(seq_off, dtype=np.uint64)
    ia = np.ascontiguousarray(ia, dtype=np.uint64)
    ib = np.ascontiguousarray(ib, dtype=np.uint64)
    out = np.zeros(ia.size, dtype=np.int32)
    if ia.size == 0:
        return out
    rc = _load().oracle_lcs_pairs(_p(codes, ctypes.c_uint8), _p(seq_off, ctypes.c_uint64), seq_off.size - 1,
                                  _p(ia, ctypes.c_uint64), _p(ib, ctypes.c_uint64), ia.size,
                                  _p(out, ctypes.c_int32))
    if rc != 0:
        raise ValueError("oracle_lcs_pairs: bad index or allocation failure")
    return out


def tile_count(k: int, r0: int, r1: int) -> int:
    """Values in rows [r0, r1) of the upper triangle of a k-family."""
    r1 = min(r1, k)
    return sum(k - 1 - i for i in range(r0, r1)) if r1 > r0 else 0


def tile_expected(codes, seq_off, fam_base: int, k: int, r0: int, r1: int) -> np.ndarray:
    """Rows [r0, r1) of a family: row i holds LCS(i, j), j = i+1..k-1, rows back to back."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    if codes.size == 0:
        codes = np.zeros(1, np.uint8)
    seq_off = np.ascontiguousarray(seq_off, dtype=np.uint64)
    out = np.zeros(tile_count(k, r0, r1), dtype=np.int32)
    if out.size == 0:
        return out
    rc = _load().oracle_lcs_rows(_p(codes, ctypes.c_uint8), _p(seq_off, ctypes.c_uint64), fam_base, k, r0, r1,
                                 _p(out, ctypes.c_int32))
    if rc != 0:
        raise MemoryError("oracle_lcs_rows failed")
    return out


def full_matrix(codes, seq_off, fam_base: int, k: int) -> np.ndarray:
    """Symmetric k x k LCS matrix of one family (diagonal = sequence length)."""
    tri = tile_expected(codes, seq_off, fam_base, k, 0, k)
    M = np.zeros((k, k), dtype=np.int64)
    p = 0
    for i in range(k):
        n = k - 1 - i
        M[i, i + 1:] = tri[p:p + n]
        p += n
    M = M + M.T
    L = np.diff(np.asarray(seq_off, dtype=np.int64))[fam_base:fam_base + k]
    M[np.arange(k), np.arange(k)] = L
    return M


# ------------------------------------------------------------- similarity

INF = float("inf")


def indel(L: int, m: int, n: int) -> int:
    """indel(A, B) = |A| + |B| - 2 * LCS_len(A, B)."""
    return m + n - 2 * L


def similarity(L: int, m: int, n: int):
    """similarity(A, B) = LCS_len / indel^2 as an exact Fraction; +inf when indel = 0."""
    d = indel(L, m, n)
    if d == 0:
        return INF
    return Fraction(L, d * d)


# ----------------------------------------------------------- single linkage

def single_linkage(lcs_mat: np.ndarray, lengths: Sequence[int]) -> Tuple[List, np.ndarray]:
    """Single linkage on similarities by Kruskal's algorithm over all pairs.

    Returns (merge heights sorted from the first merge to the last, as exact
    similarities) and the cophenetic similarity matrix (object array; the
    similarity at which i and j first share a cluster, +inf on the diagonal).
    Both are independent of how ties between equal similarities are broken.
    """
    k = lcs_mat.shape[0]
    edges = []
    for i in range(k):
        for j in range(i + 1, k):
            edges.append((similarity(int(lcs_mat[i, j]), int(lengths[i]), int(lengths[j])), i, j))
    # most similar first; ties in any order
    edges.sort(key=lambda e: e[0], reverse=True)
    parent = list(range(k))
    members = {i: [i] for i in range(k)}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    coph = np.empty((k, k), dtype=object)
    for i in range(k):
        coph[i, i] = INF
    heights = []
    for s, i, j in edges:
        ri, rj = find(i), find(j)
        if ri == rj:
            continue
        for x in members[ri]:
            for y in members[rj]:
                coph[x, y] = s
                coph[y, x] = s
        parent[rj] = ri
        members[ri] += members.pop(rj)
        heights.append(s)
    return heights, coph


def guide_tree(lcs_mat: np.ndarray, lengths: Sequence[int]) -> List[Tuple[int, int, object]]:
    """The single-linkage guide tree as a merge list (Methods, "Determination
    of the guide tree"), by Kruskal's algorithm over all pairs.

    Pairs are taken most similar first; equal similarities by the pair
    (i, j), i < j, in lexicographic order.  A pair whose ends lie in
    different clusters merges them: merge t joins the cluster holding i
    (left) and the cluster holding j (right) into cluster k + t; clusters
    0..k-1 are the sequences.  Returns [(left, right, similarity)].
    """
    k = lcs_mat.shape[0]
    edges = []
    for i in range(k):
        for j in range(i + 1, k):
            edges.append((similarity(int(lcs_mat[i, j]), int(lengths[i]), int(lengths[j])), i, j))
    edges.sort(key=lambda e: (-1, 0, e[1], e[2]) if e[0] == INF else (0, -e[0], e[1], e[2]))
    parent = list(range(k))
    cluster = list(range(k))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    merges = []
    for s, i, j in edges:
        ri, rj = find(i), find(j)
        if ri == rj:
            continue
        merges.append((cluster[ri], cluster[rj], s))
        parent[ri] = rj
        cluster[rj] = k + len(merges) - 1
    return merges
