"""Aligning one sequence to a profile -- TEST INFRASTRUCTURE (see oracle/__init__.py).

FAMSA, Methods, "Progressive construction of the alignment" and "Gap types
and costs determination".  A profile is held here as its K gapped rows of
equal width n (symbol codes, GAP for a gap).  Everything the alignment
needs is derived from the rows by definition:

* ``column_costs`` -- the profile's table of column-to-symbol costs: the
  score of aligning symbol a to column j is the sum, over the rows with a
  residue x in column j, of S[x][a] (the profile score sums the scores of
  every sequence pair; gaps already in the profile add nothing), and w_j,
  the number of rows with a residue in column j.
* ``insertion_costs`` -- the cost of inserting a run of gap columns into the
  profile at boundary p (after column p, 0 <= p <= n).  Every row gets a gap
  there, and its type follows the six situations the paper lists: a row
  with no residue on one side of p is in a terminal region, otherwise
  inside; if one of its columns next to p is already a gap, the inserted gap
  joins that series (an insertion in front of an opening gap makes the
  inserted gap the opening one and turns the old one into an extension: the
  same net cost), else it opens one.  So the first inserted column costs a
  row Te (terminal, next to a gap), To (terminal, opening), Ge (inside, next
  to a gap) or Go (inside, opening), and every further column of the run Te
  (terminal) or Ge (inside).
* gaps inserted into the sequence: a run of D columns is terminal when it
  lies before the sequence's first residue or after its last, and column j
  of it costs w_j times the open cost (first column of the run) or the
  extension cost (the others): the pairs with the rows that have a residue
  there.
* ``gap_scale`` -- the scaling of every gap cost by the family size,
  1 + ln(k / g_l) / g_d with g_l = 45 and g_d = 7 by default; the paper
  writes "log" and this reads it as the natural logarithm.
  ``scaled_gap_costs`` rounds the scaled costs to integers (half away from
  zero), the form the DP takes.

``align`` runs the DP of profile_dp.c over those numbers; ``alignment_score``
scores any given alignment directly from the rows, without the DP, and is
what the brute-force pin maximises.
"""
from __future__ import annotations

import ctypes
import math
from typing import List, Sequence, Tuple

import numpy as np

from . import _load, _p

GAP = 0xFF
OP_M, OP_D, OP_I = 0, 1, 2


def gap_scale(k: int, gl: float = 45.0, gd: float = 7.0) -> float:
    """g_scale = 1 + ln(k / g_l) / g_d."""
    return 1.0 + math.log(k / gl) / gd


def scaled_gap_costs(k: int, base: Sequence[float], gl: float = 45.0, gd: float = 7.0) -> Tuple[int, ...]:
    """(To, Te, Go, Ge) times g_scale, rounded half away from zero."""
    g = gap_scale(k, gl, gd)
    out = []
    for c in base:
        x = float(c) * g
        out.append(int(math.floor(abs(x) + 0.5)) * (1 if x >= 0 else -1))
    return tuple(out)


def _rows(rows) -> np.ndarray:
    r = np.asarray(rows, dtype=np.uint8)
    if r.ndim != 2 or r.shape[0] < 1:
        raise ValueError("a profile is K >= 1 rows of equal width")
    return r


def column_costs(rows, S: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """cost[j-1][a] and w[j-1] for columns j = 1..n (int64)."""
    r = _rows(rows)
    S = np.asarray(S, dtype=np.int64)
    sigma = S.shape[0]
    K, n = r.shape
    cost = np.zeros((n, sigma), dtype=np.int64)
    w = np.zeros(n, dtype=np.int64)
    for j in range(n):
        for s in range(K):
            x = int(r[s, j])
            if x != GAP:
                cost[j, :] += S[x, :]
                w[j] += 1
    return cost, w


def _row_first_ext(row: np.ndarray, p: int, To: int, Te: int, Go: int, Ge: int) -> Tuple[int, int]:
    """Cost of the first and of each further gap column inserted into one
    profile row at boundary p (after its column p)."""
    n = row.size
    left_res = any(int(row[c]) != GAP for c in range(0, p))
    right_res = any(int(row[c]) != GAP for c in range(p, n))
    gap_left = p >= 1 and int(row[p - 1]) == GAP
    gap_right = p < n and int(row[p]) == GAP
    adjacent_gap = gap_left or gap_right
    if not (left_res and right_res):  # terminal region of this row
        return (Te if adjacent_gap else To), Te
    return (Ge if adjacent_gap else Go), Ge


def insertion_costs(rows, To: int, Te: int, Go: int, Ge: int) -> Tuple[np.ndarray, np.ndarray]:
    """ifirst[p], iext[p] for boundaries p = 0..n, summed over the rows (int64)."""
    r = _rows(rows)
    K, n = r.shape
    first = np.zeros(n + 1, dtype=np.int64)
    ext = np.zeros(n + 1, dtype=np.int64)
    for p in range(n + 1):
        for s in range(K):
            f, e = _row_first_ext(r[s], p, To, Te, Go, Ge)
            first[p] += f
            ext[p] += e
    return first, ext


def align(seq, rows, S, costs) -> Tuple[int, List[int]]:
    """Optimal score and alignment (ops OP_M / OP_D / OP_I from the first
    column) of sequence `seq` against the profile `rows`."""
    To, Te, Go, Ge = (int(c) for c in costs)
    r = _rows(rows)
    a = np.ascontiguousarray(np.asarray(seq, dtype=np.uint8))
    S = np.asarray(S, dtype=np.int64)
    sigma = S.shape[0]
    if a.size and int(a.max()) >= sigma:
        raise ValueError("sequence code outside the substitution matrix")
    cost, w = column_costs(r, S)
    first, ext = insertion_costs(r, To, Te, Go, Ge)
    m, n = a.size, r.shape[1]
    cost = np.ascontiguousarray(cost.reshape(-1) if cost.size else np.zeros(1, np.int64))
    w = np.ascontiguousarray(w if w.size else np.zeros(1, np.int64))
    ops = np.zeros(max(1, m + n), dtype=np.uint8)
    score = ctypes.c_int64()
    nops = ctypes.c_uint32()
    pa = a if a.size else np.zeros(1, np.uint8)
    rc = _load().oracle_profile_dp(m, _p(pa, ctypes.c_uint8), n, sigma, _p(cost, ctypes.c_int64),
                                   _p(w, ctypes.c_int64), _p(first, ctypes.c_int64), _p(ext, ctypes.c_int64),
                                   To, Te, Go, Ge, ctypes.byref(score), _p(ops, ctypes.c_uint8), ctypes.byref(nops))
    if rc != 0:
        raise MemoryError("oracle_profile_dp failed")
    return int(score.value), ops[:nops.value].tolist()


def alignment_score(seq, rows, S, costs, ops: Sequence[int]) -> int:
    """Score of one given alignment, computed from the rows directly: the
    residue-to-column scores, the gap runs inserted into the sequence, and
    the gap runs inserted into the profile, each by the rules above."""
    To, Te, Go, Ge = (int(c) for c in costs)
    r = _rows(rows)
    S = np.asarray(S, dtype=np.int64)
    K, n = r.shape
    a = [int(x) for x in seq]
    m = len(a)
    if sum(1 for o in ops if o != OP_D) != m or sum(1 for o in ops if o != OP_I) != n:
        raise ValueError("the alignment does not use every residue and column once")
    total = 0
    i = j = 0
    t = 0
    while t < len(ops):
        o = ops[t]
        if o == OP_M:
            total += sum(int(S[int(r[s, j]), a[i]]) for s in range(K) if int(r[s, j]) != GAP)
            i += 1
            j += 1
            t += 1
            continue
        u = t
        while u < len(ops) and ops[u] == o:
            u += 1
        run = u - t
        if o == OP_D:  # columns j..j+run-1 against gaps in the sequence, after residue i
            terminal = i == 0 or i == m
            for q in range(run):
                c = (To if q == 0 else Te) if terminal else (Go if q == 0 else Ge)
                total -= c * sum(1 for s in range(K) if int(r[s, j + q]) != GAP)
            j += run
        else:  # residues i..i+run-1 against new gap columns at boundary j
            for s in range(K):
                f, e = _row_first_ext(r[s], j, To, Te, Go, Ge)
                total -= f + (run - 1) * e
            i += run
        t = u
    return total


def gap_runs(ops: Sequence[int]) -> Tuple[List[Tuple[int, int]], List[Tuple[int, int]]]:
    """The alignment as gap runs for the gapped representation: runs into the
    sequence ((column before which, length), columns of the ungapped
    sequence, 1-based) and runs into the profile (same, profile columns)."""
    seq_runs: List[Tuple[int, int]] = []
    prof_runs: List[Tuple[int, int]] = []
    i = j = 0
    t = 0
    while t < len(ops):
        o = ops[t]
        if o == OP_M:
            i += 1
            j += 1
            t += 1
            continue
        u = t
        while u < len(ops) and ops[u] == o:
            u += 1
        if o == OP_D:
            seq_runs.append((i + 1, u - t))
            j += u - t
        else:
            prof_runs.append((j + 1, u - t))
            i += u - t
        t = u
    return seq_runs, prof_runs
