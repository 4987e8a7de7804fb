"""Gapped sequence representation -- TEST INFRASTRUCTURE (see oracle/__init__.py).

Methods, "Progressive construction of the alignment", and Fig. 1: a gapped
sequence is kept as its symbols (a guard in front, at index 0), a gap
counter per symbol, and a tree of column counts ("dynamic position
statistics", dps) for locating columns and inserting gaps quickly.

This module works on the explicit gapped string: a Python list with one
entry per column, a symbol code or None for a gap, the guard included as
column 0.  Everything below is computed from that list by definition:

* ``no_gaps[i]``  -- gap columns right after symbol i (before symbol i+1);
  i = 0 is the guard, so no_gaps[0] counts leading gaps.  This follows the
  figure's printed numbers (its caption places the counters after the
  symbols; the text says "before the corresponding symbol").
* ``dps``          -- with P = the number of positions (guard + symbols)
  rounded up to a power of two (at least 2), dps[P/2 + j] is the number of
  columns spanned by positions 2j and 2j+1 (each position: its symbol column
  plus its gap run; positions past the end span nothing), and every other
  dps[v], 1 <= v < P/2, is the number of columns spanned by the positions
  under v, i.e. positions [v * 2^h - P ... ) in heap order.  dps[0] is unused.
  (The figure's rule dps[v] = dps[2v] + dps[2v+1] is a consequence, which
  the tests check separately.)
* ``insert_runs`` -- put ``count`` gap columns before column ``col`` (current
  coordinates, 1 <= col <= number of columns), for each run; runs refer to
  the columns before any of them is applied.
* ``locate(col)`` -- the position whose span holds column col.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

GUARD = -1  # the guard's code in an explicit gapped string


def from_symbols(codes: Sequence[int]) -> List[Optional[int]]:
    return [GUARD] + [int(c) for c in codes]


def insert_runs(g: List[Optional[int]], runs: Sequence[Tuple[int, int]]) -> List[Optional[int]]:
    """Insert gap runs (col, count); every col refers to the string before this call."""
    width = len(g)
    for col, count in runs:
        if not (1 <= col <= width) or count < 0:
            raise ValueError("run outside the sequence")
    out = list(g)
    # apply from the rightmost column so earlier columns keep their meaning;
    # runs at the same column all land there (their order does not matter)
    for col, count in sorted(runs, key=lambda r: -r[0]):
        out[col:col] = [None] * count
    return out


def symbols(g: Sequence[Optional[int]]) -> List[int]:
    return [c for c in g[1:] if c is not None]


def no_gaps(g: Sequence[Optional[int]]) -> List[int]:
    counts = []
    for c in g:
        if c is None:
            counts[-1] += 1
        else:
            counts.append(0)
    return counts


def spans(g: Sequence[Optional[int]]) -> List[int]:
    """Columns spanned by each position: its symbol plus the gaps after it."""
    return [1 + n for n in no_gaps(g)]


def dps(g: Sequence[Optional[int]]) -> List[int]:
    sp = spans(g)
    npos = len(sp)
    P = 2
    while P < npos:
        P *= 2
    sp = sp + [0] * (P - npos)
    tree = [0] * P
    for v in range(1, P):
        # node v covers the positions of its leaves: leaf P/2 + j covers 2j, 2j+1
        lo, hi = v, v + 1
        while lo < P // 2:
            lo, hi = 2 * lo, 2 * hi
        tree[v] = sum(sp[2 * (lo - P // 2):2 * (hi - P // 2)])
    return tree


def locate(g: Sequence[Optional[int]], col: int) -> int:
    """The position (0 = guard) whose span holds column col."""
    pos = -1
    for c in g[:col + 1]:
        if c is not None:
            pos += 1
    return pos


def render(g: Sequence[Optional[int]], alphabet: str) -> str:
    """The string as printed in the paper's figure caption: '-' for gaps, no guard."""
    return "".join("-" if c is None else alphabet[c] for c in g[1:])
