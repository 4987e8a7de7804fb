"""The gapped-representation oracle (oracle/gapped.py) against the numbers the
paper prints in Fig. 1 (tests/golden/gapped_fig1.txt) and against invariants
that hold for any gapped string."""
import os

import numpy as np
import pytest

from oracle import gapped as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gapped_fig1.txt")


def fig1():
    d = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        d[key] = vals
    alphabet = d["alphabet"][0]
    g = [G.GUARD] + [None if ch == "-" else alphabet.index(ch) for ch in d["gapped"][0]]
    return alphabet, g, d


def test_fig1_counters_and_tree():
    alphabet, g, d = fig1()
    assert G.render(g, alphabet) == d["gapped"][0]
    assert "".join(alphabet[c] for c in G.symbols(g)) == "CAHFQGACDLMFAPS"
    assert G.no_gaps(g) == [int(x) for x in d["no_gaps"]]
    t = G.dps(g)
    assert len(t) == 16
    assert t[1] == int(d["dps1"][0])
    assert t[2:4] == [int(x) for x in d["dps2_3"]]
    assert t[4:8] == [int(x) for x in d["dps4_7"]]
    assert t[8:16] == [int(x) for x in d["dps8_15"]]


def test_fig1_from_ungapped_by_runs():
    # the counters say where the gaps go: no_gaps[i] columns right after
    # position i, i.e. before column i + 1 of the ungapped string
    alphabet, g, d = fig1()
    ng = [int(x) for x in d["no_gaps"]]
    plain = G.from_symbols(G.symbols(g))
    runs = [(i + 1, n) for i, n in enumerate(ng) if n]
    assert G.insert_runs(plain, runs) == g


def random_gapped(rng, n, max_run=4):
    g = G.from_symbols(rng.integers(0, 20, n).tolist())
    out = [g[0]]
    for c in g[1:] + [None]:
        out += [None] * int(rng.integers(0, max_run + 1)) * int(rng.random() < 0.5)
        if c is not None:
            out.append(c)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_tree_rule_and_totals(seed):
    rng = np.random.default_rng(seed)
    for n in [0, 1, 2, 3, 7, 15, 16, 31, 100]:
        g = random_gapped(rng, n)
        t = G.dps(g)
        P = len(t)
        assert P >= 2 and P & (P - 1) == 0 and P >= n + 1 and (P == 2 or P // 2 < n + 1)
        for v in range(1, P // 2):
            assert t[v] == t[2 * v] + t[2 * v + 1]  # the figure's rule
        assert t[1] == len(g)
        assert sum(G.spans(g)) == len(g)
        assert len(G.no_gaps(g)) == n + 1


@pytest.mark.parametrize("seed", range(6))
def test_locate_and_insert(seed):
    rng = np.random.default_rng(100 + seed)
    g = random_gapped(rng, int(rng.integers(0, 60)))
    sp = G.spans(g)
    starts = np.concatenate([[0], np.cumsum(sp)[:-1]])
    for col in range(len(g)):
        p = G.locate(g, col)
        assert starts[p] <= col < starts[p] + sp[p]
    runs = sorted((int(rng.integers(1, len(g) + 1)), int(rng.integers(0, 5))) for _ in range(8))
    h = G.insert_runs(g, runs)
    assert G.symbols(h) == G.symbols(g)
    assert len(h) == len(g) + sum(n for _, n in runs)
    # the symbol at column c moves right by the gaps inserted at or before c
    for col in range(1, len(g)):
        if g[col] is not None:
            shift = sum(n for c, n in runs if c <= col)
            assert h[col + shift] == g[col]
