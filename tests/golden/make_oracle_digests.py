"""Write per-tile digests of the oracle's full LCS matrices for the c2 and c3
workloads (every value of every 1024-row tile), for the GPU test that checks
the HIP path against them value for value.

    python tests/golden/make_oracle_digests.py c2 c3 [--workers N]
    python tests/golden/make_oracle_digests.py c3 --families 25 --add


Only the oracle (oracle.tile_expected: the textbook DP, one pair at a time)
computes the values; the inputs come from the seeded generator.  A digest is
blake2b (16 bytes) over the tile's int32 values in tile order (row i holds
LCS(i, j), j = i+1..k-1, rows back to back), little-endian.

Families with more than MAX_FAMILY_CELLS all-pairs DP cells are left out (in
c3 the largest, 74% of its cells, which takes the oracle hours on a few
cores) unless named with --families; --add merges the new tiles into the
file already written.  The file lists the families it does not hold.
"""
import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1603_06958_amd import inputs  # noqa: E402

TILE_ROWS = 1024
CHUNK = 16  # rows per work unit
MAX_FAMILY_CELLS = 5e12


def _rows(args):
    name, f, r0, r1 = args
    b = _batch(name)
    a = int(b.fam_off[f])
    k = int(b.fam_off[f + 1]) - a
    return oracle.tile_expected(b.codes, b.seq_off, a, k, r0, r1)


_cache = {}


def _batch(name):
    if name not in _cache:
        _cache[name] = getattr(inputs, name)()
    return _cache[name]


def family_cells(b, f):
    a, e = int(b.fam_off[f]), int(b.fam_off[f + 1])
    lens = b.lengths()[a:e].astype(np.int64)
    return (int(lens.sum()) ** 2 - int((lens * lens).sum())) // 2


def digests(name, workers, families=None):
    b = _batch(name)
    units, tiles = [], []
    for f in range(b.nfam):
        if families is not None and f not in families:
            continue
        if families is None and family_cells(b, f) > MAX_FAMILY_CELLS:
            continue
        k = int(b.fam_off[f + 1] - b.fam_off[f])
        for t0 in range(0, k, TILE_ROWS):
            t1 = min(k, t0 + TILE_ROWS)
            tiles.append((f, t0, t1))
            for c0 in range(t0, t1, CHUNK):
                units.append((name, f, c0, min(t1, c0 + CHUNK)))
    # largest units first so the pool stays busy
    L = b.lengths()
    cost = {}
    for u in units:
        _, f, c0, c1 = u
        a = int(b.fam_off[f])
        k = int(b.fam_off[f + 1]) - a
        cost[u] = int(L[a + c0:a + c1].sum()) * int(L[a + c0:a + k].sum())
    order = sorted(units, key=lambda u: -cost[u])
    out = {}
    t0 = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        for n, (u, vals) in enumerate(zip(order, pool.imap(_rows, order, chunksize=1))):
            out[u] = vals
            if n % 500 == 0:
                print(f"{name}: {n}/{len(order)} units, {time.time() - t0:.0f} s", flush=True)
    lines = []
    for f, r0, r1 in tiles:
        parts = [out[(name, f, c0, min(r1, c0 + CHUNK))] for c0 in range(r0, r1, CHUNK)]
        v = np.concatenate(parts).astype("<i4") if parts else np.zeros(0, "<i4")
        lines.append(f"{f} {r0} {r1} {v.size} {hashlib.blake2b(v.tobytes(), digest_size=16).hexdigest()}")
    return lines


def read_lines(path):
    if not os.path.exists(path):
        return []
    return [ln.rstrip("\n") for ln in open(path) if ln.strip() and not ln.startswith("#")]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=["c2", "c3"])
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--families", type=int, nargs="+", help="only these families (whatever their size)")
    ap.add_argument("--add", action="store_true", help="merge into the file already written")
    a = ap.parse_args()
    oracle.build()
    for name in a.names:
        path = os.path.join(HERE, f"oracle_digests_{name}.txt")
        new = digests(name, a.workers, set(a.families) if a.families else None)
        have = {tuple(ln.split()[:3]): ln for ln in (read_lines(path) if a.add else [])}
        have.update({tuple(ln.split()[:3]): ln for ln in new})
        lines = [have[key] for key in sorted(have, key=lambda t: tuple(int(x) for x in t))]
        held = {int(ln.split()[0]) for ln in lines}
        b = _batch(name)
        skipped = [f for f in range(b.nfam) if f not in held and int(b.fam_off[f + 1] - b.fam_off[f]) > 1]
        with open(path, "w") as fh:
            fh.write(f"# oracle per-tile digests: {name}, generator version {inputs.GENERATOR_VERSION}, "
                     f"tile_rows {TILE_ROWS}\n# written by tests/golden/make_oracle_digests.py {name}\n"
                     f"# families left out (over {MAX_FAMILY_CELLS:.0e} cells): "
                     f"{' '.join(map(str, skipped)) or 'none'}\n"
                     "# family row_begin row_end values blake2b-128\n")
            fh.write("\n".join(lines) + "\n")
        print(f"wrote {path}: {len(lines)} tiles", flush=True)


if __name__ == "__main__":
    main()
