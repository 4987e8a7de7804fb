"""Shared helpers for GPU parity tests: expected tiles come only from the
oracle; sampled checks pick seeded positions inside delivered tiles."""
import numpy as np

import oracle


def tile_positions(k, r0, r1):
    """(i, j) of every value of rows [r0, r1) in tile order."""
    ii, jj = [], []
    for i in range(r0, min(r1, k)):
        n = k - 1 - i
        ii.append(np.full(n, i, np.int64))
        jj.append(np.arange(i + 1, k, dtype=np.int64))
    if not ii:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(ii), np.concatenate(jj)


def expected_tile(b, fam, r0, r1):
    a = int(b.fam_off[fam])
    k = int(b.fam_off[fam + 1]) - a
    return oracle.tile_expected(b.codes, b.seq_off, a, k, r0, r1)


def check_all_tiles(b, tiles, tile_rows):
    """Every tile of every family present and equal to the oracle."""
    nfam = b.nfam
    want = set()
    for f in range(nfam):
        k = int(b.fam_off[f + 1] - b.fam_off[f])
        for r0 in range(0, k, tile_rows):
            want.add((f, r0, min(k, r0 + tile_rows)))
    assert set(tiles.keys()) == want
    for (f, r0, r1), got in tiles.items():
        exp = expected_tile(b, f, r0, r1)
        if not np.array_equal(got, exp):
            bad = np.nonzero(got != exp)[0]
            k = int(b.fam_off[f + 1] - b.fam_off[f])
            ii, jj = tile_positions(k, r0, r1)
            p = bad[0]
            raise AssertionError(f"family {f} tile [{r0},{r1}): {bad.size} mismatches, first at ({ii[p]},{jj[p]}): "
                                 f"got {got[p]} want {exp[p]}")


def digest(a: np.ndarray) -> bytes:
    """128-bit digest of an array's bytes (xxh3 when available, else blake2b)."""
    try:
        import xxhash
        return xxhash.xxh3_128_digest(np.ascontiguousarray(a).view(np.uint8))
    except ImportError:
        import hashlib
        return hashlib.blake2b(np.ascontiguousarray(a).tobytes(), digest_size=16).digest()


class RowStream:
    """A family's values as one stream, whatever the tiles: tiles must come in
    row order and cover rows 0..k without gaps; the digest is that of the
    upper triangle row by row (row i holds LCS(i, j), j = i+1..k-1)."""

    def __init__(self, k):
        self.k = k
        self.next = 0
        self.tiles = 0
        try:
            import xxhash
            self.h = xxhash.xxh3_128()
        except ImportError:
            import hashlib
            self.h = hashlib.blake2b(digest_size=16)

    def feed(self, t):
        r0, r1 = int(t.row_begin), int(t.row_end)
        assert r0 == self.next and r1 > r0, f"tile [{r0},{r1}) after row {self.next}"
        import paper_1603_06958_amd.binding as B
        self.h.update(np.ascontiguousarray(B.tile_array(t)).view(np.uint8))
        self.next = r1
        self.tiles += 1

    def digest(self):
        assert self.next == self.k, f"rows up to {self.next} of {self.k}"
        return self.h.digest()


class Sampler:
    """Tile callback keeping `per_tile` seeded samples (and bound checks)."""

    def __init__(self, b, per_tile=64, seed=0, bound_check_every=1):
        self.b = b
        self.rng = np.random.default_rng(seed)
        self.per_tile = per_tile
        self.samples = []  # (global_i, global_j, value)
        self.L = b.lengths()
        self.every = bound_check_every
        self.ntiles = 0
        self.count = 0

    def __call__(self, t):
        from paper_1603_06958_amd.binding import tile_array
        vals = tile_array(t)
        f, k, r0, r1 = int(t.family), int(t.k), int(t.row_begin), int(t.row_end)
        base = int(self.b.fam_off[f])
        self.count += int(t.count)
        if t.count:
            pos = self.rng.integers(0, t.count, min(self.per_tile, int(t.count)))
            # locate rows by prefix
            rows = np.arange(r0, r1, dtype=np.int64)
            pref = np.concatenate([[0], np.cumsum(k - 1 - rows)])
            ri = np.searchsorted(pref, pos, side="right") - 1
            i = rows[ri]
            j = i + 1 + (pos - pref[ri])
            for a, c, v in zip(i, j, vals[pos]):
                self.samples.append((base + int(a), base + int(c), int(v)))
            if self.ntiles % self.every == 0:
                # 0 <= LCS <= min(|A_i|, |A_j|) over every value of the tile
                assert (vals >= 0).all(), "negative LCS"
                Lf = self.L[base:base + k]
                p = 0
                for i in range(r0, r1):
                    n = k - 1 - i
                    if n and (vals[p:p + n] > np.minimum(Lf[i], Lf[i + 1:])).any():
                        raise AssertionError(f"LCS above the shorter length in row {i} of family {f}")
                    p += n
        self.ntiles += 1
        return 0

    def check(self):
        s = np.array(self.samples, dtype=np.int64).reshape(-1, 3)
        exp = oracle.lcs_pairs(self.b.codes, self.b.seq_off, s[:, 0], s[:, 1])
        bad = np.nonzero(exp != s[:, 2])[0]
        assert bad.size == 0, f"{bad.size}/{len(s)} sampled mismatches, e.g. pair {s[bad[0], :2]}: " \
                              f"got {s[bad[0], 2]} want {exp[bad[0]]}"
        return len(s)
