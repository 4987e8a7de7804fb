"""Parity at the length limit (FAMSA_LCS_MAX_LEN = 65535 residues): rows of
2048 dwords go through the segmented long-row kernel, whose per-wave carry
scratch is sized by the longest column; every value of every tile equals the
oracle's, in family mode and in tile mode, at alphabets 20 and 32."""
import numpy as np
import pytest

from helpers import check_all_tiles
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def family20():
    rng = np.random.default_rng(90)
    a = rng.integers(0, 20, B.MAX_LEN).astype(np.uint8)
    b = a.copy()
    hit = rng.random(b.size) < 0.1  # a close relative: long runs of carries
    b[hit] = rng.integers(0, 20, int(hit.sum()))
    seqs = [a, b] + [rng.integers(0, 20, L).astype(np.uint8) for L in (16384, 4096, 4097, 897, 896, 33, 1, 0)]
    return inputs.from_sequences(seqs, name="maxlen20")


def family32():
    rng = np.random.default_rng(91)
    seqs = [np.full(B.MAX_LEN, 31, np.uint8)]  # homopolymer: the carry ripples through all 2048 dwords
    seqs += [rng.integers(0, 32, L).astype(np.uint8) for L in (40000, 8192, 513, 512, 0)]
    return inputs.from_sequences(seqs, name="maxlen32")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("make,sigma", [(family20, 20), (family32, 32)])
@pytest.mark.parametrize("tile_rows", [1024, 3])
def test_max_length_against_oracle(make, sigma, tile_rows):
    b = make()
    print(f"{b.name}: tile_rows {tile_rows}, lengths {b.lengths().tolist()}", flush=True)
    with B.Plan.from_batch(b, alphabet_size=sigma, tile_rows=tile_rows) as p:
        tiles = p.collect()
    check_all_tiles(b, tiles, tile_rows)
