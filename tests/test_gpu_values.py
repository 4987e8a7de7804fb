"""Tiles of indel distances or float32 similarities instead of LCS values
(FAMSA_LCS_OUT_INDEL / FAMSA_LCS_OUT_SIM): every value equals the one
derived from the oracle's LCS by the paper's definitions (indel = |A| + |B|
- 2 LCS; similarity = LCS / indel^2, here the float32 rounding of the
correctly rounded double, +inf for indel 0), bit for bit, in every kernel
class and mode.  The single-linkage consumers refuse such tiles."""
import numpy as np
import pytest

from helpers import expected_tile
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs
from test_gpu_parity import edge_family

pytestmark = pytest.mark.gpu


def derived(b, fam, r0, r1, kind):
    L = expected_tile(b, fam, r0, r1).astype(np.int64)
    base = int(b.fam_off[fam])
    k = int(b.fam_off[fam + 1]) - base
    lens = b.lengths().astype(np.int64)[base:base + k]
    ii = np.concatenate([np.full(k - 1 - i, i) for i in range(r0, r1)]) if r1 > r0 else np.zeros(0, np.int64)
    jj = np.concatenate([np.arange(i + 1, k) for i in range(r0, r1)]) if r1 > r0 else np.zeros(0, np.int64)
    d = lens[ii] + lens[jj] - 2 * L
    if kind == B.OUT_INDEL:
        return d.astype(np.int32)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (L.astype(np.float64) / (d.astype(np.float64) ** 2)).astype(np.float32)
    s[d == 0] = np.float32(np.inf)
    return s


def check_values(b, tiles, kind):
    assert tiles
    for (fam, r0, r1), got in tiles.items():
        want = derived(b, fam, r0, r1, kind)
        assert got.dtype == want.dtype
        bad = np.nonzero(got.view(np.uint32) != want.view(np.uint32))[0]
        assert bad.size == 0, f"family {fam} tile [{r0},{r1}): {bad.size} mismatches, first {got[bad[0]]} vs {want[bad[0]]}"


CASES = {
    "c1": (lambda: inputs.c1(), {}),
    "edges_family": (lambda: edge_family(3), {}),
    "edges_tiles": (lambda: edge_family(4), dict(tile_rows=5, step_values=700)),
    "sigma32_long": (lambda: inputs.random_family(40, 600, 1400, 9, alphabet=32), dict(alphabet_size=32, tile_rows=16)),
    "plain": (lambda: inputs.random_family(60, 0, 300, 14), dict(flags=B.PLAIN, tile_rows=25)),
    "multi": (lambda: inputs.from_sequences([np.full(n % 37, n % 20, np.uint8) for n in range(90)], [30, 0, 60]),
              dict(tile_rows=11, flags=B.NO_GRAPH)),
}


@pytest.mark.parametrize("kind", [B.OUT_INDEL, B.OUT_SIM])
@pytest.mark.parametrize("case", sorted(CASES))
def test_values_match_definitions(case, kind):
    make, opt = CASES[case]
    b = make()
    opt = dict(opt)
    flags = opt.pop("flags", 0) | kind
    with B.Plan.from_batch(b, flags=flags, **opt) as p:
        tiles = p.collect()
    check_values(b, tiles, kind)


def test_consumers_refuse_non_lcs_tiles():
    b = inputs.random_family(50, 10, 200, 15)
    s = B.SLink(b.lengths())
    with B.Plan.from_batch(b, flags=B.DESCENDING | B.OUT_INDEL) as p:
        with pytest.raises(B.FamsaError) as e:
            p.run_native(B.SLink.consume_fn(), s.handle)
        assert e.value.code == B.ECANCELED
    s.close()
    m = B.Mst(b.lengths())
    with B.Plan.from_batch(b, flags=B.DEVICE_TILES | B.OUT_SIM) as p:
        with pytest.raises(B.FamsaError) as e:
            p.run_native(B.Mst.consume_fn(), m.handle)
        assert e.value.code == B.ECANCELED
    m.close()
