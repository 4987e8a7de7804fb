"""Host-side work decomposition, checked on the CPU through the dry-run entry
point: emulating the kernels' index arithmetic over the dumped work lists,
every value of every tile must be written exactly once, with the pair the
tile layout puts there (row i holds LCS(i, j), j = i+1..k-1)."""
import numpy as np
import pytest

from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs
from workdump import check_coverage, dry_run


def edge_family(seed):
    rng = np.random.default_rng(seed)
    lens = [0, 1, 31, 32, 33, 64, 255, 256, 257, 512, 513, 992, 993, 1024, 1025, 2600] * 2
    return inputs.from_sequences([rng.integers(0, 20, L).astype(np.uint8) for L in lens])


CASES = {
    "c1": (lambda: inputs.c1(), {}),
    "c1_desc_tiles": (lambda: inputs.c1(), dict(tile_rows=7, flags=B.DESCENDING)),
    "c1_plain": (lambda: inputs.c1(), dict(tile_rows=13, flags=B.PLAIN)),
    "edges_family": (lambda: edge_family(1), {}),
    "edges_tile5": (lambda: edge_family(2), dict(tile_rows=5, step_values=200)),
    "edges_tile1": (lambda: edge_family(3), dict(tile_rows=1, step_values=50)),
    "sigma32": (lambda: inputs.random_family(50, 0, 900, 4, alphabet=32), dict(alphabet_size=32, tile_rows=9)),
    "small_cols": (lambda: inputs.random_family(300, 0, 500, 5), dict(tile_rows=64, step_values=9000,
                                                                      cols_per_item=16)),
    "desc_steps": (lambda: inputs.random_family(300, 0, 500, 7), dict(tile_rows=20, step_values=9000,
                                                                      flags=B.DESCENDING)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_coverage(name):
    make, opt = CASES[name]
    b = make()
    d, info = dry_run(b, **opt)
    assert info.pairs == b.pairs()
    assert info.cells == b.cells()
    check_coverage(d)


def test_multi_family_coverage_and_whole_families():
    rng = np.random.default_rng(6)
    seqs, sizes = [], []
    for k in [0, 1, 2, 3, 64, 65, 130, 7, 0, 200]:
        seqs += [rng.integers(0, 20, int(rng.integers(0, 400))).astype(np.uint8) for _ in range(k)]
        sizes.append(k)
    b = inputs.from_sequences(seqs, sizes)
    for opt in [dict(tile_rows=50), dict(tile_rows=50, step_values=5000), dict(tile_rows=3, step_values=100)]:
        d, info = dry_run(b, **opt)
        check_coverage(d)
        # a family whose triangle fits one step keeps all its tiles in that step
        sv = opt.get("step_values", 1 << 27)
        for f in range(b.nfam):
            k = int(b.fam_off[f + 1] - b.fam_off[f])
            steps = set(int(t["step"]) for t in d["tiles"] if t["fam"] == f)
            if k * (k - 1) // 2 <= sv and k:
                assert len(steps) == 1


def test_dry_run_validates():
    with pytest.raises(B.FamsaError):
        dry_run(inputs.from_sequences([np.array([25], np.uint8)]))


@pytest.mark.parametrize("opt", [dict(tile_rows=20, step_values=9000), dict(tile_rows=20, step_values=9000,
                                                                          flags=B.DESCENDING),
                                 dict(tile_rows=7, step_values=3000, cols_per_item=16)])
def test_tile_mode_walks_no_column_below_its_rows(opt):
    # Several tiles per step: every group starts at the column position after
    # its first row, its rows hold consecutive positions, and the only columns
    # it walks without storing are those of its own 64 x 64 corner.
    b = inputs.random_family(300, 0, 500, 8)
    d, info = dry_run(b, **opt)
    check_coverage(d)
    assert len(d["steps"]) > 2 and (d["steps"]["tile_end"] - d["steps"]["tile_begin"]).max() > 1
    G, L, I = d["groups"], d["lanes"], d["items"]
    first_c0 = {}
    for it in I:
        first_c0[int(it["group"])] = min(first_c0.get(int(it["group"]), 1 << 32), int(it["c0"]))
    for gi, g in enumerate(G):
        assert g["colmap_base"] != 0xFFFFFFFF  # the step's rows are one range: columns are mapped
        pos = L[g["lane_first"]:g["lane_first"] + g["nrows"]]["pos"].astype(np.int64)
        assert np.array_equal(pos, pos[0] + np.arange(g["nrows"]))
        assert first_c0[gi] == pos[0] + 1


@pytest.mark.parametrize("name,sigma,wlmax", [("edges_family", 20, 28), ("edges_tile5", 20, 28), ("sigma32", 32, 16)])
def test_lanes_per_row_groups(name, sigma, wlmax):
    # long rows spread over several lanes: the rows of a group and their
    # lanes fit one wave, each lane holds between 8 and the LDS limit of
    # dwords, the group's widest row fits its lanes, and such groups exist
    make, opt = CASES[name]
    b = make()
    d, _ = dry_run(b, **opt)
    g = d["groups"]
    skew = g[g["lpr"] > 0]
    assert len(skew) > 0
    L = skew["lpr"].astype(np.int64)
    wl = (skew["W"].astype(np.int64) + L - 1) // L
    assert (skew["nrows"] * L <= 64).all()
    assert ((wl >= 8) & (wl <= wlmax)).all()
    assert (wl * L >= skew["W"]).all()
    lens = b.lengths()
    for gr in skew:
        ln = d["lanes"][gr["lane_first"]:gr["lane_first"] + gr["nrows"]]
        assert ((lens[ln["seq"]] + 31) // 32 <= gr["W"]).all()
