"""Bit-exact parity of the HIP path with the CPU oracle on small inputs that
still span several groups, column chunks, tiles and every kernel class.
Every GPU result goes through the C-ABI (famsa_lcs_plan / famsa_lcs_tiles)."""
import ctypes

import numpy as np
import pytest

import oracle
from helpers import check_all_tiles, expected_tile
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu

EDGE_LENGTHS = [0, 1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 511, 512, 513, 767, 768, 769,
                1023, 1024, 1025, 1500, 2047, 2048, 2049, 2600]


def run(b, **opt):
    with B.Plan.from_batch(b, **opt) as p:
        return p.collect(), p.info(), p.stats()


def test_c1_full():
    b = inputs.c1()
    tiles, info, st = run(b)
    assert info.pairs == 4950
    check_all_tiles(b, tiles, 1024)


@pytest.mark.parametrize("flags", [B.NO_GRAPH, B.PLAIN, B.PLAIN | B.PLAIN_ASYNC, B.DESCENDING,
                                   B.NO_GRAPH | B.DESCENDING])
def test_c1_modes(flags):
    b = inputs.c1()
    tiles, _, _ = run(b, flags=flags, tile_rows=37)
    check_all_tiles(b, tiles, 37)


def edge_family(seed=0):
    rng = np.random.default_rng(seed)
    seqs = []
    for L in EDGE_LENGTHS:
        seqs.append(rng.integers(0, 20, L).astype(np.uint8))
    # homopolymers: carries ripple across every dword
    seqs += [np.full(L, 7, np.uint8) for L in (1, 33, 64, 65, 257, 1025, 2049)]
    # alternating / periodic / codes 19 and 0 only
    seqs += [np.tile(np.array([19, 0], np.uint8), 200), np.tile(np.arange(20, dtype=np.uint8), 30),
             np.tile(np.array([0, 0, 19], np.uint8), 90), np.full(129, 19, np.uint8), np.full(96, 0, np.uint8)]
    rng.shuffle(seqs)
    return inputs.from_sequences(seqs, name="edges")


def test_edge_lengths_family_mode():
    b = edge_family(1)
    tiles, info, _ = run(b)
    check_all_tiles(b, tiles, 1024)


@pytest.mark.parametrize("tile_rows", [1, 5, 64])
def test_edge_lengths_tile_mode(tile_rows):
    b = edge_family(2)
    # a step budget below the family's triangle forces tile mode
    tiles, info, _ = run(b, tile_rows=tile_rows, step_values=700)
    check_all_tiles(b, tiles, tile_rows)


def test_random_tile_mode_several_steps():
    b = inputs.random_family(300, 0, 700, 3)
    tiles, info, _ = run(b, tile_rows=70, step_values=20000, cols_per_item=16)
    assert info.nsteps >= 3
    check_all_tiles(b, tiles, 70)


@pytest.mark.parametrize("flags", [B.DESCENDING, B.DESCENDING | B.NO_GRAPH, B.TWO_STREAMS,
                                   B.TWO_STREAMS | B.NO_GRAPH | B.DESCENDING])
def test_tile_mode_several_tiles_per_step(flags):
    # steps of several tiles: the step's rows come first among the column
    # positions, in length order, so pairs of two step rows land in the
    # lower-indexed row's tile
    b = inputs.random_family(300, 0, 700, 14)
    tiles, info, _ = run(b, tile_rows=30, step_values=9000, flags=flags)
    assert info.nsteps >= 3 and info.nsteps < info.ntiles
    check_all_tiles(b, tiles, 30)


def test_multi_family_uneven():
    fams, sizes = [], []
    rng = np.random.default_rng(4)
    for k in [0, 1, 2, 3, 64, 65, 130, 7, 0, 200]:
        for _ in range(k):
            fams.append(rng.integers(0, 20, int(rng.integers(0, 400))).astype(np.uint8))
        sizes.append(k)
    b = inputs.from_sequences(fams, sizes)
    tiles, info, _ = run(b, tile_rows=50)
    assert info.nfam == 10
    check_all_tiles(b, tiles, 50)
    for flags in (B.PLAIN, B.PLAIN | B.PLAIN_ASYNC):
        tiles2, _, _ = run(b, tile_rows=50, flags=flags)
        assert tiles2.keys() == tiles.keys()
        for key in tiles:
            assert np.array_equal(tiles[key], tiles2[key])


@pytest.mark.parametrize("sigma", [1, 2, 32])
def test_alphabets(sigma):
    b = inputs.random_family(90, 0, 300, 5 + sigma, alphabet=sigma)
    tiles, _, _ = run(b, alphabet_size=sigma)
    check_all_tiles(b, tiles, 1024)


def test_sigma32_long_rows_segmented():
    # with 32 symbols the fast classes hold rows of at most 16 dwords; longer
    # rows go to the segmented long-row kernel on the GPU
    b = inputs.random_family(40, 600, 1400, 9, alphabet=32)
    tiles, _, st = run(b, alphabet_size=32, tile_rows=16)
    check_all_tiles(b, tiles, 16)
    assert st.cells[3] > 0


def test_cancel_resume_and_busy():
    b = inputs.random_family(150, 10, 200, 11)
    with B.Plan.from_batch(b, tile_rows=20, step_values=3000) as p:
        full = p.collect()
        seen = []

        def stop_at_3(t):
            seen.append(t.tile_index)
            return 1 if t.tile_index == 3 else 0

        with pytest.raises(B.FamsaError) as e:
            p.run(stop_at_3)
        assert e.value.code == B.ECANCELED and seen[-1] == 3
        # the plan still works, and resuming from tile 4 gives the same tiles
        part = p.collect(first_tile=4)
        order = sorted(full.keys(), key=lambda x: x[1])
        assert list(part.keys()) == order[4:]
        for key in part:
            assert np.array_equal(part[key], full[key])

        def reenter(t):
            rc = B.lib().famsa_lcs_tiles(p.handle, 0, B.TILE_FN(lambda u, tt: 0), None)
            assert rc == B.EBUSY
            return 0

        p.run(reenter)
        with pytest.raises(B.FamsaError):
            p.run(lambda t: 0, first_tile=10**6)


def test_device_tiles():
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    b = inputs.random_family(120, 0, 500, 12)
    got = {}
    with B.Plan.from_batch(b, flags=B.DEVICE_TILES, tile_rows=40) as p:
        def fn(t):
            a = np.zeros(t.count, np.int32)
            assert hip.hipStreamSynchronize(t.stream) == 0
            if t.count:
                assert hip.hipMemcpy(a.ctypes.data, ctypes.cast(t.lcs, ctypes.c_void_p), a.nbytes, 2) == 0
            got[(t.family, t.row_begin, t.row_end)] = a
            return 0
        p.run(fn)
    check_all_tiles(b, got, 40)


def test_torch_stream_and_repeat():
    torch = pytest.importorskip("torch")
    b = inputs.random_family(70, 20, 260, 13)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with B.Plan.from_batch(b, stream=B.torch_stream_handle()) as p:
            t1 = p.collect()
            t2 = p.collect()
    for key in t1:
        assert np.array_equal(t1[key], t2[key])
    check_all_tiles(b, t1, 1024)


def long_rows_family(seed, sigma, k, lo, hi):
    rng = np.random.default_rng(seed)
    lens = list(rng.integers(lo, hi + 1, k))
    lens[:6] = [hi, hi, lo, 897, 1791, 1792][:6]
    seqs = [rng.integers(0, sigma, int(L)).astype(np.uint8) for L in lens]
    seqs[5] = seqs[0].copy()                     # identical long rows
    seqs += [np.full(3000, sigma - 1, np.uint8), np.zeros(0, np.uint8), np.full(40, sigma - 1, np.uint8)]
    return inputs.from_sequences(seqs, name=f"long{sigma}")


@pytest.mark.parametrize("sigma,lo,hi", [(20, 800, 3100), (32, 400, 2100), (2, 850, 2000)])
@pytest.mark.parametrize("tile_rows", [1024, 7])
def test_long_rows_lanes_per_row_and_segmented(sigma, lo, hi, tile_rows):
    # rows longer than one lane holds: the lanes-per-row mode (default) and
    # the segmented kernel both give the oracle's values, in family mode and
    # tile mode
    b = long_rows_family(61 + sigma, sigma, 70, lo, hi)
    a = max(sigma, 2)
    t_lpr, _, st = run(b, alphabet_size=a, tile_rows=tile_rows)
    assert st.cells[3] > 0  # long rows ran in the long-row kernel
    check_all_tiles(b, t_lpr, tile_rows)
    t_seg, _, _ = run(b, alphabet_size=a, tile_rows=tile_rows, flags=B.LONG_SEGMENTED)
    assert t_seg.keys() == t_lpr.keys()
    assert all(np.array_equal(t_seg[key], t_lpr[key]) for key in t_lpr)


def test_long_rows_autotuned_word_width():
    # the tuner searches the long rows' word width per lane (and the
    # segmented kernel); whatever it picks, values equal the oracle's
    b = long_rows_family(70, 20, 90, 900, 2500)
    with B.Plan.from_batch(b, flags=B.NO_GRAPH) as p:
        p.autotune(None)
        tiles = p.collect()
    check_all_tiles(b, tiles, 1024)
