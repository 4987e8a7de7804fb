"""famsa_lcs_family_noalloc (static device scratch, planning on the device,
no allocation) against famsa_lcs_plan + famsa_lcs_tiles on the same family:
every value equal, over calls in a row whose inputs shrink, at both alphabet
caps, at the sequence-count limit and on degenerate families; invalid input
gives status EINVAL and -1 in every slot, and the next valid call is exact
again; repeated calls take no device memory."""
import numpy as np
import pytest
import torch

import oracle
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def plan_values(b, sigma):
    k = b.nseq
    with B.Plan.from_batch(b, tile_rows=max(k, 1), alphabet_size=sigma) as p:
        tiles = p.collect()
    if k < 2:
        return np.zeros(0, np.int32)
    assert list(tiles) == [(0, 0, k)]
    return tiles[(0, 0, k)]


def noalloc_values(b, sigma, fill=-7):
    k = b.nseq
    n = k * (k - 1) // 2
    codes = torch.from_numpy(b.codes if b.codes.size else np.zeros(1, np.uint8)).to(DEV)
    off = torch.from_numpy(b.seq_off.astype(np.int64)).to(DEV)
    out = torch.full((max(n, 1),), fill, dtype=torch.int32, device=DEV)
    status = torch.full((1,), 99, dtype=torch.int32, device=DEV)
    print(f"noalloc k={k} sigma={sigma} residues={int(b.seq_off[-1])}", flush=True)
    B.family_noalloc(codes.data_ptr(), off.data_ptr(), k, out.data_ptr(), status.data_ptr(), alphabet_size=sigma,
                     stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:n], int(status.item())


def with_edge_rows(b, dup=(), empty=()):
    seqs = [b.seq(i).copy() for i in range(b.nseq)]
    for a, c in dup:
        seqs[a] = seqs[c].copy()
    for e in empty:
        seqs[e] = np.zeros(0, np.uint8)
    return inputs.from_sequences(seqs)


def check_equal(b, sigma, nsample=200, seed=0):
    got, st = noalloc_values(b, sigma)
    assert st == B.OK
    exp = plan_values(b, sigma)
    assert got.shape == exp.shape
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, f"{bad.size} values differ from the plan path, first at {bad[0]}"
    k = b.nseq
    if got.size:  # a few seeded values against the oracle as well
        rng = np.random.default_rng(seed)
        i = rng.integers(0, k - 1, nsample)
        j = np.array([rng.integers(a + 1, k) for a in i])
        pos = i * k - i * (i + 1) // 2 + (j - i - 1)
        assert np.array_equal(oracle.lcs_pairs(b.codes, b.seq_off, i, j), got[pos].astype(np.int64))
    return got


def test_two_calls_in_a_row_second_smaller():
    # first: 2000 rows over all three fast classes (lengths 0..896), ragged
    # last group, equal and empty rows; second: a smaller family that reuses
    # the scratch the first call left behind
    big = with_edge_rows(inputs.random_family(2000, 0, B.NOALLOC_MAX_LEN, seed=71), dup=((5, 9), (1999, 9)),
                         empty=(3, 1000))
    check_equal(big, 20, seed=1)
    small = with_edge_rows(inputs.random_family(300, 0, 400, seed=72), dup=((0, 299),), empty=(150,))
    check_equal(small, 20, seed=2)


def test_alphabet_32_and_small_alphabets():
    check_equal(inputs.random_family(700, 0, B.NOALLOC_MAX_LEN_S32, seed=73, alphabet=32), 32, seed=3)
    check_equal(inputs.random_family(257, 1, 300, seed=74, alphabet=2), 2, seed=4)
    check_equal(inputs.random_family(65, 30, 40, seed=75, alphabet=1), 1, seed=5)


def test_degenerate_families():
    for k in (0, 1):
        got, st = noalloc_values(inputs.random_family(k, 0, 10, seed=76), 20)
        assert st == B.OK and got.size == 0
    check_equal(inputs.random_family(2, 5, 9, seed=77), 20, nsample=4)
    check_equal(inputs.from_sequences([np.zeros(0, np.uint8)] * 70), 20, nsample=10)
    check_equal(inputs.random_family(64, 896, 896, seed=78), 20, nsample=50)


def test_sequence_count_limit():
    b = inputs.random_family(B.NOALLOC_MAX_SEQ, 0, 48, seed=79)
    check_equal(b, 20, nsample=300, seed=6)


def test_invalid_input_sets_status_and_next_call_recovers():
    b = inputs.random_family(120, 10, 60, seed=80)
    bad_code = inputs.from_sequences([b.seq(i) for i in range(b.nseq)])
    bad_code.codes[77] = 20  # outside the 20-letter alphabet
    got, st = noalloc_values(bad_code, 20)
    assert st == B.EINVAL and (got == -1).all()
    long = inputs.random_family(50, 10, 60, seed=81)
    seqs = [long.seq(i) for i in range(50)]
    seqs[17] = np.zeros(B.NOALLOC_MAX_LEN + 1, np.uint8)
    got, st = noalloc_values(inputs.from_sequences(seqs), 20)
    assert st == B.EINVAL and (got == -1).all()
    seqs[17] = np.zeros(B.NOALLOC_MAX_LEN_S32 + 1, np.uint8)
    got, st = noalloc_values(inputs.from_sequences(seqs), 32)
    assert st == B.EINVAL and (got == -1).all()
    check_equal(b, 20, seed=7)


def test_host_side_rejections():
    with pytest.raises(B.FamsaError) as e:
        B.family_noalloc(1, 1, B.NOALLOC_MAX_SEQ + 1, 1, None)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.FamsaError) as e:
        B.family_noalloc(1, 1, 10, 1, None, alphabet_size=33)
    assert e.value.code == B.EINVAL


def test_repeated_calls_take_no_device_memory():
    b = inputs.random_family(1500, 0, 500, seed=82)
    noalloc_values(b, 20)  # the first call on the device may load the library's code objects
    codes = torch.from_numpy(b.codes).to(DEV)
    off = torch.from_numpy(b.seq_off.astype(np.int64)).to(DEV)
    out = torch.empty(b.nseq * (b.nseq - 1) // 2, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for _ in range(3):
        B.family_noalloc(codes.data_ptr(), off.data_ptr(), b.nseq, out.data_ptr(), None,
                         stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(0)[0] == free0
    assert np.array_equal(out.cpu().numpy(), plan_values(b, 20))
