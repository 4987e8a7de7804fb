"""Aligning one sequence to a profile on the GPU (famsa_profile_align)
against the oracle (oracle/profile.py: column costs, gap-type rules and the
affine-gap DP derived from the gapped rows): the same optimal score and the
same alignment, op for op, under the fixed tie rule; and the GPU alignment's
score recomputed from the rows equals the GPU score."""
import numpy as np
import pytest

from oracle import profile as OP
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def check_batch(problems, S, costs, sigma=None):
    print(f"profile batch: {len(problems)} problems, sigma {S.shape[0]}", flush=True)
    got_s, got_ops = B.profile_align([(p.seq, p.rows) for p in problems], S, costs, alphabet_size=sigma)
    for q, p in enumerate(problems):
        exp_s, exp_ops = OP.align(p.seq, p.rows, S, costs)
        assert int(got_s[q]) == exp_s, f"problem {q} (m={p.seq.size}, K,n={p.rows.shape}): score {got_s[q]} != {exp_s}"
        assert got_ops[q].tolist() == exp_ops, f"problem {q}: alignment differs from the oracle's"
        assert OP.alignment_score(p.seq, p.rows, S, costs, got_ops[q].tolist()) == exp_s


def test_shapes_and_edges():
    # strips of 64 rows (m = 63, 64, 65, 128, 129), empty sequence or profile,
    # single rows and columns, all-gap rows and columns
    rng = np.random.default_rng(11)
    S = inputs.synthetic_subst(20, 1)
    costs = OP.scaled_gap_costs(300, (9, 2, 12, 3))
    probs = []
    for m, n, K in [(0, 0, 1), (0, 7, 3), (5, 0, 2), (1, 1, 1), (63, 70, 4), (64, 64, 3), (65, 40, 5),
                    (128, 130, 2), (129, 100, 6), (40, 129, 8), (200, 3, 2), (3, 200, 3), (150, 150, 12)]:
        probs.append(inputs.profile_problem(m, n, K, rng))
    empty = inputs.profile_problem(30, 40, 5, rng)
    empty.rows[2, :] = inputs.GAP          # a row of gaps only
    empty.rows[:, 7] = inputs.GAP          # a column of gaps only
    probs.append(empty)
    probs.append(inputs.profile_problem(60, 50, 6, rng, p_empty_row=0.5, p_terminal=0.9))
    check_batch(probs, S, costs)


@pytest.mark.parametrize("seed,sigma", [(21, 20), (22, 32), (23, 2)])
def test_random_levels(seed, sigma):
    rng = np.random.default_rng(seed)
    S = inputs.synthetic_subst(sigma, seed)
    costs = OP.scaled_gap_costs(int(rng.integers(50, 5000)), (8, 1, 11, 2))
    probs = [inputs.profile_problem(int(rng.integers(1, 220)), int(rng.integers(1, 200)), int(rng.integers(1, 16)),
                                    rng, alphabet=sigma) for _ in range(24)]
    check_batch(probs, S, costs)


def test_ties_everywhere():
    # one-letter and two-letter alphabets with flat scores: many optimal
    # alignments, so the result rests on the tie rule alone
    rng = np.random.default_rng(31)
    for sigma, S in [(1, np.zeros((1, 1), np.int32)), (2, np.ones((2, 2), np.int32))]:
        probs = [inputs.profile_problem(int(rng.integers(1, 90)), int(rng.integers(1, 90)), int(rng.integers(1, 6)),
                                        rng, alphabet=sigma) for _ in range(10)]
        check_batch(probs, S, (0, 0, 0, 0))
        check_batch(probs, S, (1, 1, 1, 1))


def test_negative_and_zero_costs():
    rng = np.random.default_rng(41)
    S = inputs.synthetic_subst(20, 4)
    probs = [inputs.profile_problem(int(rng.integers(1, 120)), int(rng.integers(1, 120)), int(rng.integers(1, 8)), rng)
             for _ in range(8)]
    check_batch(probs, S, (-2, 0, 3, -1))


def test_long_problem():
    # many strips and trace-back windows: m = 1500, n = 1300 (DP inputs too
    # large for LDS, read from global memory), and m = 1500, n = 400 (24
    # strips over the waves of one workgroup, DP inputs in LDS)
    rng = np.random.default_rng(51)
    S = inputs.synthetic_subst(20, 5)
    costs = OP.scaled_gap_costs(1000, (9, 2, 12, 3))
    check_batch([inputs.profile_problem(1500, 1300, 3, rng)], S, costs)
    check_batch([inputs.profile_problem(1500, 400, 5, rng), inputs.profile_problem(1300, 420, 2, rng)], S, costs)


def test_rejects_bad_input():
    S = inputs.synthetic_subst(20, 1)
    p = inputs.profile_problem(10, 10, 2, np.random.default_rng(0))
    bad = p.rows.copy()
    bad[0, 0] = 25
    with pytest.raises(B.FamsaError):
        B.profile_align([(p.seq, bad)], S, (1, 1, 1, 1))
    with pytest.raises(B.FamsaError):
        B.profile_align([(p.seq, np.zeros((0, 10), np.uint8))], S, (1, 1, 1, 1))


def test_wide_values_and_mixed_batches():
    # scores and gap costs near the library's limits: the DP runs in int64
    # for these problems and in int32 for the small ones of the same batch;
    # problems read their DP inputs from LDS or, when too wide, from global
    # memory
    rng = np.random.default_rng(61)
    S = (inputs.synthetic_subst(20, 6).astype(np.int64) * 85).astype(np.int32)  # |S| up to 1020
    costs = (900_000, 30_000, 1_000_000, 50_000)
    probs = [inputs.profile_problem(int(rng.integers(60, 200)), int(rng.integers(60, 200)), int(rng.integers(20, 60)),
                                    rng) for _ in range(6)]
    check_batch(probs, S, costs)
    # int64 problems too wide for their records, costs and edge rows to sit
    # in LDS (they read them from global memory), beside ones that fit
    wide = [inputs.profile_problem(int(rng.integers(550, 700)), int(rng.integers(550, 700)), int(rng.integers(20, 40)),
                                   rng) for _ in range(2)]
    check_batch(wide + probs[:2], S, costs)
    # int32 values with costs too large for 16 bits (K max|S| >= 2^15): the
    # cost table stays int32 in LDS
    mid = [inputs.profile_problem(int(rng.integers(60, 150)), int(rng.integers(60, 150)), int(rng.integers(40, 60)),
                                  rng) for _ in range(4)]
    check_batch(mid, S, (700, 150, 900, 200))
    # one row and at most 40 columns and residues: below 2^28 even at these costs
    small = [inputs.profile_problem(int(rng.integers(1, 40)), int(rng.integers(1, 40)), 1, rng) for _ in range(6)]
    mixed = [p for pair in zip(probs, small) for p in pair]
    check_batch(mixed, inputs.synthetic_subst(20, 6), (9, 2, 12, 3))
    check_batch(mixed, S, costs)


def test_large_level_waves_capped():
    # a level of 1,100 problems (four or more per CU on a 256-CU GPU: at
    # most four waves per problem), a few of them wide enough for ten strips
    # and more strips than waves, so each wave takes several strips in turn
    rng = np.random.default_rng(71)
    S = inputs.synthetic_subst(20, 7)
    costs = OP.scaled_gap_costs(2000, (9, 2, 12, 3))
    probs = [inputs.profile_problem(int(rng.integers(5, 120)), int(rng.integers(5, 120)), int(rng.integers(1, 20)), rng)
             for _ in range(1094)]
    probs += [inputs.profile_problem(int(rng.integers(580, 700)), int(rng.integers(500, 640)), int(rng.integers(2, 12)),
                                     rng) for _ in range(6)]
    check_batch(probs, S, costs)
