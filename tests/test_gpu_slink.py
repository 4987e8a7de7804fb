"""The host SLINK consumer fed the GPU's tiles (FAMSA_LCS_DESCENDING, host
delivery, the consumer as the plan's native callback) against the oracle's
single linkage (Kruskal over the exact similarities of oracle LCS values):
the same multiset of merge similarities and the same cophenetic similarity
for every pair, on families with repeated and empty sequences."""
import numpy as np
import pytest

import oracle
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs
from test_slink import pointer_to_linkage

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,k,lo,hi,sigma,R,flags", [
    (41, 180, 0, 60, 2, 32, 0), (42, 160, 20, 400, 20, 1024, 0), (43, 200, 5, 120, 20, 17, B.NO_GRAPH),
    (44, 150, 1, 30, 2, 1, 0)])
def test_gpu_tiles_into_host_slink_match_oracle(seed, k, lo, hi, sigma, R, flags):
    b = inputs.random_family(k, lo, hi, seed, alphabet=sigma)
    seqs = [b.seq(i) for i in range(k)]
    seqs[3] = seqs[10].copy()      # identical pairs: similarity +inf
    seqs[11] = seqs[10].copy()
    seqs[20] = np.zeros(0, np.uint8)
    seqs[21] = np.zeros(0, np.uint8)
    b = inputs.from_sequences(seqs)
    L = b.lengths()
    s = B.SLink(L)
    with B.Plan.from_batch(b, tile_rows=R, alphabet_size=max(sigma, 2), flags=B.DESCENDING | flags) as p:
        p.run_native(B.SLink.consume_fn(), s.handle)
    assert s.rows_done() == k
    pi, num, den = s.result()
    s.close()
    h, coph = pointer_to_linkage(pi, num, den)
    M = oracle.full_matrix(b.codes, b.seq_off, 0, k)
    h_ref, c_ref = oracle.single_linkage(M, L)
    assert sorted(h, reverse=True) == sorted(h_ref, reverse=True)
    assert (coph == c_ref).all()
