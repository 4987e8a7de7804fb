"""Batched execution (many families in one persistent, graph-replayed launch
per step) equals plain per-family launches and the oracle; autotuned launch
parameters never change a result."""
import os

import numpy as np
import pytest

from helpers import Sampler, check_all_tiles
from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu


def small_c3(seed=2, nfam=12):
    # the c3 recipe with smaller families so the oracle checks everything
    return inputs.c3(seed=seed, nfam=nfam, k_range=(20, 300), root_range=(30, 1200))


def test_batched_equals_plain_and_oracle():
    b = small_c3()
    with B.Plan.from_batch(b) as p:
        bat = p.collect()
        assert p.info().nsteps == 1
    with B.Plan.from_batch(b, flags=B.PLAIN) as p:
        pla = p.collect()
    assert bat.keys() == pla.keys()
    for key in bat:
        assert np.array_equal(bat[key], pla[key]), key
    check_all_tiles(b, bat, 1024)


def test_autotune_keeps_results(tmp_path):
    b = small_c3(seed=5, nfam=6)
    cache = str(tmp_path / "tune.txt")
    with B.Plan.from_batch(b) as p:
        before = p.collect()
        p.autotune(cache)
        after = p.collect()
        info = p.info()
    assert os.path.exists(cache) and open(cache).read().strip()
    for key in before:
        assert np.array_equal(before[key], after[key])
    # a second plan picks the cached parameters up
    os.environ["FAMSA_LCS_TUNE_CACHE"] = cache
    try:
        with B.Plan.from_batch(b) as p2:
            assert p2.info().cols_per_item == info.cols_per_item
            again = p2.collect()
    finally:
        del os.environ["FAMSA_LCS_TUNE_CACHE"]
    for key in before:
        assert np.array_equal(before[key], again[key])


@pytest.mark.parametrize("cols", [16, 64, 512])
def test_cols_per_item_keeps_results(cols):
    b = small_c3(seed=7, nfam=5)
    with B.Plan.from_batch(b, cols_per_item=cols) as p:
        check_all_tiles(b, p.collect(), 1024)
