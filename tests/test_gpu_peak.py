"""The integer-VALU ceiling microbenchmark runs on every CU and reports a
rate, a clock and lane operations per clock per CU that are physically
possible (a CU has four SIMDs; a lane operation rate above 256 per clock
would mean the counting is wrong)."""
import pytest

from paper_1603_06958_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_valu_peak_is_plausible(variant):
    r = B.valu_peak(variant, blocks_per_cu=4, iters=2000)
    assert r.cus >= 1
    assert r.ms > 0 and r.lane_ops == 2000 * 192 * 4 * 256 * r.cus
    assert 0.3 < r.clock_ghz < 4.0
    assert 4.0 < r.lane_ops_per_clk_per_cu <= 256.0
