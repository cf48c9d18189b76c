"""GPU: the unit microbenchmarks behind the roofline figures run through the C ABI
and report plausible rates (positive, below the device's issue limits)."""
import math

import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

CLK_CU = 2.4e9 * 256      # clock x compute units of the device


@pytest.mark.parametrize("kind", ["lds_or_random", "lds_or_spread", "valu_int32", "mod64"])
def test_microbench_rates(kind):
    from paper_1111_3297_amd import api
    say("microbench %s" % kind)
    r = api.microbench(kind, 256)
    assert math.isfinite(r) and r > 0
    # per lane operations: at most 64 lanes of LDS access and 4 x 16 lanes of VALU per clock and CU
    # (3x slack for a clock above the nominal one)
    assert r < 3 * 64 * CLK_CU, r


def test_microbench_rejects_bad_arguments():
    from paper_1111_3297_amd import _lib, api
    with pytest.raises(_lib.SieveError):
        api.microbench("lds_or_random", 0)
