"""The streaming-read probe that the tracer's gathers are compared with."""
import pytest

from tests import parity_util as PU

pytestmark = pytest.mark.gpu


def test_read_bandwidths_are_ordered_and_below_the_hbm_peak():
    if not PU.gpu_available():
        pytest.skip("no GPU")
    from paper_2606_02413_amd import rtsun as R
    print("case read probe", flush=True)
    bw = R.read_bandwidths(0)
    print("read bandwidths GB/s", bw, flush=True)
    # HBM3E peak 8 TB/s; the die-local L2 and the Infinity Cache serve more
    assert 1000.0 < bw["hbm_GBps"] < 8000.0
    assert bw["l2_GBps"] > bw["hbm_GBps"]
    assert bw["infinity_cache_GBps"] > bw["hbm_GBps"]
