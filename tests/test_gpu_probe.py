"""The v_sad_u8 issue-rate probe runs and stays under the roofline's peak
(256 CUs x 64 lanes x 2.4 GHz)."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_sad_rate_below_peak():
    import paper_2001_07809_amd as sbs
    r = sbs.probe_sad_rate(blocks=4096, trips=200)
    assert r["ms"] > 0
    assert 0 < r["lane_ops_per_s"] <= 1.05 * 256 * 64 * 2.4e9
