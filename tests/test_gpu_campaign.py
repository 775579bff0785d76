"""The small-L campaign driver end to end on a tiny point: converged weights,
a peak of C(Delta) inside the scanned range with jackknife errors, and the
equal-height field at a first-order temperature."""
import math
import sys

import numpy as np
import pytest

from paper_1502_07214_amd import campaign

pytestmark = pytest.mark.gpu


def test_campaign_point_l4():
    print("[campaign] L=4 T=1.0", flush=True)
    sys.stdout.flush()
    out = campaign.run_point(4, 1.0, 64, 500, 300, 4, 2000, seed=3)
    assert out["flat"], out
    assert not out["scan_peak_at_edge"], out
    assert math.isfinite(out["delta_star"]) and out["delta_star_err"] >= 0.0
    assert out["C_star"] > 0.0 and out["C_star_err"] >= 0.0
    dm = campaign.delta_mid(1.0)
    assert dm - 1.0 < out["delta_star"] < dm + 0.5
    if "delta_eqh" in out:
        assert abs(out["delta_eqh"] - out["delta_star"]) < 0.5
        assert np.isfinite(out["barrier"])
