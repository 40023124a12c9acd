"""The low-resolution equidistant vs stretched comparison (paper Sect. 2.2,
Fig. 1) through the library: the same wind and cone CME on 300 equidistant
radial cells (1.362 R_sun at 1 AU) and on 60 stretched ones (10.7 R_sun at
1 AU).  Both record a shock at Earth within a few hours of each other; the
stretched grid's shock is less sharp (wider, smaller average gradient), as
the paper reports.  A shortened relaxation (2 days) keeps the test short."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_stretched_grid_smears_the_shock_at_earth():
    from paper_2211_12867_amd import forecast
    res = forecast.stretching_comparison(relax_days=2.0, cme_days=2.5, log=None)
    eq, st = res["low_equidistant"], res["low_stretched"]
    assert abs(eq["dr_1au_rsun"] - 1.362) < 0.01 and abs(st["dr_1au_rsun"] - 10.7) < 0.1
    for r in (eq, st):
        assert not math.isnan(r["arrival_h"]) and r["width_h"] > 0.0, r
    assert abs(eq["arrival_h"] - st["arrival_h"]) < 6.0, (eq["arrival_h"], st["arrival_h"])
    assert st["width_h"] > eq["width_h"], (st["width_h"], eq["width_h"])
    assert st["gradient_kms_h"] < eq["gradient_kms_h"], (st["gradient_kms_h"], eq["gradient_kms_h"])
