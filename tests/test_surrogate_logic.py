"""Host logic of the order surrogate: feature/target maps, the scan's
required order, and the fallback that keeps the plain simulation the judge."""
import math

import numpy as np
import pytest

from paper_1611_05712_amd import surrogate as S


def test_features_map_scan_ranges_to_unit_box():
    lo = S.features(8, 0.01, 0.03, 500.0, 10.0)
    hi = S.features(0, 0.05, 0.08, 4000.0, 100.0)
    np.testing.assert_allclose(lo, [1.0, -1.0, -1.0, -1.0, -1.0], atol=1e-4)
    np.testing.assert_allclose(hi, [-1.0, 1.0, 1.0, 1.0, 1.0], atol=1e-4)


def test_targets_round_trip():
    y = S.targets(0.07, -0.002)
    np.testing.assert_allclose(S.errors_from_targets(y), [0.07, 0.002], rtol=1e-5)


def _record(errs):
    return {"tuple": 0, "dz": 0.02, "dr": 0.05, "gamma_w": 1000.0, "charge_w_pC": 50.0,
            "errors": {str(p): {"err_sigma_gamma": a, "err_eps": b} for p, (a, b) in errs.items()}}


def test_required_order_is_the_lowest_passing_order():
    t = _record({8: (0.2, 0.01), 16: (0.04, 0.06), 24: (0.03, 0.02), 32: (0.06, 0.0),
                 48: (0.01, 0.0), 64: (0.0, 0.0)})
    assert S.required_order(t) == 24
    t = _record({p: (0.5, 0.0) for p in S.ORDERS})
    assert S.required_order(t) == 0


@pytest.mark.parametrize("pick,want,ran", [(8, 24, [8, 16, 24]), (24, 24, [24]), (32, 48, [32, 48]),
                                           (0, 0, [])])
def test_fallback_climbs_until_the_judge_accepts(pick, want, ran):
    t = _record({8: (0.2, 0.01), 16: (0.04, 0.06), 24: (0.03, 0.02), 32: (0.06, 0.0),
                 48: (0.01, 0.0), 64: (0.0, 0.0)})
    got, r = S.select_with_fallback(pick, S.table_judge(t))
    assert got == want and r == ran


def test_fallback_ends_at_infinite_order():
    t = _record({p: (0.5, 0.0) for p in S.ORDERS})
    got, r = S.select_with_fallback(48, S.table_judge(t))
    assert got == 0 and r == [48, 64]
