"""Host logic of the order surrogate: feature/target maps, the scan's
required order, and the fallback that keeps the plain simulation the referee."""
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
def test_fallback_climbs_until_the_referee_accepts(pick, want, ran):
    t = _record({8: (0.2, 0.01), 16: (0.04, 0.06), 24: (0.03, 0.02), 32: (0.06, 0.0),
                 48: (0.01, 0.0), 64: (0.0, 0.0)})
    got, r = S.select_with_fallback(pick, S.table_referee(t))
    assert got == want and r == ran


def test_fallback_ends_at_infinite_order():
    t = _record({p: (0.5, 0.0) for p in S.ORDERS})
    got, r = S.select_with_fallback(48, S.table_referee(t))
    assert got == 0 and r == [48, 64]


def test_settle_cost_counts_the_infinite_order_run():
    # a pick of infinity costs its one production run; a finite pick costs the
    # twin plus every order the fallback climbed through
    assert S.settle_cost([]) == 1
    assert S.settle_cost([16, 24]) == 3


def test_compare_pickers_against_no_network_baselines():
    recs = [_record({8: (0.2, 0.0), 16: (0.01, 0.0), 24: (0.0, 0.0), 32: (0.0, 0.0), 48: (0.0, 0.0),
                     64: (0.0, 0.0)}),
            _record({p: (0.5, 0.0) for p in S.ORDERS}),
            _record({p: (0.0, 0.0) for p in S.ORDERS})]
    for k, r in enumerate(recs):
        r["tuple"] = k
    scan = {"tuples": recs}
    want = [16, 0, 8]
    assert [S.required_order(r) for r in recs] == want
    assert S.majority_order(scan, [0, 1, 2]) == 8      # all counts 1: the lowest order wins the tie
    oracle_pick = {0: 16, 1: 0, 2: 8}
    res = S.compare_pickers(scan, [0, 1, 2], {
        "perfect": lambda t: oracle_pick[t["tuple"]],
        "infinite": lambda t: 0,
        "climb": lambda t: S.ORDERS[0]})
    assert res["scan"] == {"runs": 21, "exact": 3, "over": 0}
    assert res["perfect"] == {"runs": 2 + 1 + 2, "exact": 3, "over": 0}
    assert res["infinite"] == {"runs": 3, "exact": 1, "over": 2}
    # climbing from the lowest order always finds the answer, at 3 + 7 + 2 runs
    assert res["climb"] == {"runs": 3 + 7 + 2, "exact": 3, "over": 0}
