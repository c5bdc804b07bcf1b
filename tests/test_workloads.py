"""Seeded input generators (no method arithmetic): shapes, ranges, determinism."""
def test_scan_instances_cover_the_scan_ranges():
    from workloads import SCAN_ORDERS, scan_instances
    a = scan_instances()
    b = scan_instances()
    assert len(a) == 64 and [x.__dict__ for x in a] == [x.__dict__ for x in b]   # seeded
    assert {x.order for x in a} == set(SCAN_ORDERS)
    for x in a:
        assert x.nz in (512, 1024, 2048) and x.nr in (128, 256)
        assert 0.01 <= x.dz <= 0.05 and 0.03 <= x.dr <= 0.08
        assert 500 <= x.gamma_w <= 4000 and 10e-12 <= x.charge_w_C <= 100e-12
        assert x.nz * x.dz >= 8.0                  # driver, 4/k_p gap and witness fit
        assert x.features()[0] == (0.0 if x.order == 0 else 2.0 / x.order)
    # every physical tuple is run at every order
    per = {}
    for x in a[:63]:
        per.setdefault(x.tuple_index, set()).add(x.order)
    assert all(v == set(SCAN_ORDERS) for v in per.values()) and len(per) == 9
