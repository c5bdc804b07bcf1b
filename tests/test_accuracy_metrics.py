"""Host-side error metrics of the scan and the accuracy study (Eqs. (11)-(13)):
slices of two runs are matched by their offset from each beam's centroid."""
import math

import numpy as np
import pytest

from paper_1611_05712_amd.scan import err_sigma_gamma
from paper_1611_05712_amd.accuracy import errors


def test_err_sigma_gamma_matches_slices_by_offset():
    # finite run: 6 slices (offsets -3..2), reference: 8 slices (offsets -4..3)
    sg_f = [1.1, 2.2, 3.3, 4.4, 5.5, 6.6]
    sg_i = [9.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 9.0]
    cnt = [100] * 8
    # matched pairs: offsets -3..2 -> every ratio 1.1
    assert err_sigma_gamma(sg_f, cnt[:6], sg_i, cnt) == pytest.approx(0.1, rel=1e-12)


def test_err_sigma_gamma_skips_sparse_slices():
    sg_f = [2.0, 1.0, 1.5, 3.0]
    sg_i = [1.0, 1.0, 1.0, 1.0]
    cnt_f = [5, 100, 100, 100]          # slice 0 below the 10-particle floor
    cnt_i = [100, 100, 100, 9]          # slice 3 below it in the reference
    # remaining relative deviations: 0, 0.5 -> rms = sqrt(0.125)
    assert err_sigma_gamma(sg_f, cnt_f, sg_i, cnt_i) == pytest.approx(math.sqrt(0.125), rel=1e-12)
    assert math.isnan(err_sigma_gamma([1.0], [1], [1.0], [1]))


def _run(order, eps, sg):
    w = {"eps_nx": eps, "slice_sigma_gamma": sg, "slice_count": [50] * len(sg)}
    return {"order": order, "marks": [{"step": 10, "witness": w}]}


def test_errors_of_a_run_against_its_twin():
    ref = _run(0, 2.0, [1.0, 2.0, 4.0, 8.0])
    f = _run(16, 2.5, [1.0, 2.0, 4.0, 8.0])
    e = errors(f, ref)
    assert e["err_sigma_gamma"] == 0.0 and e["err_eps"] == pytest.approx(0.25)
    rng = np.random.default_rng(0)
    ez = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    e = errors(f, ref, ez * 1.01, ez)
    assert e["err_ez"] == pytest.approx(0.01, rel=1e-12)


@pytest.mark.parametrize("order", [4, 8, 16, 32, 64])
def test_report_resonance_matches_oracle(order):
    # the report's own [k_z] and resonance root against the oracle's
    from oracle import spectral as sp
    from oracle import stencil as st
    from paper_1611_05712_amd.accuracy import modified_kz, resonance_kz
    dz = 0.0119
    kz = np.linspace(0.1, np.pi / dz, 50)
    np.testing.assert_allclose(modified_kz(kz, dz, order), sp.kz_modified(kz, dz, order), rtol=1e-12, atol=1e-12)
    want = st.resonance_kz(1958.0, order, dz, 0.0)
    got = resonance_kz(1958.0, order, dz)
    if np.isnan(want):
        assert np.isnan(got)
    else:
        assert got == pytest.approx(want, rel=1e-6)


def test_resonance_table_of_the_survey():
    # k_z dz at the resonance for gamma = 2000 (on axis): 0.3079 (p = 8),
    # 0.8188 (16), 1.3764 (32), 1.8511 (64)
    from paper_1611_05712_amd.accuracy import resonance_kz
    for p, want in ((8, 0.3079), (16, 0.8188), (32, 1.3764), (64, 1.8511)):
        assert resonance_kz(2000.0, p, 1.0) == pytest.approx(want, abs=2e-4)
