"""Pins of the oracle's accuracy metrics, Eqs. (11)-(13) of the section
"Accurate modeling of plasma accelerators in finite order PSATD", against
values worked out by hand, and of the scan's host-side Err_sigma_gamma against
the oracle's on matched slices."""
import math

import numpy as np
import pytest

from oracle import diag


def test_err_sigma_gamma_is_the_rms_of_the_relative_slice_deviations():
    # Eq. (11): deviations +0.1, -0.2, 0 and +0.3 of the reference spreads
    ref = np.array([2.0, 4.0, 1.0, 0.5])
    fin = ref * np.array([1.1, 0.8, 1.0, 1.3])
    want = math.sqrt((0.01 + 0.04 + 0.0 + 0.09) / 4)      # 0.18708...
    assert diag.err_sigma_gamma(fin, ref) == pytest.approx(want, rel=1e-13)
    # a mean of absolute deviations would give 0.15, a plain rms of differences
    # (no division by the reference) 0.2
    assert abs(diag.err_sigma_gamma(fin, ref) - 0.15) > 0.03
    # sign-symmetric: the square removes the sign of each deviation
    assert diag.err_sigma_gamma(ref * np.array([0.9, 1.2, 1.0, 0.7]), ref) == pytest.approx(want, rel=1e-13)
    assert diag.err_sigma_gamma(ref, ref) == 0.0


def test_err_emittance_is_relative_to_the_infinite_order_run():
    # Eq. (12): signed, normalized by the reference emittance
    assert diag.err_emittance(1.25, 1.0) == pytest.approx(0.25, rel=1e-15)
    assert diag.err_emittance(3.0, 4.0) == pytest.approx(-0.25, rel=1e-15)
    # normalizing by the finite-order value instead would give 0.2 here
    assert diag.err_emittance(5.0, 4.0) == pytest.approx(0.25, rel=1e-15)


def test_err_ez_normalized_closed_forms():
    rng = np.random.default_rng(3)
    ez = rng.standard_normal((16, 32))
    # a uniform relative error a: both Eq. (13) and its normalized L2 form give a
    assert diag.err_ez_normalized(1.03 * ez, ez) == pytest.approx(0.03, rel=1e-12)
    assert diag.err_ez_pointwise(1.03 * ez, ez) == pytest.approx(0.03, rel=1e-12)
    # Parseval: the spectral norm ratio equals the real-space one
    d = 1e-3 * rng.standard_normal(ez.shape)
    want = np.linalg.norm(d) / np.linalg.norm(ez)
    assert diag.err_ez_normalized(ez + d, ez) == pytest.approx(want, rel=1e-12)
    # one added Fourier mode of amplitude 0.01 on a single-mode reference of
    # amplitude 1 (orthogonal modes): the norm ratio is 0.01
    nz_, nr_ = 32, 16
    zz, rr = np.meshgrid(np.arange(nz_), np.arange(nr_))
    base = np.cos(2 * np.pi * 3 * zz / nz_)
    extra = 0.01 * np.cos(2 * np.pi * 5 * zz / nz_ + 2 * np.pi * 2 * rr / nr_)
    assert diag.err_ez_normalized(base + extra, base) == pytest.approx(0.01, rel=1e-12)


def test_err_ez_pointwise_follows_eq13_where_the_reference_is_nonzero():
    # spectral cells with a zero reference spectrum are skipped (Eq. (13) is
    # undefined there); elsewhere each cell contributes its relative deviation
    nz_, nr_ = 8, 4
    ref_hat = np.zeros((nr_, nz_), complex)
    ref_hat[0, 1], ref_hat[0, -1] = 2.0, 2.0
    ref_hat[1, 2], ref_hat[-1, -2] = 1.0, 1.0
    fin_hat = ref_hat.copy()
    fin_hat[0, 1] *= 1.2
    fin_hat[0, -1] *= 1.2
    fin_hat[1, 2] *= 0.9
    fin_hat[-1, -2] *= 0.9
    ref = np.fft.ifft2(ref_hat).real
    fin = np.fft.ifft2(fin_hat).real
    want = math.sqrt((2 * 0.2 ** 2 + 2 * 0.1 ** 2) / 4)
    assert diag.err_ez_pointwise(fin, ref) == pytest.approx(want, rel=1e-9)


def test_scan_err_sigma_gamma_equals_the_oracle_on_matched_slices():
    # the scan's host metric matches slices by their offset from each beam's
    # centroid and skips sparse ones; on the slices it keeps it must be
    # exactly the oracle's Eq. (11)
    from paper_1611_05712_amd.scan import err_sigma_gamma as scan_err
    rng = np.random.default_rng(5)
    ref = rng.uniform(0.5, 2.0, 10)
    fin = ref * rng.uniform(0.7, 1.3, 10)
    cnt = [50] * 10
    assert scan_err(fin, cnt, ref, cnt) == pytest.approx(diag.err_sigma_gamma(fin, ref), rel=1e-14)
    # the finite run has two fewer slices (one on each side): offsets -4..3
    got = scan_err(fin[1:-1], cnt[1:-1], ref, cnt)
    assert got == pytest.approx(diag.err_sigma_gamma(fin[1:-1], ref[1:-1]), rel=1e-14)
    # sparse slices dropped from both sides of the comparison
    cnt_f = [50] * 10
    cnt_f[3] = 4
    keep = [k for k in range(10) if k != 3]
    assert scan_err(fin, cnt_f, ref, cnt) == pytest.approx(diag.err_sigma_gamma(fin[keep], ref[keep]), rel=1e-14)
