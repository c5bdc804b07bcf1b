"""Pins of the oracle's spectral side against what the paper and mathematics fix."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import jv, jvp, jn_zeros

from oracle import spectral as sp
from oracle import stencil as st
from workloads import random_spectral


# --- finite-order stencil, Eq. (3) -----------------------------------------
def test_alpha_matches_textbook_weights(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "fd_weights.json")))["weights"]
    for order, cs in gold.items():
        n = int(order) // 2
        alpha = sp.fornberg_alpha_exact(n)
        want = [2 * (j + 1) * Fraction(c) for j, c in enumerate(cs)]
        assert alpha == want, (order, alpha, want)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 32, 64])
def test_alpha_sum_is_one(n):
    # consistency of the derivative of a linear function
    assert sum(sp.fornberg_alpha_exact(n)) == 1


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_stencil_exact_for_polynomials(n):
    # an order-2n centered first-derivative stencil differentiates polynomials
    # of degree <= 2n exactly (textbook property); check it with exact rationals
    alpha = sp.fornberg_alpha_exact(n)
    p0 = Fraction(3, 7)
    for deg in range(0, 2 * n + 1):
        f = lambda x: x ** deg
        d = sum(a * (f(p0 + j) - f(p0 - j)) / (2 * j)
                for j, a in zip(range(1, n + 1), alpha))
        exact = deg * p0 ** (deg - 1) if deg else 0
        assert d == exact
    # and fails for degree 2n+1
    deg = 2 * n + 1
    d = sum(a * ((p0 + j) ** deg - (p0 - j) ** deg) / (2 * j)
            for j, a in zip(range(1, n + 1), alpha))
    assert d != deg * p0 ** (deg - 1)


# --- modified wavenumber, Eq. (5) -----------------------------------------
def test_kz_modified_hand_values():
    x = np.pi / 2
    assert sp.kz_modified(np.array([x]), 1.0, 2)[0] == pytest.approx(1.0, abs=1e-15)
    assert sp.kz_modified(np.array([x]), 1.0, 4)[0] == pytest.approx(4 / 3, abs=1e-15)
    # p = 8: 8/5 - 8/105 (hand evaluation of the sum) = 32/21
    assert sp.kz_modified(np.array([x]), 1.0, 8)[0] == pytest.approx(32 / 21, abs=1e-15)


@pytest.mark.parametrize("order", [2, 4, 8, 16, 32, 64])
def test_kz_modified_is_symbol_of_stencil(order):
    # applying the real-space stencil of Eq. (3) to exp(i k z) multiplies it by
    # i [k_z]: compare against a direct real-space evaluation on a grid
    dz = 0.37
    n = order // 2
    alpha = sp.fornberg_alpha(n)
    kz = np.linspace(-np.pi / dz, np.pi / dz, 41)
    zp = 1.3
    f = lambda z: np.exp(1j * kz * z)
    d = sum(alpha[j - 1] * (f(zp + j * dz) - f(zp - j * dz)) / (2 * j * dz)
            for j in range(1, n + 1))
    symbol = d / f(zp) / 1j
    np.testing.assert_allclose(symbol.imag, 0, atol=1e-12)
    np.testing.assert_allclose(sp.kz_modified(kz, dz, order), symbol.real, rtol=1e-12,
                               atol=1e-12)


def test_kz_modified_nyquist_zero_and_convergence():
    dz = 0.1
    for order in (2, 4, 8, 16, 32):
        assert abs(sp.kz_modified(np.array([np.pi / dz]), dz, order)[0]) < 1e-12
    # truncation error of an order-2n stencil scales as (k dz)^(2n)
    for order in (4, 8):
        e1 = 1 - sp.kz_modified(np.array([0.1]), 1.0, order)[0] / 0.1
        e2 = 1 - sp.kz_modified(np.array([0.05]), 1.0, order)[0] / 0.05
        assert e1 / e2 == pytest.approx(2.0 ** order, rel=2e-2)
    kz = sp.kz_grid(64, dz)
    kinf = sp.kz_modified(kz, dz, 0)
    # infinite order: k_z itself except the Nyquist column (index nz/2), zero
    # like every finite order there
    assert kinf[32] == 0.0 and kz[32] == pytest.approx(-np.pi / dz, rel=1e-14)
    assert np.array_equal(np.delete(kinf, 32), np.delete(kz, 32))
    assert np.abs(sp.kz_modified(kz, dz, 256) - kz)[np.abs(kz) < 0.5 * np.pi / dz].max() < 1e-10


# --- discrete Hankel transform pair ---------------------------------------
@pytest.mark.parametrize("nr", [16, 64, 256])
@pytest.mark.parametrize("kind", [sp.KPERP_JM_ZEROS, sp.KPERP_J0_ZEROS, sp.KPERP_SINE])
def test_dht_round_trip(nr, kind):
    # full-rank orders: F is the inverse, so the round trip is exact; orders
    # with a dropped near-null direction (mode 1, order 0 on the zeros of J_1;
    # mode 1, order 2 on the zeros of J_0 at large nr): B F is the orthogonal
    # projector that removes exactly that one, isolated, direction
    for m in (0, 1):
        hk = sp.HankelPair(m, nr, 0.05, kind)
        g = random_spectral((nr, 8), seed=nr + m)
        for nu in (m - 1, m, m + 1):
            B, F = hk.B[nu], hk.F[nu]
            sv = np.linalg.svd(B, compute_uv=False)
            dropped = int((sv < sp.PINV_RCOND * sv[0]).sum())
            P = B @ F
            if dropped == 0:
                back = hk.backward(hk.forward(g, nu), nu)
                assert np.abs(back - g).max() < 1e-12 * np.abs(g).max() * max(1, nr / 64)
            else:
                assert (kind, m, nu) in ((sp.KPERP_JM_ZEROS, 1, 0), (sp.KPERP_J0_ZEROS, 1, 2))
                assert dropped == 1 and sv[-2] > 100 * sp.PINV_RCOND * sv[0]
                assert np.abs(P - P.T).max() < 1e-10 and np.abs(P @ P - P).max() < 1e-10
                assert np.trace(P) == pytest.approx(nr - 1, abs=1e-8)
                assert np.abs(F @ B @ F - F).max() < 1e-10 * np.abs(F).max()


def test_jm_zero_bases_share_their_norm_and_are_orthogonal():
    # At the zeros k of J_m, J_{m-1}(k r), J_m(k r) and J_{m+1}(k r) satisfy
    # Dini conditions at R: int_0^R J_nu(k_i r) J_nu(k_j r) r dr = delta_ij N_i
    # with the same N_i = R^2/2 J_{m+1}(k_i R)^2 for the three orders (this is
    # what makes the conserved spectral energy the real-space field energy).
    # With the zeros of J_0, the order-2 basis of mode 1 is not orthogonal.
    from scipy.integrate import quad
    R = 1.0
    for m in (0, 1, 2):
        k = jn_zeros(m, 4) / R
        N = 0.5 * R * R * jv(m + 1, k * R) ** 2
        for nu in (m - 1, m, m + 1):
            for i in range(3):
                for j in range(3):
                    v = quad(lambda r: jv(nu, k[i] * r) * jv(nu, k[j] * r) * r, 0, R, limit=200)[0]
                    assert v == pytest.approx(N[i] if i == j else 0.0, abs=1e-10), (m, nu, i, j)
    k0 = jn_zeros(0, 4) / R
    off = quad(lambda r: jv(2, k0[0] * r) * jv(2, k0[1] * r) * r, 0, R)[0]
    assert abs(off) > 1e-3


def test_dht_gaussian_closed_form():
    # For k_i = j_{0,i}/R (zeros of J_0) a smooth function g(r) has the
    # Fourier-Bessel coefficients a_i = 2/(R^2 J_1(j_{0,i})^2) int_0^R g J_0(k_i r) r dr.
    # For g = exp(-r^2/(2a^2)) with a << R the integral is a^2 exp(-k^2 a^2/2)
    # (textbook Hankel transform of a Gaussian).  The discrete forward transform
    # must reproduce these coefficients.
    nr, dr = 256, 0.05
    R = nr * dr
    a = 0.08 * R
    hk = sp.HankelPair(0, nr, dr, sp.KPERP_J0_ZEROS)
    g = np.exp(-hk.r ** 2 / (2 * a * a))
    coef = hk.forward(g[:, None].astype(complex), 0)[:, 0]
    z0 = jn_zeros(0, nr)
    want = 2.0 / (R ** 2 * jv(1, z0) ** 2) * a * a * np.exp(-(z0 / R) ** 2 * a * a / 2)
    assert np.abs(coef.real - want).max() < 1e-6 * np.abs(want).max()
    # and for order 1: r exp(-r^2/2a^2) has Hankel transform a^4 k exp(-k^2 a^2/2),
    # synthesized back on the grid with J_1 of the same k grid
    g1 = hk.r * np.exp(-hk.r ** 2 / (2 * a * a))
    hk1 = sp.HankelPair(1, nr, dr, sp.KPERP_JM_ZEROS)
    c1 = hk1.forward(g1[:, None].astype(complex), 1)[:, 0]
    z1 = jn_zeros(1, nr)
    want1 = 2.0 / (R ** 2 * jv(2, z1) ** 2) * a ** 4 * (z1 / R) * np.exp(-(z1 / R) ** 2 * a * a / 2)
    assert np.abs(c1.real - want1).max() < 1e-6 * np.abs(want1).max()


def test_dht_conditioning_of_chosen_grids():
    # zeros of J_m, modes 0 and 1, Nr = 256: the order-0 synthesis of mode 1 has
    # exactly one singular value below the cutoff (cond 2e7); every other order
    # is well conditioned, and the truncated pseudo-inverse is bounded
    r = sp.r_grid(256, 0.05)
    for m in (0, 1):
        k = sp.kperp_grid(m, 256, 0.05, sp.KPERP_JM_ZEROS)
        for nu in (m - 1, m, m + 1):
            B = sp.bessel_synthesis(nu, r, k)
            sv = np.linalg.svd(B, compute_uv=False)
            if (m, nu) == (1, 0):
                assert sv[-1] / sv[0] < 1e-6 and sv[-2] / sv[0] > 1e-2
            else:
                assert sv[-1] / sv[0] > 1e-3
            F = np.linalg.pinv(B, rcond=sp.PINV_RCOND)
            assert np.linalg.norm(F, 2) * sv[0] < 1e3


@pytest.mark.parametrize("nr", [64, 256])
def test_spectral_gradient_reproduces_real_space_derivative(nr):
    # A smooth mode-1 scalar S(r) (Hankel order 1) is transformed, multiplied by
    # the gradient table (-k/2, +k/2) and synthesized with orders 2 and 0; the
    # result must equal the analytic (grad S)_+- = (dS/dr -+ S/r)/2 at the nodes.
    # This is what makes the discrete transforms a valid representation of the
    # spectral operators; the zeros of J_m and of J_0 pass, the (i+1) pi/R grid
    # does not.
    dr = 0.05
    R = nr * dr
    for kind, tol in ((sp.KPERP_JM_ZEROS, 1e-10), (sp.KPERP_J0_ZEROS, 1e-10), (sp.KPERP_SINE, None)):
        hk = sp.HankelPair(1, nr, dr, kind)
        r = hk.r
        c, s = 0.5 * R, 0.05 * R
        S = r * np.exp(-(r - c) ** 2 / (2 * s * s))
        dS = np.exp(-(r - c) ** 2 / (2 * s * s)) * (1 - r * (r - c) / (s * s))
        a = hk.F[1] @ S
        gp = hk.B[2] @ (-hk.k * a / 2)
        gm = hk.B[0] @ (hk.k * a / 2)
        err = max(np.abs(gp - 0.5 * (dS - S / r)).max(), np.abs(gm - 0.5 * (dS + S / r)).max())
        err /= np.abs(dS).max()
        if tol is not None:
            assert err < tol
        else:
            assert err > 1e-4


# --- operator table, Eqs. (2a)-(2b), against real-space derivatives ---------
def _cart_from_pm(vp, vm, vz, th):
    vr = vp + vm
    vt = 1j * (vp - vm)
    return vr * np.cos(th) - vt * np.sin(th), vr * np.sin(th) + vt * np.cos(th), vz


def _pm_from_cart(fx, fy, fz, th):
    fr = fx * np.cos(th) + fy * np.sin(th)
    ft = -fx * np.sin(th) + fy * np.cos(th)
    return (fr - 1j * ft) / 2, (fr + 1j * ft) / 2, fz


def _sample_points(seed):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.3, 2.0, 12)
    th = rng.uniform(0, 2 * np.pi, 12)
    z = rng.uniform(-1, 1, 12)
    return r, th, z


@pytest.mark.parametrize("m", [0, 1, 2])
def test_gradient_table_matches_real_space(m):
    # S = J_m(k r) exp(-i m theta) exp(i kz z): compute grad S in Cartesian
    # coordinates with the analytic derivative of J_m (scipy jvp), project to
    # (+, -, z) mode components and compare with the table's prediction
    # (-k/2) J_{m+1}, (+k/2) J_{m-1}, (i kz) J_m.
    k, kz = 1.7, 0.9
    r, th, z = _sample_points(m)
    ph = np.exp(-1j * m * th) * np.exp(1j * kz * z)
    S = jv(m, k * r)
    dSr = k * jvp(m, k * r) * ph
    dSt = (-1j * m / r) * S * ph          # (1/r) d/dtheta
    dSz = 1j * kz * S * ph
    fx = dSr * np.cos(th) - dSt * np.sin(th)
    fy = dSr * np.sin(th) + dSt * np.cos(th)
    fp, fm, fz = _pm_from_cart(fx, fy, dSz, th)
    back = np.exp(1j * m * th) * np.exp(-1j * kz * z)       # remove the mode phase
    g = sp.grad(1.0, k, kz)
    np.testing.assert_allclose(fp * back, g[0] * jv(m + 1, k * r), atol=1e-13)
    np.testing.assert_allclose(fm * back, g[1] * jv(m - 1, k * r), atol=1e-13)
    np.testing.assert_allclose(fz * back, g[2] * jv(m, k * r), atol=1e-13)


def _fd_curl_div(field, x, y, z, h=1e-5):
    # central differences of a Cartesian complex vector field (textbook)
    def d(c, axis):
        e = [0.0, 0.0, 0.0]
        e[axis] = h
        a = field(x + e[0], y + e[1], z + e[2])[c]
        b = field(x - e[0], y - e[1], z - e[2])[c]
        return (a - b) / (2 * h)
    curl = (d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1))
    dv = d(0, 0) + d(1, 1) + d(2, 2)
    return curl, dv


@pytest.mark.parametrize("m", [0, 1, 2])
def test_curl_and_div_tables_match_real_space(m):
    k, kz = 1.3, -0.7
    a, b, c = 0.4 + 0.2j, -0.3 + 0.5j, 0.6 - 0.1j   # spectral V_+, V_-, V_z

    def field(x, y, zz):
        r = np.hypot(x, y)
        th = np.arctan2(y, x)
        ph = np.exp(-1j * m * th) * np.exp(1j * kz * zz)
        vp = a * jv(m + 1, k * r) * ph
        vm = b * jv(m - 1, k * r) * ph
        vz = c * jv(m, k * r) * ph
        return _cart_from_pm(vp, vm, vz, th)

    r, th, z = _sample_points(10 + m)
    x, y = r * np.cos(th), r * np.sin(th)
    (cx, cy, cz), dv = _fd_curl_div(field, x, y, z)
    cp, cm, czz = _pm_from_cart(cx, cy, cz, th)
    back = np.exp(1j * m * th) * np.exp(-1j * kz * z)
    want = sp.curl((a, b, c), k, kz)
    np.testing.assert_allclose(cp * back, want[0] * jv(m + 1, k * r), atol=2e-8)
    np.testing.assert_allclose(cm * back, want[1] * jv(m - 1, k * r), atol=2e-8)
    np.testing.assert_allclose(czz * back, want[2] * jv(m, k * r), atol=2e-8)
    np.testing.assert_allclose(dv * back, sp.div((a, b, c), k, kz) * jv(m, k * r), atol=2e-8)


# --- PSATD time integration, Eqs. (1a)-(1b) ---------------------------------
def _curl_matrix(kp, kzm):
    return np.array([[kzm, 0, -0.5j * kp], [0, -kzm, -0.5j * kp], [1j * kp, 1j * kp, 0]])


def test_psatd_equals_exact_ode_solution():
    # with Gauss-consistent inputs (div E = rho^n, continuity for rho^{n+1})
    # the PSATD step is the exact solution of dE/dt = curl B - J, dB/dt = -curl E
    # with J constant over the step: compare with the matrix exponential
    rng = np.random.default_rng(5)
    worst = 0.0
    for trial in range(200):
        kp = rng.uniform(0.01, 5.0)
        kzm = rng.uniform(-5.0, 5.0)
        dt = rng.uniform(0.005, 0.8)
        E = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        B = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        J = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        # make B divergence free (physical) by removing its longitudinal part
        kvec_div = np.array([kp, -kp, 1j * kzm])          # div V = kvec_div . V
        g = np.array([-kp / 2, kp / 2, 1j * kzm])          # grad direction
        B = B - g * (kvec_div @ B) / (kvec_div @ g)
        rho0 = kvec_div @ E
        rho1 = rho0 - dt * (kvec_div @ J)
        K = _curl_matrix(kp, kzm)
        A = np.zeros((7, 7), complex)
        A[0:3, 3:6] = K
        A[3:6, 0:3] = -K
        A[0:3, 6] = -J
        y = expm(A * dt) @ np.concatenate([E, B, [1.0]])
        En, Bn = sp.psatd_push(tuple(E), tuple(B), tuple(J), rho0, rho1, dt, kp, kzm)
        got = np.concatenate([np.array(En), np.array(Bn)])
        worst = max(worst, np.abs(got - y[:6]).max() / np.abs(y[:6]).max())
    assert worst < 1e-12


def _rand_cells(seed, shape=(6, 10)):
    fields = [random_spectral(shape, seed + i) for i in range(11)]
    rng = np.random.default_rng(seed)
    kp = rng.uniform(0.05, 4.0, (shape[0], 1))
    kzm = rng.uniform(-4.0, 4.0, (1, shape[1]))
    return fields, kp, kzm


def test_current_correction_enforces_continuity():
    f, kp, kzm = _rand_cells(1)
    J = tuple(f[0:3])
    r0, r1 = f[3], f[4]
    dt = 0.3
    Jc = sp.current_correction(J, r0, r1, dt, kp, kzm)
    np.testing.assert_allclose(sp.div(Jc, kp, kzm), -(r1 - r0) / dt, atol=1e-12)
    # a current that already satisfies continuity is left unchanged
    Jc2 = sp.current_correction(Jc, r0, r1, dt, kp, kzm)
    for c in range(3):
        np.testing.assert_allclose(Jc2[c], Jc[c], atol=1e-12)


def test_gauss_error_scales_by_C():
    # div E^{n+1} - rho^{n+1} = C (div E^n - rho^n) for any E once continuity holds
    f, kp, kzm = _rand_cells(2)
    E, B, J = tuple(f[0:3]), tuple(f[3:6]), tuple(f[6:9])
    r0, r1 = f[9], f[10]
    dt = 0.25
    J = sp.current_correction(J, r0, r1, dt, kp, kzm)
    En, Bn = sp.psatd_push(E, B, J, r0, r1, dt, kp, kzm)
    C = np.cos(np.sqrt(kp ** 2 + kzm ** 2) * dt)
    np.testing.assert_allclose(sp.div(En, kp, kzm) - r1, C * (sp.div(E, kp, kzm) - r0), atol=1e-12)
    # div B is preserved (stays zero if it starts at zero)
    np.testing.assert_allclose(sp.div(Bn, kp, kzm), C * sp.div(B, kp, kzm), atol=1e-11)


def test_vacuum_energy_conserved_for_transverse_fields():
    f, kp, kzm = _rand_cells(3)
    g = sp.grad(1.0, kp, kzm)
    dvec = (kp, -kp, 1j * kzm)

    def transverse(V):
        d = sum(dvec[c] * V[c] for c in range(3))
        gg = sum(dvec[c] * g[c] for c in range(3))
        return tuple(V[c] - g[c] * d / gg for c in range(3))

    E, B = transverse(tuple(f[0:3])), transverse(tuple(f[3:6]))
    zero = np.zeros_like(f[0])
    En, Bn = sp.psatd_push(E, B, (zero, zero, zero), zero, zero, 0.4, kp, kzm)

    def W(E, B):
        return 2 * abs(E[0]) ** 2 + 2 * abs(E[1]) ** 2 + abs(E[2]) ** 2 \
            + 2 * abs(B[0]) ** 2 + 2 * abs(B[1]) ** 2 + abs(B[2]) ** 2
    np.testing.assert_allclose(W(En, Bn), W(E, B), rtol=1e-12)


@pytest.mark.parametrize("order", [0, 4, 16, 32])
def test_vacuum_dispersion_eigenmode(order):
    # a transverse eigenmode (E_+ = E_- = 1, E_z = 0, B = 0) oscillates as
    # cos(n k dt) with k = sqrt(k_perp^2 + [k_z]^2): the modified dispersion
    # relation omega^2 = k_perp^2 + [k_z]^2 of Eq. (8)
    dz, dt = 0.1, 0.1
    kz = sp.kz_grid(32, dz)[None, :]
    kzm = sp.kz_modified(kz, dz, order)
    kp = np.array([[0.3], [1.1], [2.9]])
    one = np.ones((3, 32), complex)
    zero = np.zeros_like(one)
    E, B = (one, one, zero), (zero, zero, zero)
    for n in range(1, 6):
        E, B = sp.psatd_push(E, B, (zero,) * 3, zero, zero, dt, kp, kzm)
        want = np.cos(n * np.sqrt(kp ** 2 + kzm ** 2) * dt)
        np.testing.assert_allclose(E[0].real, want, atol=1e-12)
        np.testing.assert_allclose(E[2], 0, atol=1e-12)


# --- stencil reach and Cherenkov resonance (Figs. 1-2, Eqs. (6), (10)) -------
def test_stencil_reach_order_32(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "stencil_reach.json")))
    ext = st.stencil_extent(g["order"], g["kperp_per_um"], g["dz_um"], g["dt_dz_over_c"],
                            floor=10.0 ** (-g["decades"] + 1))
    assert abs(ext - g["guard_cells"]) <= 6
    # low orders reach beyond their order, high orders reach about their order
    e4 = st.stencil_extent(4, 0.5, 1.0, 1.0, 1e-15)
    e128 = st.stencil_extent(128, 0.5, 1.0, 1.0, 1e-15)
    assert e4 > 4 * 4
    assert 0.8 < e128 / 128 < 1.2
    # infinite order has no finite reach
    prof = st.stencil_profile(0, 0.5, 1.0, 1.0)
    assert (prof / prof[0])[-1] > 1e-10


def test_resonance_closed_form_order4():
    # p = 4: [k_z] dz = (4/3) sin x - (1/6) sin 2x; at the resonance its ratio
    # to x equals beta(gamma = 3) = sqrt(8/9)
    x = st.resonance_kz(3.0, 4, 1.0)
    assert (4 / 3 * np.sin(x) - np.sin(2 * x) / 6) / x == pytest.approx(np.sqrt(8 / 9), abs=1e-12)
    # infinite order: phase velocity >= c everywhere, no resonance
    assert np.isnan(st.resonance_kz(3.0, 0, 1.0))
    # the resonance moves to larger k_z as the order grows (Fig. 2/3 discussion)
    ks = [st.resonance_kz(3.0, p, 1.0) for p in (4, 8, 16, 32, 64)]
    assert all(a < b for a, b in zip(ks, ks[1:]))


def test_binomial_filter_is_the_121_stencil():
    # the spectral factor cos^2(k_z dz / 2) is exactly the periodic
    # (1/4, 1/2, 1/4) average along z, and vanishes at the Nyquist wavenumber
    nz, dz = 32, 0.05
    rng = np.random.default_rng(1)
    g = rng.standard_normal(nz) + 1j * rng.standard_normal(nz)
    kz = sp.kz_grid(nz, dz)
    f = sp.binomial_filter(kz, dz, np.array([0.0]), 0.1)[0]
    got = np.fft.ifft(np.fft.fft(g) * f)
    want = 0.25 * np.roll(g, 1) + 0.5 * g + 0.25 * np.roll(g, -1)
    np.testing.assert_allclose(got, want, atol=1e-14)
    assert abs(f[nz // 2]) < 1e-30 and f[0] == 1.0


def test_two_binomial_passes_are_the_14641_stencil():
    nz, dz = 32, 0.05
    rng = np.random.default_rng(2)
    g = rng.standard_normal(nz) + 1j * rng.standard_normal(nz)
    kz = sp.kz_grid(nz, dz)
    f = sp.binomial_filter(kz, dz, np.array([0.0]), 0.1, passes=2)[0]
    got = np.fft.ifft(np.fft.fft(g) * f)
    want = (np.roll(g, 2) + 4 * np.roll(g, 1) + 6 * g + 4 * np.roll(g, -1) + np.roll(g, -2)) / 16
    np.testing.assert_allclose(got, want, atol=1e-14)


def _real_mode0_state(nz, nr, seed):
    """Real-space mode-0 fields of a real 3D field: scalars and z components
    real, F_- = conj(F_+) (F_r, F_theta real)."""
    rng = np.random.default_rng(seed)
    def cplx():
        return rng.standard_normal((nr, nz)) + 1j * rng.standard_normal((nr, nz))
    out = {}
    for name in ("E", "B", "J"):
        fp = cplx()
        out[name] = (fp, np.conj(fp), rng.standard_normal((nr, nz)) + 0j)
    out["rho0"] = rng.standard_normal((nr, nz)) + 0j
    out["rho1"] = rng.standard_normal((nr, nz)) + 0j
    return out


@pytest.mark.parametrize("order", [0, 8, 32])
def test_psatd_keeps_a_real_field_real(order):
    # mode 0 of a real field has real scalars and z components and
    # F_- = conj(F_+); one PSATD step (forward transforms, Eqs. (1a)-(1b),
    # inverse transforms) must keep that structure at every stencil order.
    # At infinite order this needs a zero derivative symbol in the Nyquist
    # column: with [k_z] = -pi/dz there, i [k_z] turns the real Nyquist
    # coefficient of a real sequence imaginary (checked last)
    nz, nr, dz, dt = 32, 12, 0.1, 0.1
    st = _real_mode0_state(nz, nr, seed=order + 5)
    hk = sp.HankelPair(0, nr, 0.1)
    nus = sp.hankel_orders(0)
    kp = hk.k[:, None]

    def step(kzm):
        fw = {k: tuple(hk.forward(st[k][c], nus[c]) for c in range(3)) for k in ("E", "B", "J")}
        r0, r1 = hk.forward(st["rho0"], 0), hk.forward(st["rho1"], 0)
        En, Bn = sp.psatd_push(fw["E"], fw["B"], fw["J"], r0, r1, dt, kp, kzm)
        return ([hk.backward(En[c], nus[c]) for c in range(3)],
                [hk.backward(Bn[c], nus[c]) for c in range(3)])

    kzm = sp.kz_modified(sp.kz_grid(nz, dz), dz, order)[None, :]
    E, B = step(kzm)
    for F in (E, B):
        scale = max(np.abs(f).max() for f in F)
        assert np.abs(F[2].imag).max() < 1e-12 * scale
        assert np.abs(F[1] - np.conj(F[0])).max() < 1e-12 * scale
    if order == 0:
        raw = sp.kz_grid(nz, dz)[None, :]          # Nyquist column left at -pi/dz
        E, _ = step(raw)
        assert np.abs(E[2].imag).max() > 1e-3 * np.abs(E[2]).max()
