"""Pins of the Galilean PSATD step (fields in coordinates moving with the
grid at velocity v along z): the exact solution of the moving-frame ODE
(matrix exponential), Gauss's law and continuity in the moving frame, the
stationary field of a charge that moves with the grid, and the translations
that carry the sources onto the moving grid."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import spectral as sp
from workloads import random_spectral


def _curl_matrix(kp, kzm):
    return np.array([[kzm, 0, -0.5j * kp], [0, -kzm, -0.5j * kp], [1j * kp, 1j * kp, 0]])


def test_galilean_step_equals_exact_moving_frame_solution():
    # with Gauss-consistent inputs (div E = rho^n) and rho^{n+1} from the
    # moving-frame continuity equation, the step is the exact solution of
    # dE/dt = curl B - J + i w E, dB/dt = -curl E + i w B (J constant)
    rng = np.random.default_rng(11)
    worst = 0.0
    for trial in range(300):
        kp = rng.uniform(0.01, 5.0)
        kzm = rng.uniform(-5.0, 5.0)
        dt = rng.uniform(0.005, 0.8)
        v = rng.uniform(-1.0, 1.0) if trial % 3 else 1.0
        E = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        B = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        J = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        kvec_div = np.array([kp, -kp, 1j * kzm])
        g = np.array([-kp / 2, kp / 2, 1j * kzm])
        B = B - g * (kvec_div @ B) / (kvec_div @ g)
        w = kzm * v
        rho0 = kvec_div @ E
        # rho(dt) of d rho/dt = -div J + i w rho, written out
        rho1 = np.exp(1j * w * dt) * rho0 - (kvec_div @ J) * (np.expm1(1j * w * dt) / (1j * w) if w else dt)
        K = _curl_matrix(kp, kzm)
        A = np.zeros((7, 7), complex)
        A[0:3, 3:6] = K
        A[3:6, 0:3] = -K
        A[0:6, 0:6] += 1j * w * np.eye(6)
        A[0:3, 6] = -J
        y = expm(A * dt) @ np.concatenate([E, B, [1.0]])
        En, Bn = sp.psatd_push_galilean(tuple(E), tuple(B), tuple(J), rho0, rho1, dt, kp, kzm, v)
        got = np.concatenate([np.array(En), np.array(Bn)])
        worst = max(worst, np.abs(got - y[:6]).max() / np.abs(y[:6]).max())
    assert worst < 1e-11


def _rand_cells(seed, shape=(6, 10)):
    fields = [random_spectral(shape, seed + i) for i in range(11)]
    rng = np.random.default_rng(seed)
    kp = rng.uniform(0.05, 4.0, (shape[0], 1))
    kzm = rng.uniform(-4.0, 4.0, (1, shape[1]))
    return fields, kp, kzm


@pytest.mark.parametrize("v", [0.5, 1.0])
def test_galilean_continuity_and_gauss(v):
    f, kp, kzm = _rand_cells(3)
    E, B, J = tuple(f[0:3]), tuple(f[3:6]), tuple(f[6:9])
    r0, r1 = f[9], f[10]
    dt = 0.3
    th2, C, _, _, _, ph = sp.galilean_coefficients(kp, kzm, dt, v)
    Jc = sp.current_correction_galilean(J, r0, r1, dt, kp, kzm, v)
    # continuity in the moving frame: rho1 = th2 rho0 - phi div J
    np.testing.assert_allclose(r1, th2 * r0 - ph * sp.div(Jc, kp, kzm), atol=1e-12)
    # Gauss's law error is carried along and scaled by th2 C, as C in the lab frame
    En, Bn = sp.psatd_push_galilean(E, B, Jc, r0, r1, dt, kp, kzm, v)
    np.testing.assert_allclose(sp.div(En, kp, kzm) - r1, th2 * C * (sp.div(E, kp, kzm) - r0), atol=1e-11)
    np.testing.assert_allclose(sp.div(Bn, kp, kzm), th2 * C * sp.div(B, kp, kzm), atol=1e-11)


@pytest.mark.parametrize("v", [0.9, 0.999, 1.0])
def test_field_of_a_charge_moving_with_the_grid_is_stationary(v):
    # a rigid charge moving at the grid's velocity is at rest in the moving
    # coordinates: rho^{n+1} = rho^n, J_z = v rho, and its own field (the
    # relativistic Poisson solution of the same operators) must not change,
    # step after step -- no numerical Cherenkov radiation from such a beam
    rng = np.random.default_rng(21)
    kp = rng.uniform(0.05, 4.0, (8, 1))
    kz = sp.kz_grid(32, 0.1)[None, :]
    for order in (0, 8, 32):
        kzm = sp.kz_modified(kz, 0.1, order)
        rho = random_spectral((8, 32), 5)
        ig2 = 1.0 - v * v
        phi = rho / (kp ** 2 + kzm ** 2 * ig2)
        gph = sp.grad(phi, kp, kzm)
        E = (-gph[0], -gph[1], -gph[2] * ig2)
        B = (-1j * v * E[0], 1j * v * E[1], np.zeros_like(phi))
        J = (np.zeros_like(rho), np.zeros_like(rho), v * rho)
        E1, B1 = E, B
        for _ in range(20):
            Jc = sp.current_correction_galilean(J, rho, rho, 0.1, kp, kzm, v)
            E1, B1 = sp.psatd_push_galilean(E1, B1, Jc, rho, rho, 0.1, kp, kzm, v)
        scale = max(np.abs(np.array(E)).max(), np.abs(np.array(B)).max())
        assert np.abs(np.array(E1) - np.array(E)).max() < 1e-11 * scale, order
        assert np.abs(np.array(B1) - np.array(B)).max() < 1e-11 * scale, order
    # the lab-frame update (v = 0) does move such a field
    E0, _ = sp.psatd_push(E, B, J, rho, rho - 0.1 * sp.div(J, kp, kzm), 0.1, kp, kzm)
    assert np.abs(np.array(E0) - np.array(E)).max() > 1e-3 * scale


def test_translations_onto_the_moving_grid():
    rng = np.random.default_rng(4)
    nz, dz = 64, 0.1
    kz = sp.kz_grid(nz, dz)
    x = rng.standard_normal((3, nz))
    one, half = sp.galilean_translations(kz, dz)
    # one cell: node j of the new grid is node j + 1 of the old one (periodic)
    np.testing.assert_allclose(np.fft.ifft(one * np.fft.fft(x, axis=-1), axis=-1).real, np.roll(x, -1, axis=-1),
                               atol=1e-13)
    # half a cell keeps a real signal real, and twice half a cell is one cell
    # for a signal without a Nyquist component
    y = np.fft.ifft(half * np.fft.fft(x, axis=-1), axis=-1)
    assert np.abs(y.imag).max() < 1e-13
    xf = np.fft.fft(x, axis=-1)
    xf[:, nz // 2] = 0.0
    x2 = np.fft.ifft(half * half * xf, axis=-1).real
    np.testing.assert_allclose(x2, np.roll(np.fft.ifft(xf, axis=-1).real, -1, axis=-1), atol=1e-13)


def test_galilean_cycle_keeps_the_field_of_a_comoving_beam():
    # the full cycle (gather, push, deposit, transforms, update, window): a
    # quiet gamma = 1000 beam moving with the window keeps its own field under
    # the Galilean update, up to its O(1/gamma^2) slip behind the grid, while
    # the lab-frame update with the window shift changes it three orders of
    # magnitude more
    from oracle.cycle import OracleSim
    from workloads import Workload, KPERP_JM_ZEROS, quiet_beam
    change = {}
    for gal in (True, False):
        b = quiet_beam("beam", 1000.0, 0.05, 128, 32, 0.05, 0.05, 3.2, 0.5, 0.2)
        wl = Workload("beam", 128, 32, 2, 16, 0.05, 0.05, 0.05, 0.0, True, KPERP_JM_ZEROS, 1, [b], galilean=gal)
        o = OracleSim(wl)
        E0 = o.E[0].copy()
        o.step(20)
        change[gal] = np.linalg.norm(o.E[0] - E0) / np.linalg.norm(E0)
    assert change[True] < 2e-6
    assert change[False] > 1e-3
