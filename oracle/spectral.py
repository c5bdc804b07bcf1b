"""Spectral side of the oracle (FP64): grids, finite-order wavenumber, Hankel
transform pair, quasi-cylindrical spectral operators, current correction and
the PSATD update.

Conventions (the paper's operator table fixes them, see the notes below):
  * a field is F(r, theta, z) = sum_{m=-M..M} F_m(r, z) exp(-i m theta) with
    F_{-m} = conj(F_m) for real fields;
  * vector fields are carried as F_+ = (F_r - i F_theta)/2,
    F_- = (F_r + i F_theta)/2 and F_z; in mode m the Hankel order of F_+ is
    m + 1, of F_- is m - 1 and of F_z (and of scalars) is m;
  * plasma units, c = 1: the paper's Eqs. (1a)-(1b) are written with the
    vacuum permittivity set to one and B standing for cB, which is exactly the
    form they take in these units.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np
from scipy.special import jv, jn_zeros

KPERP_J0_ZEROS, KPERP_SINE, KPERP_JM_ZEROS = 0, 1, 2


# ---------------------------------------------------------------------------
# Finite-order modification (paper, Sec. "Finite order pseudo-spectral
# solvers", Eq. (3) and Eq. (5))
# ---------------------------------------------------------------------------
def fornberg_alpha_exact(n: int):
    """Centered stencil coefficients alpha_{n,j}, j = 1..n, of the order-2n
    first derivative, Eq. (3): (-1)^(j+1) 2 (n!)^2 / ((n-j)! (n+j)!), exact."""
    return [Fraction((-1) ** (j + 1) * 2 * factorial(n) ** 2,
                     factorial(n - j) * factorial(n + j)) for j in range(1, n + 1)]


def fornberg_alpha(n: int) -> np.ndarray:
    return np.array([float(a) for a in fornberg_alpha_exact(n)], dtype=np.float64)


def kz_grid(nz: int, dz: float) -> np.ndarray:
    """Discrete longitudinal wavenumbers of a periodic z grid (FFT order,
    Nyquist at -pi/dz)."""
    return 2.0 * np.pi * np.fft.fftfreq(nz, dz)


def kz_modified(kz: np.ndarray, dz: float, order: int) -> np.ndarray:
    """Modified wavenumber [k_z] = sum_j alpha_{n,j} sin(k_z j dz)/(j dz),
    Eq. (5), with stencil order p = 2n.  order == 0 stands for the infinite
    order (unmodified k_z, zero at the Nyquist wavenumber)."""
    kz = np.asarray(kz, dtype=np.float64)
    if order == 0:
        # infinite order: k_z itself, except at the z Nyquist wavenumber pi/dz,
        # where k_z and -k_z are the same grid mode.  There the odd symbol of a
        # first derivative must vanish (else a real field picks up an
        # imaginary part), which is also the limit of every finite order of
        # Eq. (5): sin(pi j) = 0 for all j.
        out = kz.copy()
        out[np.abs(np.abs(kz * dz) - np.pi) <= 1e-12 * np.pi] = 0.0
        return out
    if order < 2 or order % 2:
        raise ValueError("stencil order must be even and >= 2 (or 0 for infinite)")
    n = order // 2
    alpha = fornberg_alpha(n)
    out = np.zeros_like(kz)
    for j in range(1, n + 1):
        out += alpha[j - 1] * np.sin(kz * j * dz) / (j * dz)
    return out


# ---------------------------------------------------------------------------
# Radial grid and discrete Hankel transform pair (the paper names a Hankel
# transform along r for the quasi-cylindrical scheme; the discrete pair is
# this implementation's reading, see the design notes)
# ---------------------------------------------------------------------------
def r_grid(nr: int, dr: float) -> np.ndarray:
    """Cell-centred radial nodes r_i = (i + 1/2) dr."""
    return (np.arange(nr, dtype=np.float64) + 0.5) * dr


def kperp_grid(m: int, nr: int, dr: float, kind: int = KPERP_JM_ZEROS) -> np.ndarray:
    """Radial wavenumbers of mode m (all strictly positive).

    KPERP_JM_ZEROS (default): k_i = j_{m,i}/R.  At the zeros of J_m the three
      bases J_{m-1}(k r), J_m(k r), J_{m+1}(k r) of the (-, z, +) components all
      satisfy Dini boundary conditions at R and have the same norm
      (R^2/2) J_{m+1}(k R)^2 for every k, so the energy the spectral PSATD
      update conserves, sum_k N_k (2|E+|^2 + 2|E-|^2 + |Ez|^2), is the field
      energy the particles exchange with.  The order-0 basis of mode 1
      (Neumann at R) misses the constant eigenfunction, which leaves one
      near-null direction in its synthesis matrix (see HankelPair).
    KPERP_J0_ZEROS: k_i = j_{0,i}/R for every mode.  Well conditioned, but the
      order-2 basis of mode 1 is neither orthogonal nor of equal norm, and
      mode 1 then grows without bound in a beam-plasma run.
    KPERP_SINE: k_i = (i + 1) pi / R (a poor interpolant; for comparison)."""
    R = nr * dr
    if kind == KPERP_SINE:
        return (np.arange(nr, dtype=np.float64) + 1.0) * np.pi / R
    if kind == KPERP_JM_ZEROS:
        return jn_zeros(m, nr) / R
    if kind == KPERP_J0_ZEROS:
        return jn_zeros(0, nr) / R
    raise ValueError(kind)


def bessel_synthesis(nu: int, r: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Backward (synthesis) matrix B_nu[i_r, i_k] = J_nu(k_ik r_ir)."""
    return jv(nu, np.outer(r, k))


# singular values of a synthesis matrix below this fraction of its largest are
# dropped from the forward transform
PINV_RCOND = 1e-4


class HankelPair:
    """Backward B_nu and forward F_nu matrices of one mode for the three orders
    nu = m - 1, m, m + 1 used by F_-, scalars/F_z and F_+.

    F_nu is the Moore-Penrose pseudo-inverse of B_nu with singular values below
    PINV_RCOND * sigma_max dropped.  For the default grid this is the exact
    inverse except for isolated near-null directions (mode 1, order 0: the
    constant eigenfunction its Neumann basis lacks; higher modes: near-axis
    orders), which are projected out instead of amplified."""

    def __init__(self, m: int, nr: int, dr: float, kind: int = KPERP_JM_ZEROS):
        self.m = m
        self.r = r_grid(nr, dr)
        self.k = kperp_grid(m, nr, dr, kind)
        self.B = {}
        self.F = {}
        for nu in (m - 1, m, m + 1):
            B = bessel_synthesis(nu, self.r, self.k)
            self.B[nu] = B
            self.F[nu] = np.linalg.pinv(B, rcond=PINV_RCOND)

    def forward(self, g: np.ndarray, nu: int) -> np.ndarray:
        """Real space [r, z] -> spectral [k_perp, k_z]: FFT along z, then F_nu."""
        return self.F[nu] @ np.fft.fft(g, axis=-1)

    def backward(self, gh: np.ndarray, nu: int) -> np.ndarray:
        """Spectral [k_perp, k_z] -> real space [r, z]: B_nu, then inverse FFT."""
        return np.fft.ifft(self.B[nu] @ gh, axis=-1)


# ---------------------------------------------------------------------------
# Quasi-cylindrical spectral operators (paper, Eqs. (2a)-(2b)); kp broadcasts
# along k_perp (shape [Nr, 1]), kzm is [k_z] (shape [1, Nz]).
# ---------------------------------------------------------------------------
def grad(s, kp, kzm):
    """Spectral gradient of a scalar, Eq. (2a): (-kp s/2, +kp s/2, i[k_z] s)."""
    return (-kp * s / 2.0, kp * s / 2.0, 1j * kzm * s)


def curl(v, kp, kzm):
    """Spectral curl of a vector (V_+, V_-, V_z), Eq. (2b)."""
    vp, vm, vz = v
    return (kzm * vp - 1j * kp * vz / 2.0,
            -kzm * vm - 1j * kp * vz / 2.0,
            1j * kp * (vp + vm))


def div(v, kp, kzm):
    """Spectral divergence consistent with Eqs. (2a)-(2b):
    kp (V_+ - V_-) + i[k_z] V_z, so that div(grad s) = -(kp^2 + [k_z]^2) s."""
    vp, vm, vz = v
    return kp * (vp - vm) + 1j * kzm * vz


def current_correction(J, rho_old, rho_new, dt, kp, kzm):
    """Spectral current correction: J <- J + grad F with
    F = (div J + (rho_new - rho_old)/dt) / k^2, so that afterwards
    div J = -(rho_new - rho_old)/dt exactly (the paper requires charge
    conservation, Sec. "Finite order pseudo-spectral solvers"; this is its
    global spectral form on one domain)."""
    k2 = kp ** 2 + kzm ** 2
    F = (div(J, kp, kzm) + (rho_new - rho_old) / dt) / k2
    g = grad(F, kp, kzm)
    return tuple(J[c] + g[c] for c in range(3))


def psatd_push(E, B, J, rho_old, rho_new, dt, kp, kzm):
    """One PSATD step, Eqs. (1a)-(1b) with the operators of Eqs. (2a)-(2b)
    and k_z replaced by [k_z] everywhere, including inside k, C and S.

    E^{n+1} = C E + (S/k) curl B - (S/k) J
              + (1/k^2) grad[(S/(k dt) - 1) rho_new + (C - S/(k dt)) rho_old]
    B^{n+1} = C B - (S/k) curl E + ((1 - C)/k^2) curl J
    """
    k = np.sqrt(kp ** 2 + kzm ** 2)
    C = np.cos(k * dt)
    S = np.sin(k * dt)
    x = k * dt
    cB = curl(B, kp, kzm)
    cE = curl(E, kp, kzm)
    cJ = curl(J, kp, kzm)
    g = grad((S / x - 1.0) * rho_new + (C - S / x) * rho_old, kp, kzm)
    En = tuple(C * E[c] + (S / k) * cB[c] - (S / k) * J[c] + g[c] / k ** 2 for c in range(3))
    Bn = tuple(C * B[c] - (S / k) * cE[c] + ((1.0 - C) / k ** 2) * cJ[c] for c in range(3))
    return En, Bn


# --- Galilean PSATD (the scheme the paper names as intrinsically stable for
# drifting plasmas, Sec. "Finite order pseudo-spectral solvers") -------------
# Fields expressed in coordinates z' = z - v t that move with the grid obey
# Maxwell's equations plus the advection term v d/dz', which in spectral form
# adds i w F with w = [k_z] v (the same order-p derivative as in Maxwell's
# curl).  With J constant over the step in those coordinates the update is the
# exact solution of
#   dE/dt = curl B - J + i w E,   dB/dt = -curl E + i w B,
#   d rho/dt = -div J + i w rho  (continuity in the moving coordinates).
def phase_integral(a, dt):
    """int_0^dt exp(i a u) du = dt exp(i a dt/2) sinc(a dt/2)."""
    return dt * np.exp(0.5j * a * dt) * np.sinc(a * dt / (2.0 * np.pi))


def galilean_coefficients(kp, kzm, dt, v):
    """theta^2 = exp(i w dt), C, S, and the source integrals
    X1 = int_0^dt exp(i w u) cos(k u) du, X2 = int_0^dt exp(i w u) sin(k u) du,
    phi = int_0^dt exp(i w u) du, with w = [k_z] v, k = sqrt(k_perp^2 + [k_z]^2)."""
    k = np.sqrt(kp ** 2 + kzm ** 2)
    w = kzm * v
    pp, pm = phase_integral(w + k, dt), phase_integral(w - k, dt)
    return (np.exp(1j * w * dt), np.cos(k * dt), np.sin(k * dt), 0.5 * (pp + pm), (pp - pm) / 2j,
            phase_integral(w, dt))


def current_correction_galilean(J, rho_old, rho_new, dt, kp, kzm, v):
    """J <- J + grad F with F chosen so that afterwards
    div J = (theta^2 rho_old - rho_new) / phi, the continuity equation in the
    moving coordinates integrated over the step with J constant
    (rho_new = theta^2 rho_old - phi div J)."""
    th2, _, _, _, _, ph = galilean_coefficients(kp, kzm, dt, v)
    k2 = kp ** 2 + kzm ** 2
    F = (div(J, kp, kzm) + (rho_new - th2 * rho_old) / ph) / k2
    g = grad(F, kp, kzm)
    return tuple(J[c] + g[c] for c in range(3))


def psatd_push_galilean(E, B, J, rho_old, rho_new, dt, kp, kzm, v):
    """One Galilean PSATD step (rho_old, E, B on the grid at t^n; rho_new on the
    grid at t^{n+1}; J in the moving coordinates):
      E' = th2 C E + th2 (S/k) curl B - X1 J
           + (1/k^2) grad[(X1/phi - 1) rho_new + th2 (C - X1/phi) rho_old]
      B' = th2 C B - th2 (S/k) curl E + (X2/k) curl J
    The transverse part is the exact solution above; the longitudinal part is
    fixed by Gauss's law at t^{n+1} given Gauss's law at t^n and the continuity
    of current_correction_galilean.  v = 0 gives psatd_push."""
    th2, C, S, X1, X2, ph = galilean_coefficients(kp, kzm, dt, v)
    k = np.sqrt(kp ** 2 + kzm ** 2)
    cB = curl(B, kp, kzm)
    cE = curl(E, kp, kzm)
    cJ = curl(J, kp, kzm)
    g = grad((X1 / ph - 1.0) * rho_new + th2 * (C - X1 / ph) * rho_old, kp, kzm)
    En = tuple(th2 * C * E[c] + th2 * (S / k) * cB[c] - X1 * J[c] + g[c] / k ** 2 for c in range(3))
    Bn = tuple(th2 * C * B[c] - th2 * (S / k) * cE[c] + (X2 / k) * cJ[c] for c in range(3))
    return En, Bn


def galilean_translations(kz, dz, n_shift=1.0):
    """Spectral factors that move a field from the grid at t^n to the grid
    n_shift cells ahead (periodic along z): exp(i k_z n_shift dz) on the DFT
    wavenumbers, for whole and half cells.  A half-cell move of the Nyquist
    component of a real signal has no real value; it is taken as the average of
    its two readings, cos(pi/2) = 0 (as the derivative symbol there)."""
    kz = np.asarray(kz)
    one = np.exp(1j * kz * dz * n_shift)
    half = np.exp(0.5j * kz * dz * n_shift)
    nyq = np.abs(np.abs(kz * dz) - np.pi) <= 1e-12 * np.pi
    half = np.where(nyq, 0.0, half)
    return one, half


def binomial_filter(kz, dz, kperp, dr, passes=1):
    """`passes` (1/4, 1/2, 1/4) smoothing passes along z and along r in spectral
    form, [cos^2(k_z dz/2) cos^2(k_perp dr/2)]^passes, shape [k_perp, k_z] (an
    option of the field update, not part of the paper's scheme)."""
    f = np.cos(0.5 * np.asarray(kperp)[:, None] * dr) ** 2 * np.cos(0.5 * np.asarray(kz)[None, :] * dz) ** 2
    return f ** passes


def hankel_orders(m: int):
    """Hankel orders of the (+, -, z) components of mode m."""
    return (m + 1, m - 1, m)
