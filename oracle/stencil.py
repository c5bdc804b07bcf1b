"""Stencil reach and numerical dispersion of the order-p PSATD solver (FP64).

* stencil_profile: the real-space reach of the update operators along z,
  obtained by inverse-transforming C and the two S-weighted direction
  cosines (paper, Sec. "Finite order pseudo-spectral solvers", Eq. (6); the
  printed formula is garbled, the reading used here is
  alpha* = sqrt(|IFFT(C)|^2 + |IFFT(S k_perp/k)|^2 + |IFFT(S [k_z]/k)|^2)).
* phase_velocity / resonance_kz: the vacuum dispersion
  omega^2 = k_perp^2 + [k_z]^2 (Eq. (8)) and the numerical Cherenkov
  resonance v_beam = sqrt(k_perp^2 + [k_z]^2)/k_z (Eq. (10)).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

from .spectral import kz_grid, kz_modified


def stencil_profile(order: int, kperp: float, dz: float, dt: float, nz: int = 1024):
    """|alpha*| as a function of the cell distance 0..nz/2 (c = 1)."""
    kz = kz_grid(nz, dz)
    kzm = kz_modified(kz, dz, order)
    k = np.sqrt(kperp ** 2 + kzm ** 2)
    C = np.cos(k * dt)
    S = np.sin(k * dt)
    a = np.abs(np.fft.ifft(C)) ** 2 + np.abs(np.fft.ifft(S * kperp / k)) ** 2 \
        + np.abs(np.fft.ifft(S * kzm / k)) ** 2
    return np.sqrt(a)[: nz // 2 + 1]


def stencil_extent(order: int, kperp: float, dz: float, dt: float, floor: float = 1e-15,
                   nz: int = 1024) -> int:
    """First cell distance at which alpha*/alpha*(0) falls below `floor`."""
    prof = stencil_profile(order, kperp, dz, dt, nz)
    rel = prof / prof[0]
    below = np.nonzero(rel < floor)[0]
    return int(below[0]) if below.size else nz // 2


def phase_velocity_z(kz, kperp, dz, order):
    """omega / k_z with omega = sqrt(k_perp^2 + [k_z]^2) (c = 1)."""
    kzm = kz_modified(np.asarray(kz, np.float64), dz, order)
    return np.sqrt(kperp ** 2 + kzm ** 2) / kz


def resonance_kz(gamma: float, order: int, dz: float, kperp: float = 0.0) -> float:
    """Smallest k_z in (0, pi/dz) where the modified-dispersion phase velocity
    equals the beam velocity beta = sqrt(1 - 1/gamma^2) (Eq. (10))."""
    beta = np.sqrt(1.0 - 1.0 / gamma ** 2)

    def f(kz):
        return float(phase_velocity_z(kz, kperp, dz, order)) - beta

    grid = np.linspace(1e-6, np.pi / dz * (1.0 - 1e-9), 20001)   # the open interval (0, pi/dz)
    vals = np.array([f(k) for k in grid])
    idx = np.nonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    if idx.size == 0:
        return float("nan")
    i = idx[0]
    return brentq(f, grid[i], grid[i + 1], xtol=1e-14)
