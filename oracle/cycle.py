"""The oracle's PIC cycle (FP64, plain NumPy).

The state is spectral: per mode, Eh and Bh hold E^n and B^n on the
(k_perp, k_z) grid (momenta live at half-integer times).  E and B hold the
real-space fields the particles see.  Per step n:
  1. gather E^n, B^n at x^n, Boris push u^{n-1/2} -> u^{n+1/2},
     move x^{n+1} = x^n + dt v^{n+1/2};
  2. deposit rho^n at x^n, J^{n+1/2} at x^{n+1/2} = (x^n + x^{n+1})/2 with
     v^{n+1/2}, rho^{n+1} at x^{n+1} (the time levels the paper's Eq. (1a)
     uses), immobile species included in both densities;
  3. forward transforms (FFT along z, discrete Hankel along r) of J, rho^n,
     rho^{n+1};
  4. spectral current correction, then the order-p PSATD update of Eh, Bh;
  5. inverse transforms of Eh, Bh to real space E, B;
  6. moving window (when enabled): zmin advances by dz; the real-space fields
     shift one cell toward the tail and the head column is zeroed; the
     spectral state gets the same shift, Fh <- exp(i k_z dz) (Fh - Hankel
     transform of the departed tail column); particles behind the new zmin
     are removed and a fresh lattice column is injected at the head;
  7. absorbing layers (when enabled, `damp_cells` = N > 0): the real-space
     E, B at the N nodes nearest each z end are multiplied by
     sin^2(pi s / (2N)), s the node's distance in cells from the end node,
     and the damped real-space fields become the state (forward transformed
     at the next spectral push).
Galilean variant (`galilean`, with the moving window): the fields live in
coordinates moving with the grid (v = dz/dt, one cell per step); at step 4
rho^{n+1} is moved onto the grid at t^{n+1} (one cell) and J onto the grid at
t^{n+1/2} (half a cell) in spectral form, the current correction and the
update are the Galilean ones (spectral.psatd_push_galilean), and at step 6 the
fields are not shifted (they already are on the moved grid).

Fields written in real space with set_fields() become the state at the next
spectral push (they are forward transformed then).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import spectral as sp
from . import particles as pt


@dataclasses.dataclass
class OSpecies:
    name: str
    q: float
    m: float
    mobile: bool
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    w: np.ndarray
    inject: bool
    ppc: tuple
    density: float
    diag: bool


def damping_profile(nz: int, n: int) -> np.ndarray:
    """Per-node factor of the absorbing layers: sin^2(pi s / (2n)) at the n
    nodes nearest each end (s = distance in cells from the end node), 1 in
    between."""
    w = np.ones(nz)
    s = np.arange(n)
    ramp = np.sin(0.5 * np.pi * s / n) ** 2
    w[:n] = ramp
    w[nz - 1 - s] = ramp
    return w


class OracleSim:
    def __init__(self, wl, current_correction: bool = True):
        self.nz, self.nr, self.M = wl.nz, wl.nr, wl.n_modes
        self.dz, self.dr, self.dt = wl.dz, wl.dr, wl.dt
        self.zmin0 = wl.zmin
        self.zmin = wl.zmin
        self.order = wl.order
        self.moving_window = wl.moving_window
        self.correct = current_correction
        self.filter = int(getattr(wl, "filter", 0))
        self.damp = int(getattr(wl, "damp_cells", 0))
        self.galilean = bool(getattr(wl, "galilean", False))
        self.shape = int(getattr(wl, "shape_order", 1))
        self.n_shift = 0
        self.hankel = [sp.HankelPair(m, wl.nr, wl.dr, wl.kperp_grid) for m in range(self.M)]
        self.kzm = sp.kz_modified(sp.kz_grid(wl.nz, wl.dz), wl.dz, wl.order)[None, :]
        self.kz = sp.kz_grid(wl.nz, wl.dz)
        shape = (self.M, 3, self.nr, self.nz)
        self.Eh = np.zeros(shape, dtype=np.complex128)
        self.Bh = np.zeros(shape, dtype=np.complex128)
        self.E = np.zeros(shape, dtype=np.complex128)
        self.B = np.zeros(shape, dtype=np.complex128)
        self._real_pending = False
        self.species: List[OSpecies] = []
        for s in wl.species:
            self.species.append(OSpecies(
                s.name, s.q, s.m, s.mobile,
                s.x.astype(np.float64).copy(), s.y.astype(np.float64).copy(),
                s.z.astype(np.float64).copy(),
                s.ux.astype(np.float64), s.uy.astype(np.float64), s.uz.astype(np.float64),
                s.w.astype(np.float64), s.inject, tuple(s.ppc), s.density, s.diag))
        # last step's intermediates (exposed for stage-by-stage parity tests)
        self.J = None
        self.rho_old = None
        self.rho_new = None
        for s in wl.species:
            if getattr(s, "self_field", False) and s.mobile and s.x.size:
                self.add_beam_field(s)
        # with absorbing layers the real-space fields are the state from the start
        self._real_pending = self.damp > 0

    def add_beam_field(self, s):
        """Add the field of a cold beam's charge moving rigidly along z at its
        weighted mean u_z (relativistic spectral Poisson equation): phi =
        rho / (k_perp^2 + [k_z]^2 / gamma^2), E = -grad phi with E_z scaled by
        1 / gamma^2 (Eq. (2a)), B_theta = beta E_r, i.e. B_+ = -i beta E_+,
        B_- = +i beta E_-, B_z = 0."""
        w = s.w.astype(np.float64)
        ubar = float((w * s.uz.astype(np.float64)).sum() / w.sum())
        gam = np.sqrt(1.0 + ubar * ubar)
        beta = ubar / gam
        rho = pt.deposit_rho(self.M, s.q * w, s.x.astype(np.float64), s.y.astype(np.float64),
                             s.z.astype(np.float64), self.grid())
        for m in range(self.M):
            hk = self.hankel[m]
            kp = hk.k[:, None]
            phi = hk.forward(rho[m], m) / (kp ** 2 + self.kzm ** 2 / gam ** 2)
            g = sp.grad(phi, kp, self.kzm)
            E = (-g[0], -g[1], -g[2] / gam ** 2)
            B = (-1j * beta * E[0], 1j * beta * E[1], np.zeros_like(phi))
            nus = sp.hankel_orders(m)
            for c in range(3):
                self.Eh[m, c] += E[c]
                self.Bh[m, c] += B[c]
                self.E[m, c] = hk.backward(self.Eh[m, c], nus[c])
                self.B[m, c] = hk.backward(self.Bh[m, c], nus[c])

    # -- helpers -----------------------------------------------------------
    def set_fields(self, E=None, B=None):
        """Write real-space fields [M, 3, nr, nz] (components +, -, z); they
        replace the spectral state at the next spectral push."""
        if E is not None:
            self.E[:] = E
        if B is not None:
            self.B[:] = B
        self._real_pending = True

    def grid(self):
        return {"nz": self.nz, "nr": self.nr, "dz": self.dz, "dr": self.dr, "zmin": self.zmin,
                "shape": self.shape}

    # -- stage 1: gather + push -------------------------------------------
    def gather_push(self):
        g = self.grid()
        for s in self.species:
            if not s.mobile:
                s.xn = (s.x, s.y, s.z)
                continue
            s.xn = (s.x.copy(), s.y.copy(), s.z.copy())
            Ex, Ey, Ez = pt.gather_cartesian(self.E, s.x, s.y, s.z, g)
            Bx, By, Bz = pt.gather_cartesian(self.B, s.x, s.y, s.z, g)
            s.ux, s.uy, s.uz = pt.boris(s.ux, s.uy, s.uz, Ex, Ey, Ez, Bx, By, Bz,
                                        s.q, s.m, self.dt)
            ginv = 1.0 / np.sqrt(1.0 + s.ux ** 2 + s.uy ** 2 + s.uz ** 2)
            s.vx, s.vy, s.vz = s.ux * ginv, s.uy * ginv, s.uz * ginv
            s.x = s.x + self.dt * s.vx
            s.y = s.y + self.dt * s.vy
            s.z = s.z + self.dt * s.vz

    # -- stage 2: deposit -------------------------------------------------
    def deposit(self):
        g = self.grid()
        M = self.M
        rho_old = np.zeros((M, self.nr, self.nz), np.complex128)
        rho_new = np.zeros_like(rho_old)
        J = np.zeros((M, 3, self.nr, self.nz), np.complex128)
        for s in self.species:
            qw = s.q * s.w
            xo, yo, zo = s.xn
            rho_old += pt.deposit_rho(M, qw, xo, yo, zo, g)
            rho_new += pt.deposit_rho(M, qw, s.x, s.y, s.z, g)
            if s.mobile:
                xh, yh, zh = 0.5 * (xo + s.x), 0.5 * (yo + s.y), 0.5 * (zo + s.z)
                J += pt.deposit_current(M, qw, xh, yh, zh, s.vx, s.vy, s.vz, g)
        self.J, self.rho_old, self.rho_new = J, rho_old, rho_new

    # -- stage 3-5: spectral push -----------------------------------------
    def spectral_push(self):
        for m in range(self.M):
            hk = self.hankel[m]
            kp = hk.k[:, None]
            nus = sp.hankel_orders(m)
            if self._real_pending:
                for c in range(3):
                    self.Eh[m, c] = hk.forward(self.E[m, c], nus[c])
                    self.Bh[m, c] = hk.forward(self.B[m, c], nus[c])
            Jh = tuple(hk.forward(self.J[m, c], nus[c]) for c in range(3))
            r0 = hk.forward(self.rho_old[m], m)
            r1 = hk.forward(self.rho_new[m], m)
            if self.galilean:
                # the grid moves one cell per step: rho^{n+1} onto the grid at
                # t^{n+1}, J onto the grid at t^{n+1/2}
                one, half = sp.galilean_translations(self.kz, self.dz)
                r1 = one[None, :] * r1
                Jh = tuple(half[None, :] * j for j in Jh)
            if self.filter:
                f = sp.binomial_filter(self.kz, self.dz, hk.k, self.dr, self.filter)
                Jh = tuple(f * j for j in Jh)
                r0, r1 = f * r0, f * r1
            if self.galilean:
                v = self.dz / self.dt
                if self.correct:
                    Jh = sp.current_correction_galilean(Jh, r0, r1, self.dt, kp, self.kzm, v)
                En, Bn = sp.psatd_push_galilean(tuple(self.Eh[m]), tuple(self.Bh[m]), Jh, r0, r1, self.dt, kp,
                                                self.kzm, v)
            else:
                if self.correct:
                    Jh = sp.current_correction(Jh, r0, r1, self.dt, kp, self.kzm)
                En, Bn = sp.psatd_push(tuple(self.Eh[m]), tuple(self.Bh[m]), Jh, r0, r1, self.dt, kp, self.kzm)
            for c in range(3):
                self.Eh[m, c] = En[c]
                self.Bh[m, c] = Bn[c]
                self.E[m, c] = hk.backward(En[c], nus[c])
                self.B[m, c] = hk.backward(Bn[c], nus[c])
        self._real_pending = False
        if self.moving_window:
            self.move_window()
        if self.damp:
            self.damp_edges()

    # -- stage 7: absorbing layers ----------------------------------------
    def damp_edges(self):
        w = damping_profile(self.nz, self.damp)
        self.E *= w
        self.B *= w
        self._real_pending = True

    # -- stage 6: moving window -------------------------------------------
    def move_window(self):
        self.n_shift += 1
        self.zmin = self.zmin0 + self.n_shift * self.dz
        if self.galilean:
            pass          # the Galilean update already put E, B on the moved grid
        elif not self._real_pending:
            # a one-cell periodic shift toward the tail multiplies the z
            # spectrum by exp(i k_z dz); removing the departed column first
            # (a delta in z: the same radial transform at every k_z) leaves
            # the head empty
            ramp = np.exp(1j * self.kz * self.dz)[None, :]
            for m in range(self.M):
                hk = self.hankel[m]
                nus = sp.hankel_orders(m)
                for Fh, F in ((self.Eh, self.E), (self.Bh, self.B)):
                    for c in range(3):
                        tail = hk.F[nus[c]] @ F[m, c, :, 0]
                        Fh[m, c] = ramp * (Fh[m, c] - tail[:, None])
        if not self.galilean:
            for F in (self.E, self.B):
                F[..., :-1] = F[..., 1:].copy()
                F[..., -1] = 0.0
        for s in self.species:
            keep = s.z >= self.zmin
            for a in ("x", "y", "z", "ux", "uy", "uz", "w"):
                setattr(s, a, getattr(s, a)[keep])
            if s.inject:
                x, y, z, w = pt.lattice_column(self.nz - 1, self.zmin, self.nr, self.dz,
                                               self.dr, s.ppc, s.density)
                s.x = np.concatenate([s.x, x])
                s.y = np.concatenate([s.y, y])
                s.z = np.concatenate([s.z, z])
                s.w = np.concatenate([s.w, w.astype(np.float64)])
                zero = np.zeros(x.shape[0])
                s.ux = np.concatenate([s.ux, zero])
                s.uy = np.concatenate([s.uy, zero])
                s.uz = np.concatenate([s.uz, zero])

    def step(self, n: int = 1):
        for _ in range(n):
            self.gather_push()
            self.deposit()
            self.spectral_push()

    # -- diagnostics helpers ----------------------------------------------
    def species_by_name(self, name):
        for s in self.species:
            if s.name == name:
                return s
        raise KeyError(name)
