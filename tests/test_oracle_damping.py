"""Pins of the absorbing layers at the z ends (damp_cells): the profile's
closed values, and what an absorbing layer must do to a vacuum pulse on the
periodic z grid: nothing until the pulse arrives, then remove its energy
(monotonically) instead of letting it re-enter at the other end."""
import numpy as np
import pytest
from scipy.special import jv, jn_zeros

from oracle import spectral as sp
from oracle.cycle import OracleSim, damping_profile
from workloads import Workload, KPERP_JM_ZEROS


def test_profile_closed_values():
    w = damping_profile(64, 8)
    assert w[0] == 0.0 and w[-1] == 0.0                      # end nodes zeroed
    assert w[4] == pytest.approx(0.5, abs=1e-15)             # sin^2(pi/4)
    assert w[-5] == pytest.approx(0.5, abs=1e-15)
    assert w[2] == pytest.approx(np.sin(np.pi / 8) ** 2, abs=1e-15)
    np.testing.assert_array_equal(w[8:-8], 1.0)              # untouched interior
    np.testing.assert_array_equal(w, w[::-1])                # both ends alike
    assert np.all(np.diff(w[:9]) > 0)                        # rising into the interior


def _spectral_energy(sim):
    # the energy the vacuum update conserves: sum over modes and spectral
    # cells of 2|F_+|^2 + 2|F_-|^2 + |F_z|^2 for E and B, from the real-space
    # state (every order of the J_m grid shares one norm)
    W = 0.0
    for m in range(sim.M):
        hk = sim.hankel[m]
        nus = sp.hankel_orders(m)
        for F in (sim.E, sim.B):
            for c, wgt in zip(range(3), (2.0, 2.0, 1.0)):
                W += wgt * float(np.sum(np.abs(hk.forward(F[m, c], nus[c])) ** 2))
    return W


def _pulse_run(damp, steps, nz=128, nr=16, order=8):
    dz, dr = 0.1, 0.5
    wl = Workload("vac", nz, nr, 2, order, dz, dr, dz, 0.0, False, KPERP_JM_ZEROS, 1, [], damp_cells=damp)
    sim = OracleSim(wl)
    # a divergence-free mode-0 pulse (azimuthal E only: E_+ = -i E_theta / 2,
    # E_- = +i E_theta / 2) in the lowest radial mode, short in z: it splits
    # into two pulses running toward both ends at nearly c
    r = sim.hankel[0].r
    z = np.arange(nz)
    g = np.exp(-((z - nz / 2) / 3.0) ** 2)
    Et = jv(1, jn_zeros(1, 1)[0] * r / (nr * dr))[:, None] * g[None, :]
    E0 = np.zeros_like(sim.E)
    E0[0, 0] = -0.5j * Et
    E0[0, 1] = 0.5j * Et
    sim.set_fields(E=E0)
    sim.J = np.zeros_like(sim.E)
    sim.rho_old = np.zeros((2, nr, nz), complex)
    sim.rho_new = sim.rho_old.copy()
    W = [_spectral_energy(sim)]
    for _ in range(steps):
        sim.spectral_push()
        W.append(_spectral_energy(sim))
    return np.array(W)


def test_layers_absorb_a_vacuum_pulse():
    steps = 160          # both halves travel 64 cells to the ends, then cross a 16-cell layer
    free = _pulse_run(0, steps)
    damped = _pulse_run(16, steps)
    # without layers the vacuum update conserves the energy
    np.testing.assert_allclose(free, free[0], rtol=1e-9)
    # the layers never add energy ...
    assert np.all(np.diff(damped) <= 1e-12 * damped[0])
    # ... leave the pulse alone while it is far from them ...
    np.testing.assert_allclose(damped[:30], damped[0], rtol=1e-9)
    # ... and remove nearly all of it once it has run into them (the rest is
    # the pulse's slow, oblique part still on its way)
    assert damped[110] < 0.1 * damped[0]
    assert damped[-1] < 0.05 * damped[0]
