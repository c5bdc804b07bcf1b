"""Locality and dispersion of the order-p update, measured through the GPU
spectral push (the survey's first "next" row; paper Sec. "Finite order
pseudo-spectral solvers", Eqs. (5)-(6), and Sec. "Numerical Cherenkov
radiation", Eqs. (8)-(10)).

A unit pulse in z times one radial eigenfunction, E_+ = J_1(k_perp r) delta_{j j0}
(mode 0; B = J = rho = 0), is advanced one step.  Then E_+^{n+1} = C E_+ with
C = cos(sqrt(k_perp^2 + [k_z]^2) dt), so
  * the spectral E_+ divided by the pulse's spectrum is C(k_z) itself, which
    gives the measured [k_z], the phase velocity omega/k_z and the k_z at which
    a beam of a given gamma resonates with the numerical light (Eq. (10));
  * the real-space E_+ along z is the C term of the stencil reach alpha*
    (Eq. (6)): it spreads over a number of cells that grows with p.
"""
import numpy as np
import pytest

from oracle import spectral as sp
from oracle import stencil as st
from workloads import Workload, KPERP_JM_ZEROS

pytestmark = pytest.mark.gpu

NZ, NR, DZ, DR = 256, 32, 0.05, 0.05
J0_CELL = 100


def _pulse_step(order):
    from paper_1611_05712_amd import Simulation
    from scipy.special import jv
    wl = Workload("pulse", NZ, NR, 1, order, DZ, DR, DZ, 0.0, False, KPERP_JM_ZEROS, 1, [])
    sim = Simulation.from_workload(wl)
    kperp = sp.kperp_grid(0, NR, DR, sp.KPERP_JM_ZEROS)[0]
    r = sp.r_grid(NR, DR)
    f = np.zeros((NR, NZ), np.complex64)
    f[:, J0_CELL] = jv(1, kperp * r)
    zero = np.zeros((NR, NZ), np.complex64)
    sim.set_field(0, "E+", f)
    for c in ("E-", "Ez", "B+", "B-", "Bz", "J+", "J-", "Jz", "rho_old", "rho_new"):
        sim.set_field(0, c, zero)
    sim.spectral_push()
    Eh = sim.get_field(0, "E+", spectral=True)[0]       # k_perp row 0
    E = sim.get_field(0, "E+")
    sim.close()
    return kperp, r, Eh, E


def _C_oracle(order, kperp):
    kzm = sp.kz_modified(sp.kz_grid(NZ, DZ), DZ, order)
    return np.cos(np.sqrt(kperp ** 2 + kzm ** 2) * DZ)


@pytest.mark.parametrize("order", [8, 16, 32, 64, 0])
def test_measured_dispersion_matches_the_modified_wavenumber(order):
    kperp, _, Eh, _ = _pulse_step(order)
    kz = sp.kz_grid(NZ, DZ)
    C = (Eh / np.exp(-1j * kz * J0_CELL * DZ)).real
    np.testing.assert_allclose(C, _C_oracle(order, kperp), rtol=0, atol=5e-6)
    # [k_z] recovered from the measured C (away from C = +-1, where arccos is
    # ill-conditioned) against Eq. (5)
    w = np.arccos(np.clip(C, -1, 1)) / DZ
    sel = (np.abs(C) < 0.95) & (kz > 0)
    kzm_meas = np.sqrt(np.maximum(w[sel] ** 2 - kperp ** 2, 0.0))
    kzm = sp.kz_modified(kz[sel], DZ, order)
    assert np.abs(kzm_meas - kzm).max() < 2e-3 * np.pi / DZ


@pytest.mark.parametrize("order", [8, 16, 32, 64])
def test_measured_cherenkov_resonance(order):
    # phase velocity omega / k_z of the measured dispersion crosses the speed
    # of a gamma = 2000 beam at the k_z of Eq. (10)
    kperp, _, Eh, _ = _pulse_step(order)
    kz = sp.kz_grid(NZ, DZ)
    C = (Eh / np.exp(-1j * kz * J0_CELL * DZ)).real
    pos = (kz > 0)
    k = kz[pos]
    v = np.arccos(np.clip(C[pos], -1, 1)) / DZ / k
    beta = np.sqrt(1 - 1 / 2000.0 ** 2)
    idx = np.nonzero(np.sign(v[:-1] - beta) != np.sign(v[1:] - beta))[0]
    assert idx.size > 0
    i = idx[0]
    kres = k[i] + (beta - v[i]) * (k[i + 1] - k[i]) / (v[i + 1] - v[i])
    want = st.resonance_kz(2000.0, order, DZ, kperp)
    assert abs(kres - want) < 0.5 * (k[1] - k[0]), (kres, want)


@pytest.mark.parametrize("order", [8, 16, 32, 64])
def test_unit_pulse_reach_matches_the_stencil(order):
    kperp, r, _, E = _pulse_step(order)
    row = int(np.argmax(np.abs(E[:, J0_CELL])))
    prof = np.abs(E[row])
    prof = np.roll(prof, -J0_CELL) / prof[J0_CELL]
    want = np.abs(np.fft.ifft(_C_oracle(order, kperp)))
    want = want / want[0]
    np.testing.assert_allclose(prof, want, rtol=0, atol=5e-6)

    def reach(p, floor=1e-4):
        # last cell distance d (either side of the pulse) still at or above floor, plus one
        d = np.arange(NZ // 2 + 1)
        sym = np.maximum(p[d], p[(-d) % NZ])
        return int(np.nonzero(sym >= floor)[0][-1]) + 1
    got, exp = reach(prof), reach(want)
    print(f"p = {order}: unit pulse above 1e-4 of its peak out to {got} cells (oracle {exp})")
    assert abs(got - exp) <= 1
