"""Pins of the oracle's particle side: deposit, gather, Boris push."""
import json
import math
import os

import numpy as np
import pytest

from oracle import particles as pt
from workloads import charge_to_weight, plasma_scales, random_particles

GRID = {"nz": 24, "nr": 12, "dz": 0.1, "dr": 0.15, "zmin": 0.3}


def _vol():
    return pt.ring_volume(GRID["nr"], GRID["dr"], GRID["dz"])


def test_charge_partition_of_unity():
    p = random_particles(500, GRID["nz"], GRID["nr"] - 1, GRID["dz"], GRID["dr"],
                         GRID["zmin"], seed=1)
    qw = -p["w"].astype(np.float64)
    rho = pt.deposit_rho(2, qw, p["x"], p["y"], p["z"], GRID)
    total = (rho[0] * _vol()[:, None]).sum()
    assert total.real == pytest.approx(qw.sum(), rel=1e-13)
    assert abs(total.imag) < 1e-12


def test_single_particle_mode_phase():
    # away from the axis every node of mode 1 carries exp(i theta_p) times mode 0
    th = 0.77
    r = 0.9
    x, y, z = np.array([r * np.cos(th)]), np.array([r * np.sin(th)]), np.array([1.234])
    rho = pt.deposit_rho(3, np.array([2.0]), x, y, z, GRID)
    nz_ = rho[0] != 0
    assert nz_.sum() == 4
    np.testing.assert_allclose(rho[1][nz_] / rho[0][nz_], np.exp(1j * th), rtol=1e-13)
    np.testing.assert_allclose(rho[2][nz_] / rho[0][nz_], np.exp(2j * th), rtol=1e-13)


def test_ring_current_phases():
    # a ring of particles (uniform in theta) sharing one Cartesian velocity v:
    # mode 0 of J_z is rho_0 v_z; J_x + i J_y = 2 J_{-,1} = rho_0 (v_x + i v_y);
    # mode-0 J_+/J_- and mode-1 J_+ cancel around the ring
    L = 8
    th = 2 * np.pi * np.arange(L) / L + 0.1
    r, z = 0.8, 1.0
    x, y, zz = r * np.cos(th), r * np.sin(th), np.full(L, z)
    qw = np.full(L, 0.5)
    v = (0.3, -0.2, 0.9)
    rho = pt.deposit_rho(2, qw, x, y, zz, GRID)
    J = pt.deposit_current(2, qw, x, y, zz, np.full(L, v[0]), np.full(L, v[1]),
                           np.full(L, v[2]), GRID)
    np.testing.assert_allclose(J[0, 2], rho[0] * v[2], atol=1e-13)
    np.testing.assert_allclose(2 * J[1, 1], rho[0] * (v[0] + 1j * v[1]), atol=1e-13)
    for a in (J[0, 0], J[0, 1], J[1, 0], rho[1]):
        assert np.abs(a).max() < 1e-13


def _gather(Fm, x, y, z):
    return pt.gather_cartesian(Fm, x, y, z, GRID)


def test_gather_uniform_cartesian_field_everywhere():
    # a uniform Cartesian field E0 is E_{z,0} = E0_z and E_{-,1} = (E0_x + i E0_y)/2
    # (Hankel order 0, smooth through the axis): linear interpolation must
    # return E0 exactly at every particle, including next to the axis
    E0 = (0.3, -1.2, 0.7)
    Fm = np.zeros((2, 3, GRID["nr"], GRID["nz"]), complex)
    Fm[0, 2] = E0[2]
    Fm[1, 1] = (E0[0] + 1j * E0[1]) / 2
    p = random_particles(300, GRID["nz"], GRID["nr"] - 1, GRID["dz"], GRID["dr"],
                         GRID["zmin"], seed=2)
    ex, ey, ez = _gather(Fm, p["x"], p["y"], p["z"])
    np.testing.assert_allclose(ex, E0[0], atol=1e-13)
    np.testing.assert_allclose(ey, E0[1], atol=1e-13)
    np.testing.assert_allclose(ez, E0[2], atol=1e-13)


def test_gather_radial_linear_field_through_axis():
    # E_r = a r (mode 0: E_+ = E_- = a r / 2, Hankel orders +-1, odd through
    # the axis): the ghost-node parity makes linear interpolation exact down
    # to r = 0, giving E_x + i E_y = a (x + i y)
    a = 1.7
    r = (np.arange(GRID["nr"]) + 0.5) * GRID["dr"]
    Fm = np.zeros((1, 3, GRID["nr"], GRID["nz"]), complex)
    Fm[0, 0] = Fm[0, 1] = (a * r / 2)[:, None]
    p = random_particles(300, GRID["nz"], GRID["nr"] - 1, GRID["dz"], GRID["dr"],
                         GRID["zmin"], seed=3)
    ex, ey, ez = _gather(Fm, p["x"], p["y"], p["z"])
    np.testing.assert_allclose(ex, a * p["x"], atol=1e-13)
    np.testing.assert_allclose(ey, a * p["y"], atol=1e-13)


def test_gather_linear_in_z_and_r():
    # F_z = c0 + c1 z_rel + c2 r in mode 0: exact away from the axis and the
    # periodic seam
    c0, c1, c2 = 0.2, -0.7, 1.3
    r = (np.arange(GRID["nr"]) + 0.5) * GRID["dr"]
    zrel = np.arange(GRID["nz"]) * GRID["dz"]
    Fm = np.zeros((1, 3, GRID["nr"], GRID["nz"]), complex)
    Fm[0, 2] = c0 + c1 * zrel[None, :] + c2 * r[:, None]
    rng = np.random.default_rng(4)
    n = 200
    rr = rng.uniform(GRID["dr"], (GRID["nr"] - 1) * GRID["dr"], n)
    th = rng.uniform(0, 2 * np.pi, n)
    zz = GRID["zmin"] + rng.uniform(0, (GRID["nz"] - 1) * GRID["dz"], n)
    ex, ey, ez = _gather(Fm, rr * np.cos(th), rr * np.sin(th), zz)
    np.testing.assert_allclose(ez, c0 + c1 * (zz - GRID["zmin"]) + c2 * rr, atol=1e-12)


def test_boris_pure_electric_kick():
    E = (0.3, -0.1, 0.5)
    u = pt.boris(np.array([0.1]), np.array([0.2]), np.array([3.0]), *E, 0.0, 0.0, 0.0,
                 -1.0, 1.0, 0.2)
    eps = -1.0 * 0.2 / 2
    np.testing.assert_allclose(np.array(u).ravel(), [0.1 + 2 * eps * E[0], 0.2 + 2 * eps * E[1],
                                                     3.0 + 2 * eps * E[2]], rtol=1e-15)


def test_boris_magnetic_rotation_angle():
    # pure B along z: |u| conserved, u_perp rotates by exactly 2 atan(|t|) per step
    ux, uy, uz = np.array([1.5]), np.array([0.0]), np.array([0.7])
    Bz, q, m, dt = 2.0, -1.0, 1.0, 0.3
    g = math.sqrt(1 + 1.5 ** 2 + 0.7 ** 2)
    t = abs(q * dt / (2 * m) * Bz / g)
    ang = 0.0
    for _ in range(7):
        nx, ny, nz = pt.boris(ux, uy, uz, 0, 0, 0, 0, 0, Bz, q, m, dt)
        ang += math.atan2(ux[0] * ny[0] - uy[0] * nx[0], ux[0] * nx[0] + uy[0] * ny[0])
        ux, uy, uz = nx, ny, nz
    assert math.hypot(ux[0], uy[0]) == pytest.approx(1.5, rel=1e-14)
    assert uz[0] == pytest.approx(0.7, rel=1e-15)
    assert abs(ang) == pytest.approx(7 * 2 * math.atan(t), rel=1e-13)
    # an electron (q < 0) gyrates counter-clockwise about +B
    assert ang > 0


def test_boris_exb_drift():
    # E = Ex x^, B = Bz z^, |E| < |B|: the guiding centre drifts with E x B / B^2
    Ex, Bz = 0.2, 1.0
    ux, uy, uz = np.array([0.0]), np.array([0.0]), np.array([0.0])
    x = y = 0.0
    dt, nsteps = 0.05, 40000
    for _ in range(nsteps):
        ux, uy, uz = pt.boris(ux, uy, uz, Ex, 0.0, 0.0, 0.0, 0.0, Bz, -1.0, 1.0, dt)
        g = math.sqrt(1 + ux[0] ** 2 + uy[0] ** 2 + uz[0] ** 2)
        x += dt * ux[0] / g
        y += dt * uy[0] / g
    vd = y / (nsteps * dt)
    # E x B / B^2 = (0, -Ex Bz, 0) / Bz^2
    assert vd == pytest.approx(-Ex / Bz, rel=2e-2)
    assert abs(x / (nsteps * dt)) < 1e-2


def test_witness_peak_current_and_density(golden_dir):
    # the Gaussian-bunch convention (sigma_x = sigma_y = rms width) reproduces
    # the paper's printed 3 kA / 1e19 cm^-3 for its 50 pC witness
    g = json.load(open(os.path.join(golden_dir, "witness_beam.json")))
    n0 = g["n0_cm3"] * 1e6
    _, kp = plasma_scales(n0)
    w = charge_to_weight(g["charge_pC"] * 1e-12, 1000, n0)       # n0/kp^3 units
    sz, sr = g["sigma_z_um"] * 1e-6 * kp, g["sigma_r_um"] * 1e-6 * kp
    peak_n = 1000 * w / ((2 * np.pi) ** 1.5 * sz * sr * sr) * n0 / 1e6   # cm^-3
    current = g["charge_pC"] * 1e-12 * 299792458.0 / (math.sqrt(2 * math.pi) * g["sigma_z_um"] * 1e-6)
    tol = g["printed_precision"]
    assert current / 1e3 == pytest.approx(g["peak_current_kA"], rel=tol)
    assert peak_n == pytest.approx(g["peak_density_cm3"], rel=tol)


def _axis_particles(n, seed):
    """Particles spread over the box with a quarter of them below the first
    radial node (r < dr/2), where the inner shape node is the ghost across
    the axis."""
    rng = np.random.default_rng(seed)
    r = np.concatenate([rng.uniform(0.0, 0.5 * GRID["dr"], n // 4),
                        rng.uniform(0.0, (GRID["nr"] - 1) * GRID["dr"], n - n // 4)])
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    z = GRID["zmin"] + rng.uniform(0.0, GRID["nz"] * GRID["dz"], n)
    return r * np.cos(th), r * np.sin(th), z, r


@pytest.mark.parametrize("nu", [-1, 0, 1, 2, 3])
def test_deposit_is_the_adjoint_of_the_gather(nu):
    # the deposit spreads a particle quantity with the same node weights and
    # axis rule the gather interpolates with, so for any grid field F and
    # particle values a:  sum_nodes V_i rho_nu[i, j] F[i, j] = sum_p a_p F_nu(x_p).
    # The gather's axis rule is pinned on its own (radially linear field,
    # uniform field); this ties the deposit's ghost-node sign (-1)^nu to it
    x, y, z, r = _axis_particles(400, seed=11 + nu)
    rng = np.random.default_rng(7)
    a = rng.standard_normal(x.size) + 1j * rng.standard_normal(x.size)
    F = rng.standard_normal((GRID["nr"], GRID["nz"])) + 1j * rng.standard_normal((GRID["nr"], GRID["nz"]))
    rho = pt.deposit_scalar(a, nu, z, r, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"], GRID["nr"])
    lhs = (_vol()[:, None] * rho * F).sum()
    nodes = pt.shape_nodes(z, r, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"])
    rhs = (a * pt.gather_scalar(F, nu, nodes, GRID["nr"])).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_odd_and_even_modes_are_regular_at_the_axis(m):
    # a mode-m density behaves like r^|m| near the axis; with linear shapes
    # the deposit of a single particle must therefore vanish linearly as the
    # particle approaches the axis for odd m (ghost weight enters with -1 and
    # cancels the node-0 weight) and stay finite, equal to the r = 0 value of
    # e^{i m theta} q w / V_0 per z-node weight, for even m
    th, zp = 0.6, 1.0
    vals = []
    radii = (1e-2, 1e-3, 1e-4)
    for rp in radii:
        x, y = np.array([rp * np.cos(th)]), np.array([rp * np.sin(th)])
        rho = pt.deposit_rho(m + 1, np.array([1.0]), x, y, np.array([zp]), GRID)
        vals.append(np.abs(rho[m][0]).sum() * _vol()[0])
    vals = np.array(vals)
    if m % 2:
        # node 0 keeps (1/2 + r/dr) - (1/2 - r/dr) = 2 r/dr of the particle
        np.testing.assert_allclose(vals, 2.0 * np.array(radii) / GRID["dr"], rtol=1e-9)
    else:
        np.testing.assert_allclose(vals, 1.0, rtol=1e-3)


def test_injected_lattice_has_the_plasma_density():
    # lattice columns as injected at the head, deposited over a full box:
    # rho_0 = q n on every node away from the axis and the outer edge (the
    # weights r dr/pr dz/pz 2pi/pt sum, with linear shapes, to the ring
    # volume of each node), and the theta-symmetric lattice has no mode 1
    nz, nr, dz, dr, zmin = GRID["nz"], GRID["nr"], GRID["dz"], GRID["dr"], GRID["zmin"]
    density = 2.5
    cols = [pt.lattice_column(j, zmin, nr, dz, dr, (2, 2, 4), density) for j in range(nz)]
    x, y, z, w = (np.concatenate([c[k] for c in cols]) for k in range(4))
    rho = pt.deposit_rho(2, -w.astype(np.float64), x, y, z, GRID)
    np.testing.assert_allclose(rho[0][1:nr - 1].real, -density, rtol=1e-6)
    assert np.abs(rho[1]).max() < 1e-6 * density
    # a single injected column fills the nodes of its cell by halves
    x, y, z, w = pt.lattice_column(nz - 1, zmin, nr, dz, dr, (2, 2, 4), density)
    rho = pt.deposit_rho(1, w.astype(np.float64), x, y, z, GRID)
    np.testing.assert_allclose(rho[0][1:nr - 1, nz - 1].real, 0.5 * density, rtol=1e-6)
    np.testing.assert_allclose(rho[0][1:nr - 1, 0].real, 0.5 * density, rtol=1e-6)   # periodic wrap
    assert np.abs(rho[0][:, 1:nz - 1]).max() == 0.0


# --- cubic B-spline shapes (an option of the deposit and gather) -------------
def _bspline_cox_de_boor(x, k):
    """Uniform B-spline of degree k on knots 0, 1, ..., k+1, by the textbook
    Cox-de Boor recursion (independent of the closed forms in the oracle)."""
    if k == 0:
        return np.where((x >= 0.0) & (x < 1.0), 1.0, 0.0)
    return (x * _bspline_cox_de_boor(x, k - 1) + (k + 1 - x) * _bspline_cox_de_boor(x - 1.0, k - 1)) / k


def test_cubic_weights_are_the_cubic_bspline():
    # node at offset d from the particle's cell start gets B3 centred on the
    # particle: B3(d - f + 2) with B3 the degree-3 spline on knots 0..4
    f = np.linspace(0.0, 0.999, 37)
    for d, w in pt.bspline_weights(f, 3):
        np.testing.assert_allclose(w, _bspline_cox_de_boor(d - f + 2.0, 3), atol=1e-15)
    # and the linear ones are the degree-1 spline
    for d, w in pt.bspline_weights(f, 1):
        np.testing.assert_allclose(w, _bspline_cox_de_boor(d - f + 1.0, 1), atol=1e-15)


def test_cubic_weight_moments():
    # partition of unity, centred (first moment 0), variance 1/3 cell^2 (four
    # unit boxes convolved: 4 x 1/12)
    f = np.random.default_rng(3).uniform(0.0, 1.0, 1000)
    ws = pt.bspline_weights(f, 3)
    m0 = sum(w for _, w in ws)
    m1 = sum(w * (d - f) for d, w in ws)
    m2 = sum(w * (d - f) ** 2 for d, w in ws)
    np.testing.assert_allclose(m0, 1.0, atol=1e-14)
    np.testing.assert_allclose(m1, 0.0, atol=1e-14)
    np.testing.assert_allclose(m2, 1.0 / 3.0, atol=1e-14)


CUBIC = dict(GRID, shape=3)


@pytest.mark.parametrize("nu", [-1, 0, 1, 2, 3])
def test_cubic_deposit_is_the_adjoint_of_the_gather(nu):
    # the same adjointness as for linear shapes, with the cubic shape and its
    # two ghost nodes across the axis (r = -dr/2 -> node 0, -3dr/2 -> node 1)
    x, y, z, r = _axis_particles(400, seed=31 + nu)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(x.size) + 1j * rng.standard_normal(x.size)
    F = rng.standard_normal((GRID["nr"], GRID["nz"])) + 1j * rng.standard_normal((GRID["nr"], GRID["nz"]))
    rho = pt.deposit_scalar(a, nu, z, r, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"], GRID["nr"], 3)
    lhs = (_vol()[:, None] * rho * F).sum()
    nodes = pt.shape_nodes(z, r, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"], 3)
    rhs = (a * pt.gather_scalar(F, nu, nodes, GRID["nr"])).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_cubic_gather_of_polynomials_in_z():
    # a cubic B-spline reproduces linear functions exactly and smooths a
    # quadratic by its variance: the gather of z^2 is z^2 + dz^2 / 3
    rng = np.random.default_rng(5)
    n = 300
    zs = rng.uniform(0.3, 0.7, n) * GRID["nz"] * GRID["dz"] + GRID["zmin"]
    rs = rng.uniform(3.0, 6.0, n) * GRID["dr"]            # away from axis and edge
    zj = GRID["zmin"] + np.arange(GRID["nz"]) * GRID["dz"]
    nodes = pt.shape_nodes(zs, rs, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"], 3)
    lin = np.tile(2.0 * zj - 0.3, (GRID["nr"], 1)).astype(complex)
    quad = np.tile(zj ** 2, (GRID["nr"], 1)).astype(complex)
    np.testing.assert_allclose(pt.gather_scalar(lin, 0, nodes, GRID["nr"]).real, 2.0 * zs - 0.3, atol=1e-12)
    np.testing.assert_allclose(pt.gather_scalar(quad, 0, nodes, GRID["nr"]).real,
                               zs ** 2 + GRID["dz"] ** 2 / 3.0, atol=1e-12)


def test_cubic_single_particle_charge_and_mode_phase():
    # an interior particle puts its whole charge on 16 nodes, with the mode
    # phase e^{i m theta}
    th = 0.9
    rp, zp = 2.37 * GRID["dr"], GRID["zmin"] + 5.61 * GRID["dz"]
    x, y = np.array([rp * np.cos(th)]), np.array([rp * np.sin(th)])
    rho = pt.deposit_rho(3, np.array([1.0]), x, y, np.array([zp]), CUBIC)
    for m in range(3):
        q = (rho[m] * _vol()[:, None]).sum()
        np.testing.assert_allclose(q, np.exp(1j * m * th), atol=1e-13)
        assert np.count_nonzero(np.abs(rho[m]) > 0) == 16


def test_cubic_gather_through_the_axis():
    # near the axis the cubic shape reaches both ghost nodes (-dr/2 and -3dr/2);
    # standing for nodes 0 and 1 with the factor (-1)^nu they continue an even
    # field (nu = 0) evenly and an odd one (nu = 1) oddly across r = 0, so the
    # spline still reproduces polynomials: r^2 -> s^2 + dr^2/3, r -> s
    s = np.random.default_rng(8).uniform(0.0, 2.0, 200) * GRID["dr"]
    z = np.full(s.size, GRID["zmin"] + 7.3 * GRID["dz"])
    ri = (np.arange(GRID["nr"]) + 0.5) * GRID["dr"]
    nodes = pt.shape_nodes(z, s, GRID["zmin"], GRID["dz"], GRID["dr"], GRID["nz"], 3)
    even = np.tile((ri ** 2)[:, None], (1, GRID["nz"])).astype(complex)
    odd = np.tile(ri[:, None], (1, GRID["nz"])).astype(complex)
    np.testing.assert_allclose(pt.gather_scalar(even, 0, nodes, GRID["nr"]).real, s ** 2 + GRID["dr"] ** 2 / 3.0,
                               atol=1e-12)
    np.testing.assert_allclose(pt.gather_scalar(odd, 1, nodes, GRID["nr"]).real, s, atol=1e-12)
