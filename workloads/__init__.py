"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module only *generates inputs*: grid parameters, initial macro-particle
positions/momenta/weights and random spectral test fields.  It holds none of
the method's arithmetic (no deposit, transform, field update or push), so it
may be imported by both the product path and the oracle without coupling them.

Units are normalized plasma units: lengths in 1/k_p, time in 1/omega_p,
momenta u = gamma*beta, densities in n0, charges in e, masses in m_e.  The
workloads follow the beam-plasma setup of the paper's simulation section
(cold drive and witness electron bunches in a uniform plasma sampled with
2 x 2 x 4 macro-particles per cell in (z, r, theta), two azimuthal modes,
dt = dz / c); the sizes are the ones of the workload presets below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# CODATA 2018 exact / recommended values (SI)
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
EPS0 = 8.8541878128e-12
C_LIGHT = 299792458.0

# kperp grid choices (mirrors the enum of the C interface)
KPERP_J0_ZEROS = 0   # every mode: zeros of J_0 / R
KPERP_SINE = 1       # every mode: (i + 1) * pi / R
KPERP_JM_ZEROS = 2   # mode m: zeros of J_m / R (default of every preset)


def plasma_scales(n0_m3: float) -> Tuple[float, float]:
    """Return (omega_p [1/s], k_p [1/m]) for an electron density n0 [1/m^3]."""
    wp = math.sqrt(n0_m3 * E_CHARGE ** 2 / (EPS0 * M_E))
    return wp, wp / C_LIGHT


def charge_to_weight(charge_C: float, n_macro: int, n0_m3: float) -> float:
    """Macro-particle weight (in units of n0 / k_p^3) of a bunch of total
    charge |charge_C| split into n_macro equal macro-particles."""
    _, kp = plasma_scales(n0_m3)
    n_phys = abs(charge_C) / E_CHARGE
    return n_phys / n_macro * kp ** 3 / n0_m3


@dataclasses.dataclass
class Species:
    name: str
    q: float                 # charge in units of e
    m: float                 # mass in units of m_e
    mobile: bool
    x: np.ndarray            # float64
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray           # float32, gamma * beta
    uy: np.ndarray
    uz: np.ndarray
    w: np.ndarray            # float32, macro-particle weight (n0 / k_p^3 units)
    inject: bool = False     # re-created as a lattice column at the head when the window moves
    ppc: Tuple[int, int, int] = (2, 2, 4)
    density: float = 1.0     # lattice density in units of n0 (for injection)
    diag: bool = False       # beam species reported by the diagnostics
    self_field: bool = False  # start with the beam's own (rigidly moving) space-charge field

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "Species":
        return dataclasses.replace(self, **{k: getattr(self, k).copy() for k in
                                            ("x", "y", "z", "ux", "uy", "uz", "w")})


@dataclasses.dataclass
class Workload:
    name: str
    nz: int
    nr: int
    n_modes: int
    order: int               # stencil order p = 2n; 0 means infinite order
    dz: float
    dr: float
    dt: float
    zmin: float
    moving_window: bool
    kperp_grid: int
    steps: int
    species: List[Species]
    n0_m3: float = 1e23
    filter: int = 0          # binomial J / rho smoothing passes before the field update (0 or 1)
    damp_cells: int = 0      # absorbing layer width at each z end (0: none)
    galilean: bool = False   # Galilean field update in coordinates moving with the window
    shape_order: int = 1     # particle shape: 1 linear, 3 cubic B-spline

    @property
    def n_mobile(self) -> int:
        return sum(s.n for s in self.species if s.mobile)

    def copy(self) -> "Workload":
        return dataclasses.replace(self, species=[s.copy() for s in self.species])


def lattice(nz: int, nr: int, dz: float, dr: float, zmin: float,
            ppc: Tuple[int, int, int] = (2, 2, 4), density: float = 1.0,
            j_range: Optional[Tuple[int, int]] = None) -> Dict[str, np.ndarray]:
    """Cold uniform lattice with ppc = (pz, pr, pt) macro-particles per cell.

    Cell (j, i) holds particles at z = zmin + (j + (a + 1/2)/pz) dz,
    r = (i + (b + 1/2)/pr) dr, theta = 2 pi l / pt; the weight is the
    sub-cell volume r (dr/pr)(dz/pz)(2 pi/pt) times the density.
    """
    pz, pr, pt = ppc
    j0, j1 = (0, nz) if j_range is None else j_range
    j = np.arange(j0, j1, dtype=np.float64)
    i = np.arange(nr, dtype=np.float64)
    a = (np.arange(pz) + 0.5) / pz
    b = (np.arange(pr) + 0.5) / pr
    th = 2.0 * np.pi * np.arange(pt) / pt
    # ordering: z-cell outermost, then r-cell, then sub-positions (cell-sorted)
    J, A, I, B, T = np.meshgrid(j, a, i, b, th, indexing="ij")
    z = zmin + (J + A) * dz
    r = (I + B) * dr
    x = r * np.cos(T)
    y = r * np.sin(T)
    w = density * r * (dr / pr) * (dz / pz) * (2.0 * np.pi / pt)
    # reorder so that all particles of one (j, i) cell are contiguous
    perm = np.transpose(np.arange(J.size).reshape(J.shape), (0, 2, 1, 3, 4)).ravel()
    out = {
        "x": x.ravel()[perm].astype(np.float64),
        "y": y.ravel()[perm].astype(np.float64),
        "z": z.ravel()[perm].astype(np.float64),
        "w": w.ravel()[perm].astype(np.float32),
    }
    n = out["x"].shape[0]
    for k in ("ux", "uy", "uz"):
        out[k] = np.zeros(n, dtype=np.float32)
    return out


def gaussian_bunch(n: int, charge_C: float, gamma: float, sigma_r: float, sigma_z: float,
                   z_center: float, seed: int, n0_m3: float = 1e23) -> Dict[str, np.ndarray]:
    """Cold Gaussian electron bunch (sigma_x = sigma_y = sigma_r) moving along +z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(0.0, sigma_r, n)
    y = rng.normal(0.0, sigma_r, n)
    z = rng.normal(z_center, sigma_z, n)
    uz = math.sqrt(gamma * gamma - 1.0)
    w = charge_to_weight(charge_C, n, n0_m3)
    return {
        "x": x.astype(np.float64), "y": y.astype(np.float64), "z": z.astype(np.float64),
        "ux": np.zeros(n, np.float32), "uy": np.zeros(n, np.float32),
        "uz": np.full(n, uz, np.float32), "w": np.full(n, w, np.float32),
    }


def quiet_beam(name: str, gamma: float, total_weight: float, nz: int, nr: int, dz: float, dr: float,
               zc: float, sigma_z: float, sigma_r: float, ppc=(2, 2, 4), q: float = -1.0) -> "Species":
    """A cold beam without shot noise: particles on the regular 2x2x4 lattice of
    the grid's cells, weights following a Gaussian profile (times r, the ring
    volume), all moving along z with the same gamma; lattice points whose
    weight is below 1e-6 of the largest are left out."""
    pz, pr, pt = ppc
    j, a, i, b, l = np.meshgrid(np.arange(nz), np.arange(pz), np.arange(nr), np.arange(pr), np.arange(pt),
                                indexing="ij")
    z = ((j + (a + 0.5) / pz) * dz).ravel()
    r = ((i + (b + 0.5) / pr) * dr).ravel()
    th = (2.0 * np.pi * (l + 0.5) / pt).ravel()
    w = np.exp(-0.5 * ((z - zc) / sigma_z) ** 2 - 0.5 * (r / sigma_r) ** 2) * r
    keep = w > 1e-6 * w.max()
    z, r, th, w = z[keep], r[keep], th[keep], w[keep]
    w = (w / w.sum() * total_weight).astype(np.float32)
    n = z.size
    uz = np.full(n, np.sqrt(gamma ** 2 - 1.0), np.float32)
    zero = np.zeros(n, np.float32)
    return Species(name, q, 1.0, True, r * np.cos(th), r * np.sin(th), z, zero, zero.copy(), uz, w, diag=True,
                   self_field=True)


def _plasma_species(nz, nr, dz, dr, zmin, ppc=(2, 2, 4)):
    lat = lattice(nz, nr, dz, dr, zmin, ppc)
    ele = Species("plasma_e", -1.0, 1.0, True, inject=True, ppc=ppc, **lat)
    ion_lat = {k: v.copy() for k, v in lat.items()}
    ion = Species("plasma_ion", +1.0, 1836.15267343, False, inject=True, ppc=ppc, **ion_lat)
    return ele, ion


def _bunch_species(name, n, charge_C, gamma, sigma_r, sigma_z, zc, seed, diag, self_field=False):
    b = gaussian_bunch(n, charge_C, gamma, sigma_r, sigma_z, zc, seed)
    return Species(name, -1.0, 1.0, True, diag=diag, self_field=self_field, **b)


def preset(name: str, seed: int = 0) -> Workload:
    """Workload presets.

    * ``c0``    256 x 64 cells, 2 modes, p = 16, dz = dr = 0.05, 1e4-particle
                100 pC drive bunch (gamma 1000, sigma 0.5), 50 steps.
    * ``c1``    2048 x 256 cells, 2 modes, p = 32, dz = 0.02, dr = 0.05, 1 nC drive
                (1e6 particles) + 50 pC witness (2e5 particles), gamma 2000.
    * ``tiny``  64 x 32 cells, 2 modes, p = 8, a 64-particle bunch: test-sized.
    * ``small`` 128 x 32 cells, 2 modes, p = 16, plasma + bunch: several tiles,
                ragged particle counts; the oracle finishes in seconds.
    """
    if name == "c0":
        nz, nr, dz, dr = 256, 64, 0.05, 0.05
        zmin = 0.0
        ele, ion = _plasma_species(nz, nr, dz, dr, zmin)
        drive = _bunch_species("drive", 10_000, 100e-12, 1000.0, 0.5, 0.5,
                               zmin + 0.7 * nz * dz, seed, True)
        return Workload("c0", nz, nr, 2, 16, dz, dr, dz, zmin, True, KPERP_JM_ZEROS, 50,
                        [ele, ion, drive])
    if name == "c1":
        nz, nr, dz, dr = 2048, 256, 0.02, 0.05
        zmin = 0.0
        ele, ion = _plasma_species(nz, nr, dz, dr, zmin)
        zd = zmin + 0.7 * nz * dz
        drive = _bunch_species("drive", 1_000_000, 1e-9, 2000.0, 0.5, 0.5, zd, seed, False)
        wit = _bunch_species("witness", 200_000, 50e-12, 2000.0, 0.1, 0.1, zd - 4.0,
                             seed + 1, True)
        return Workload("c1", nz, nr, 2, 32, dz, dr, dz, zmin, True, KPERP_JM_ZEROS, 2000,
                        [ele, ion, drive, wit])
    if name == "tiny":
        nz, nr, dz, dr = 64, 32, 0.1, 0.1
        zmin = 0.0
        b = _bunch_species("bunch", 64, 20e-12, 50.0, 0.3, 0.4, 3.2, seed, True)
        return Workload("tiny", nz, nr, 2, 8, dz, dr, dz, zmin, False, KPERP_JM_ZEROS, 4, [b])
    if name == "small":
        nz, nr, dz, dr = 128, 32, 0.05, 0.05
        zmin = 0.0
        ele, ion = _plasma_species(nz, nr, dz, dr, zmin)
        drive = _bunch_species("drive", 3001, 50e-12, 500.0, 0.3, 0.4,
                               zmin + 0.6 * nz * dz, seed, True)
        return Workload("small", nz, nr, 2, 16, dz, dr, dz, zmin, True, KPERP_JM_ZEROS, 10,
                        [ele, ion, drive])
    raise KeyError(name)


# ---------------------------------------------------------------------------
# the paper's accuracy set-up (Sec. "Accurate modeling of plasma accelerators
# in finite order PSATD")
# ---------------------------------------------------------------------------
M_E_MEV = 0.51099895000
UM = 1e-6 * 5.9507e4        # one micrometre in 1/k_p at n0 = 1e17 cm^-3 (k_p = 5.9507e4 1/m)
PAPER_DZ = 0.2 * UM         # 5 cells per micrometre along z
PAPER_DR = UM / 1.5         # 1.5 cells per micrometre along r
PAPER_STEPS = 175_000       # 35 mm of propagation at dt = dz / c


def paper_accuracy(order: int, witness_offset: float, seed: int = 0, n_drive: int = 1_000_000,
                   n_witness: int = 200_000, nz: int = 1024, nr: int = 320,
                   self_field: bool = True, witness_mev: float = 25.0, filter: int = 0) -> Workload:
    """Cold 1 GeV, 180 pC drive (8.4 um rms length, 5 um rms width) and cold
    25 MeV, 50 pC witness (2 um, 1 um) in a 1e17 cm^-3 plasma, 2x2x4 particles
    per cell, two modes, dt = dz/c, moving window.  The box is the paper's
    900 x 300 cells rounded up to 1024 x 320 (the FFT length and the radial tile
    size); the drive sits at 3/4 of the box, the witness `witness_offset`
    (1/k_p) behind it.  Both beams start with their own space-charge field
    (`self_field`).  `witness_mev` is the witness kinetic energy (25 MeV in
    the paper)."""
    zmin = 0.0
    ele, ion = _plasma_species(nz, nr, PAPER_DZ, PAPER_DR, zmin)
    zd = zmin + 0.75 * nz * PAPER_DZ
    g_drive = 1.0 + 1000.0 / M_E_MEV
    g_wit = 1.0 + witness_mev / M_E_MEV
    drive = _bunch_species("drive", n_drive, 180e-12, g_drive, 5.0 * UM, 8.4 * UM, zd, seed, True,
                           self_field)
    species = [ele, ion, drive]
    if n_witness:
        species.append(_bunch_species("witness", n_witness, 50e-12, g_wit, 1.0 * UM, 2.0 * UM,
                                      zd - witness_offset, seed + 1, True, self_field))
    return Workload(f"paper_p{order}", nz, nr, 2, order, PAPER_DZ, PAPER_DR, PAPER_DZ, zmin, True,
                    KPERP_JM_ZEROS, PAPER_STEPS, species, filter=filter)


# ---------------------------------------------------------------------------
# parameter scans
# ---------------------------------------------------------------------------
SCAN_ORDERS = (8, 16, 24, 32, 48, 64, 0)          # 0 = infinite order
SCAN_NZ = (512, 1024, 2048)
SCAN_NR = (128, 256)


@dataclasses.dataclass
class ScanInstance:
    """One run of a parameter scan: grid, stencil order and witness beam."""
    index: int
    tuple_index: int
    order: int
    nz: int
    nr: int
    dz: float
    dr: float
    gamma_w: float
    charge_w_C: float
    seed: int

    def features(self) -> Tuple[float, float, float, float, float]:
        """(2/p, k_p dz, k_p dr, log gamma, witness charge in pC); 2/p = 0 for p = inf."""
        return (0.0 if self.order == 0 else 2.0 / self.order, self.dz, self.dr,
                math.log(self.gamma_w), self.charge_w_C * 1e12)


def scan_instances(n_tuples: int = 9, orders=SCAN_ORDERS, seed: int = 0, extra: int = 1,
                   nz_choices=SCAN_NZ, nr_choices=SCAN_NR) -> List[ScanInstance]:
    """Seeded scan: n_tuples physical set-ups (N_z, N_r, k_p dz in [0.01, 0.05],
    k_p dr in [0.03, 0.08], witness gamma in [500, 4000], witness charge in
    [10, 100] pC; boxes shorter than 8/k_p are redrawn, since driver, 4/k_p gap
    and witness must fit), each run at every order, plus `extra` repeats of
    the first tuples at infinite order (64 runs for the defaults)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tuples = []
    while len(tuples) < n_tuples:
        nz = int(rng.choice(nz_choices))
        nr = int(rng.choice(nr_choices))
        dz = float(rng.uniform(0.01, 0.05))
        dr = float(rng.uniform(0.03, 0.08))
        g = float(math.exp(rng.uniform(math.log(500.0), math.log(4000.0))))
        q = float(rng.uniform(10e-12, 100e-12))
        if nz * dz < 8.0:
            continue
        tuples.append((nz, nr, dz, dr, g, q))
    out = []
    for t, (nz, nr, dz, dr, g, q) in enumerate(tuples):
        for p in orders:
            out.append(ScanInstance(len(out), t, p, nz, nr, dz, dr, g, q, seed * 1000 + t))
    for e in range(extra):
        nz, nr, dz, dr, g, q = tuples[e % len(tuples)]
        out.append(ScanInstance(len(out), e % len(tuples), 0, nz, nr, dz, dr, g, q,
                                seed * 1000 + e % len(tuples)))
    return out


def scan_workload(inst: ScanInstance, steps: int = 500) -> Workload:
    """The beam-plasma set-up of one scan run: 2x2x4 plasma over the box with
    immobile ions, the 1 nC drive (1e6 particles, gamma 2000, sigma 0.5) at 0.7 of
    the box and the witness (2e5 particles, sigma 0.1) 4/k_p behind it, moving
    window, dt = dz, two modes."""
    zmin = 0.0
    ele, ion = _plasma_species(inst.nz, inst.nr, inst.dz, inst.dr, zmin)
    zd = zmin + 0.7 * inst.nz * inst.dz
    drive = _bunch_species("drive", 1_000_000, 1e-9, 2000.0, 0.5, 0.5, zd, inst.seed, False)
    wit = _bunch_species("witness", 200_000, inst.charge_w_C, inst.gamma_w, 0.1, 0.1, zd - 4.0,
                         inst.seed + 1, True)
    return Workload(f"scan{inst.index}", inst.nz, inst.nr, 2, inst.order, inst.dz, inst.dr, inst.dz,
                    zmin, True, KPERP_JM_ZEROS, steps, [ele, ion, drive, wit])


def random_spectral(shape, seed: int) -> np.ndarray:
    """Seeded complex128 array with standard-normal real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_particles(n: int, nz: int, nr: int, dz: float, dr: float, zmin: float,
                     seed: int, u_scale: float = 1.0) -> Dict[str, np.ndarray]:
    """Seeded particles spread uniformly over the box (r up to nr * dr, any z)
    with random momenta and weights: used by deposit/gather/push parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.sqrt(rng.uniform(0.0, 1.0, n)) * nr * dr
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    z = zmin + rng.uniform(0.0, nz * dz, n)
    return {
        "x": r * np.cos(th), "y": r * np.sin(th), "z": z,
        "ux": (u_scale * rng.standard_normal(n)).astype(np.float32),
        "uy": (u_scale * rng.standard_normal(n)).astype(np.float32),
        "uz": (u_scale * rng.standard_normal(n)).astype(np.float32),
        "w": rng.uniform(0.5, 1.5, n).astype(np.float32),
    }


# ---------------------------------------------------------------------------
# surrogate network: initial parameters and minibatch order
# ---------------------------------------------------------------------------
def mlp_layer_sizes(n_in: int = 5, hidden: int = 128, n_hidden_layers: int = 4,
                    n_out: int = 2) -> List[Tuple[int, int]]:
    """(in, out) of every layer of the surrogate network."""
    dims = [n_in] + [hidden] * n_hidden_layers + [n_out]
    return list(zip(dims[:-1], dims[1:]))


def mlp_init(sizes, seed: int = 0) -> np.ndarray:
    """Flat float32 parameters, layer by layer (W_l [out][in], then b_l), each
    drawn uniformly from +-1/sqrt(in) of its layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for (i, n) in sizes:
        bound = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-bound, bound, n * i))
        parts.append(rng.uniform(-bound, bound, n))
    return np.concatenate(parts).astype(np.float32)


def minibatch_indices(n_data: int, batch: int, steps: int, seed: int = 0) -> np.ndarray:
    """Row indices of `steps` minibatches of `batch` rows (int32), drawn as
    consecutive slices of fresh random permutations of the data set (rows
    repeat within a batch only when batch > n_data)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    need = steps * batch
    out = []
    have = 0
    while have < need:
        p = rng.permutation(n_data)
        out.append(p)
        have += p.size
    return np.concatenate(out)[:need].astype(np.int32)
