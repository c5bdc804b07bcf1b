"""Particle side of the oracle (FP64): linear-shape deposit and gather on the
quasi-cylindrical (r, z) grid of each azimuthal mode, Boris push and lattice
injection.

The paper treats the particle coupling as standard PIC; the shape order, the
treatment of the axis and the pusher are this implementation's readings:
  * linear (cloud-in-cell) shapes in z (periodic) and r, nodes at
    z_j = zmin + j dz and r_i = (i + 1/2) dr; or, as an option, cubic
    B-spline shapes over the four nearest nodes along each axis;
  * a particle below the first radial node shares weight with ghost nodes
    at r = -dr/2 (and -3dr/2 for cubic shapes), which stand for nodes 0 (and
    1) seen across the axis; a component of Hankel order nu takes the factor
    (-1)^nu there;
  * nodes at i >= Nr are outside the box and dropped;
  * mode-m densities use the phase exp(i m theta_p) (the conjugate of the
    exp(-i m theta) field decomposition), divided by the ring volume
    2 pi r_i dr dz;
  * Boris push (J. P. Boris, 1970), with E, B in plasma units.
"""
from __future__ import annotations

import numpy as np


def _phase(x, y):
    """exp(i theta) of each particle (1 on the axis)."""
    r = np.hypot(x, y)
    safe = np.where(r > 0.0, r, 1.0)
    return np.where(r > 0.0, (x + 1j * y) / safe, 1.0 + 0j), r


def bspline_weights(f, order):
    """(offset, weight) of the nodes of a particle at fractional position f in
    [0, 1) past node 0: linear, nodes 0 and 1; cubic B-spline (the fourfold
    convolution of the unit box), nodes -1 .. 2."""
    if order == 1:
        return ((0, 1.0 - f), (1, f))
    g = 1.0 - f
    return ((-1, g ** 3 / 6.0), (0, (4.0 - 6.0 * f ** 2 + 3.0 * f ** 3) / 6.0),
            (1, (4.0 - 6.0 * g ** 2 + 3.0 * g ** 3) / 6.0), (2, f ** 3 / 6.0))


def shape_nodes(z, r, zmin, dz, dr, nz, order=1):
    """The (j, i, weight) nodes of each particle's shape (order 1: linear, 4
    nodes; 3: cubic, 16).  i may be negative (ghosts across the axis) or
    >= Nr (outside); j is wrapped."""
    sz = (z - zmin) / dz
    j0 = np.floor(sz)
    fz = sz - j0
    j0 = j0.astype(np.int64)
    sr = r / dr - 0.5
    i0 = np.floor(sr)
    fr = sr - i0
    i0 = i0.astype(np.int64)
    nodes = []
    for dj, wz in bspline_weights(fz, order):
        for di, wr in bspline_weights(fr, order):
            nodes.append(((j0 + dj) % nz, i0 + di, wz * wr))
    return nodes


def ring_volume(nr, dr, dz):
    return 2.0 * np.pi * (np.arange(nr) + 0.5) * dr * dr * dz


def deposit_scalar(val, nu, z, r, zmin, dz, dr, nz, nr, order=1):
    """Deposit a complex per-particle quantity of Hankel order nu onto the
    [Nr, Nz] grid (a density: divided by the ring volume)."""
    acc = np.zeros(nr * nz, dtype=np.complex128)
    sgn = -1.0 if (nu % 2) else 1.0
    for j, i, wgt in shape_nodes(z, r, zmin, dz, dr, nz, order):
        # ghost node -1 - i' stands for node i' across the axis
        fold = np.where(i < 0, sgn, 1.0)
        ii = np.where(i < 0, -1 - i, i)
        keep = ii < nr
        idx = ii[keep] * nz + j[keep]
        v = (wgt * fold * val)[keep]
        acc.real += np.bincount(idx, weights=v.real, minlength=nr * nz)
        acc.imag += np.bincount(idx, weights=v.imag, minlength=nr * nz)
    return acc.reshape(nr, nz) / ring_volume(nr, dr, dz)[:, None]


def deposit_rho(n_modes, qw, x, y, z, grid):
    """rho_m for m = 0..M-1: sum of q w exp(i m theta_p) over the shape."""
    ph, r = _phase(x, y)
    out = np.zeros((n_modes, grid["nr"], grid["nz"]), dtype=np.complex128)
    for m in range(n_modes):
        out[m] = deposit_scalar(qw * ph ** m, m, z, r, grid["zmin"], grid["dz"],
                                grid["dr"], grid["nz"], grid["nr"], grid.get("shape", 1))
    return out


def deposit_current(n_modes, qw, x, y, z, vx, vy, vz, grid):
    """(J_+, J_-, J_z) of every mode from charges q w moving with velocity v.
    J_r -/+ i J_theta = (v_x -/+ i v_y) exp(+/- i theta), so mode m of J_+ takes
    (v_x - i v_y) exp(i (m+1) theta)/2 and of J_- takes
    (v_x + i v_y) exp(i (m-1) theta)/2; J_z takes v_z exp(i m theta)."""
    ph, r = _phase(x, y)
    out = np.zeros((n_modes, 3, grid["nr"], grid["nz"]), dtype=np.complex128)
    args = (z, r, grid["zmin"], grid["dz"], grid["dr"], grid["nz"], grid["nr"], grid.get("shape", 1))
    for m in range(n_modes):
        out[m, 0] = deposit_scalar(qw * (vx - 1j * vy) / 2.0 * ph ** (m + 1), m + 1, *args)
        out[m, 1] = deposit_scalar(qw * (vx + 1j * vy) / 2.0 * ph ** (m - 1), m - 1, *args)
        out[m, 2] = deposit_scalar(qw * vz * ph ** m, m, *args)
    return out


def gather_scalar(F, nu, nodes, nr):
    sgn = -1.0 if (nu % 2) else 1.0
    out = 0.0
    for j, i, wgt in nodes:
        fold = np.where(i < 0, sgn, 1.0)
        ii = np.where(i < 0, -1 - i, i)
        keep = ii < nr
        iic = np.where(keep, ii, 0)
        out = out + np.where(keep, wgt * fold * F[iic, j], 0.0)
    return out


def gather_cartesian(Fm, x, y, z, grid):
    """Cartesian (F_x, F_y, F_z) at the particles from the mode fields
    Fm[m] = (F_+, F_-, F_z) (each [Nr, Nz]):
      F_z = sum_{m=-M..M} F_{z,m} exp(-i m theta)
      F_x + i F_y = 2 [ sum_{m>=0} F_{-,m} exp(-i (m-1) theta)
                       + sum_{m>=1} conj(F_{+,m}) exp(i (m+1) theta) ]
    using F_{-,-m} = conj(F_{+,m})."""
    ph, r = _phase(x, y)
    nodes = shape_nodes(z, r, grid["zmin"], grid["dz"], grid["dr"], grid["nz"], grid.get("shape", 1))
    nr = grid["nr"]
    fz = np.zeros(x.shape, dtype=np.float64)
    fxy = np.zeros(x.shape, dtype=np.complex128)
    for m in range(Fm.shape[0]):
        gp = gather_scalar(Fm[m, 0], m + 1, nodes, nr)
        gm = gather_scalar(Fm[m, 1], m - 1, nodes, nr)
        gz = gather_scalar(Fm[m, 2], m, nodes, nr)
        if m == 0:
            fz += gz.real
            fxy += 2.0 * gm * ph
        else:
            fz += 2.0 * (gz * np.conj(ph) ** m).real
            fxy += 2.0 * (gm * np.conj(ph) ** (m - 1) + np.conj(gp) * ph ** (m + 1))
    return fxy.real, fxy.imag, fz


def boris(ux, uy, uz, Ex, Ey, Ez, Bx, By, Bz, q, m, dt):
    """Boris rotation: half electric kick, magnetic rotation, half kick.
    du/dt = (q/m)(E + u x B / gamma) in plasma units."""
    eps = q * dt / (2.0 * m)
    umx = ux + eps * Ex
    umy = uy + eps * Ey
    umz = uz + eps * Ez
    g = np.sqrt(1.0 + umx ** 2 + umy ** 2 + umz ** 2)
    tx, ty, tz = eps * Bx / g, eps * By / g, eps * Bz / g
    t2 = tx ** 2 + ty ** 2 + tz ** 2
    sx, sy, sz = 2 * tx / (1 + t2), 2 * ty / (1 + t2), 2 * tz / (1 + t2)
    upx = umx + (umy * tz - umz * ty)
    upy = umy + (umz * tx - umx * tz)
    upz = umz + (umx * ty - umy * tx)
    uqx = umx + (upy * sz - upz * sy)
    uqy = umy + (upz * sx - upx * sz)
    uqz = umz + (upx * sy - upy * sx)
    return uqx + eps * Ex, uqy + eps * Ey, uqz + eps * Ez


def lattice_column(j, zmin, nr, dz, dr, ppc, density):
    """Cold lattice particles of z-cell j (used for head injection)."""
    pz, pr, pt = ppc
    i = np.arange(nr, dtype=np.float64)
    a = (np.arange(pz) + 0.5) / pz
    b = (np.arange(pr) + 0.5) / pr
    th = 2.0 * np.pi * np.arange(pt) / pt
    I, A, B, T = np.meshgrid(i, a, b, th, indexing="ij")
    z = zmin + (j + A) * dz
    r = (I + B) * dr
    w = (density * r * (dr / pr) * (dz / pz) * (2.0 * np.pi / pt)).astype(np.float32)
    return r.ravel() * np.cos(T.ravel()), r.ravel() * np.sin(T.ravel()), z.ravel(), w.ravel()
