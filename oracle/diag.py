"""Beam diagnostics and accuracy metrics of the oracle (FP64).

The paper judges a solver order by the beam's normalized emittance and slice
energy spread, and by the spatial spectrum of E_z (Sec. "Accurate modeling of
plasma accelerators in finite order PSATD", Eqs. (11)-(13)).  All moments here
are weighted by the macro-particle weight and central (two passes).
"""
from __future__ import annotations

import math

import numpy as np


def beam_moments(x, y, z, ux, uy, uz, w, slice_len, n_sigma=3.0, min_per_slice=10):
    """Normalized rms emittances, mean/rms gamma, z centroid/rms and the mean
    slice energy spread.

    eps_n,x = sqrt(<dx^2><dux^2> - <dx dux>^2) (same for y).
    Slices have length slice_len, are anchored at the centroid (xi = z - <z>)
    and cover |xi| <= n_sigma * sigma_z; slice s spans
    [(s - h) L, (s - h + 1) L) with h = ceil(n_sigma sigma_z / L).  A slice with
    fewer than min_per_slice particles is skipped; the result averages the
    weighted rms gamma of the remaining slices."""
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    ux, uy, uz, w = (np.asarray(a, np.float64) for a in (ux, uy, uz, w))
    W = w.sum()
    out = {"n": int(x.shape[0])}
    if x.shape[0] == 0 or W <= 0:
        return dict(out, eps_nx=0.0, eps_ny=0.0, mean_gamma=0.0, sigma_gamma=0.0,
                    mean_slice_sigma_gamma=0.0, z_mean=0.0, sigma_z=0.0, n_slices=0,
                    nan_flag=0)

    def mean(a):
        return float((w * a).sum() / W)

    g = np.sqrt(1.0 + ux ** 2 + uy ** 2 + uz ** 2)
    for (p, u, key) in ((x, ux, "eps_nx"), (y, uy, "eps_ny")):
        dp = p - mean(p)
        du = u - mean(u)
        val = mean(dp * dp) * mean(du * du) - mean(dp * du) ** 2
        out[key] = math.sqrt(max(val, 0.0))
    mg = mean(g)
    out["mean_gamma"] = mg
    out["sigma_gamma"] = math.sqrt(mean((g - mg) ** 2))
    zm = mean(z)
    sz = math.sqrt(mean((z - zm) ** 2))
    out["z_mean"], out["sigma_z"] = zm, sz
    sg, cnt = slice_spreads(z, g, w, slice_len, n_sigma, min_per_slice)
    spreads = [v for v, c in zip(sg, cnt) if c >= min_per_slice]
    out["n_slices"] = len(spreads)
    out["mean_slice_sigma_gamma"] = float(np.mean(spreads)) if spreads else 0.0
    finite = all(np.isfinite(a).all() for a in (x, y, z, ux, uy, uz))
    out["nan_flag"] = 0 if finite else 1
    return out


def slice_spreads(z, gamma, w, slice_len, n_sigma=3.0, min_per_slice=10):
    """Per-slice weighted rms gamma and macro-particle count of the slices of
    beam_moments: slice s covers xi = z - <z> in [(s - h) L, (s - h + 1) L),
    s = 0 .. 2h - 1, h = ceil(n_sigma sigma_z / L), particles with
    |xi| <= n_sigma sigma_z only; the spread is 0 for a slice with fewer than
    min_per_slice particles."""
    z, g, w = (np.asarray(a, np.float64) for a in (z, gamma, w))
    W = w.sum()
    zm = float((w * z).sum() / W)
    sz = math.sqrt(float((w * (z - zm) ** 2).sum() / W))
    h = int(math.ceil(n_sigma * sz / slice_len)) if sz > 0 else 0
    xi = z - zm
    sel = np.abs(xi) <= n_sigma * sz
    sidx = np.floor(xi[sel] / slice_len).astype(np.int64) + h
    gs, ws = g[sel], w[sel]
    sg = np.zeros(2 * h)
    cnt = np.zeros(2 * h, np.int64)
    for k in range(2 * h):
        mk = sidx == k
        cnt[k] = int(mk.sum())
        if cnt[k] < min_per_slice:
            continue
        ww = ws[mk]
        Ws = ww.sum()
        gm = (ww * gs[mk]).sum() / Ws
        sg[k] = math.sqrt((ww * (gs[mk] - gm) ** 2).sum() / Ws)
    return sg, cnt


def err_sigma_gamma(slice_f, slice_inf):
    """Err_{sigma gamma}, Eq. (11): rms over slices of the relative deviation
    of the finite-order slice energy spread from the infinite-order one."""
    a = np.asarray(slice_f, np.float64)
    b = np.asarray(slice_inf, np.float64)
    return float(np.sqrt(np.mean(((a - b) / b) ** 2)))


def err_emittance(eps_f, eps_inf):
    """Err_eps, Eq. (12): relative emittance deviation."""
    return (eps_f - eps_inf) / eps_inf


def err_ez_pointwise(ez_f, ez_inf, floor: float = 1e-12):
    """Eq. (13) as printed: rms over the spectral cells of the relative
    deviation of FFT2(Ez) from the infinite-order spectrum.  Cells where the
    reference spectrum is below floor times its maximum are skipped (the ratio
    is undefined there); the mean runs over the remaining cells."""
    a = np.fft.fft2(ez_f)
    b = np.fft.fft2(ez_inf)
    keep = np.abs(b) > floor * np.abs(b).max()
    return float(np.sqrt(np.mean(np.abs((a[keep] - b[keep]) / b[keep]) ** 2)))


def err_ez_normalized(ez_f, ez_inf):
    """Normalized L2 form of Eq. (13): ||FFT2(Ez_f) - FFT2(Ez_inf)|| / ||FFT2(Ez_inf)||
    (the pointwise ratio of Eq. (13) is undefined where the reference spectrum
    vanishes, so the norm ratio is used)."""
    a = np.fft.fft2(ez_f)
    b = np.fft.fft2(ez_inf)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
