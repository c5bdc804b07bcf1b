"""The paper's accuracy study on one GPU: the same beam-plasma set-up run at
several stencil orders for 35 mm, each compared with the infinite-order run
(Sec. "Accurate modeling of plasma accelerators in finite order PSATD",
Eqs. (11)-(13)).

    python -m paper_1611_05712_amd.accuracy --orders 4 8 0 --out DIR
    python -m paper_1611_05712_amd.accuracy --report DIR

A run writes DIR/run_p<order>.json (witness and drive moments and the witness
slice energy spreads at regular marks) and DIR/ez_p<order>.npy (the final
on-grid E_z of mode 0); the report computes Err_sigma_gamma (Eq. (11), slices
matched by offset from the centroid), Err_eps (Eq. (12), on eps_n,x) and the
normalized form of Err_Ez (Eq. (13)) of every finite order against p = inf,
and locates the numerical Cherenkov excess in the E_z spectrum against the
resonance of Eq. (10) for the drive beam.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from .pic import Simulation
from .scan import SLICE_LEN, err_sigma_gamma

WITNESS_OFFSET = 4.463      # 1/k_p (75 um): the accelerating phase near the back of the first bubble


def _state(sim, name):
    d, sg, cnt = sim.diagnostics_slices(name, slice_len=SLICE_LEN, allow_nan=True)
    out = {k: d[k] for k in ("eps_nx", "eps_ny", "mean_gamma", "sigma_gamma", "mean_slice_sigma_gamma", "z_mean",
                             "sigma_z", "n", "n_slices", "nan_flag")}
    out["slice_sigma_gamma"] = [float(v) for v in sg]
    out["slice_count"] = [int(v) for v in cnt]
    return out


def run_order(order: int, steps: int, outdir: str, marks: int = 25_000, device="cuda:0", log=print,
              witness_offset: float = WITNESS_OFFSET, witness_mev: float = 25.0, filter: int = 0):
    from workloads import paper_accuracy
    wl = paper_accuracy(order, witness_offset, witness_mev=witness_mev, filter=filter)
    t0 = time.perf_counter()
    sim = Simulation.from_workload(wl, device=device)
    init_s = time.perf_counter() - t0
    del wl
    rec = {"order": order, "steps": steps, "marks": [], "init_s": init_s, "witness_mev": witness_mev,
           "filter": filter}
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        n = min(marks, steps - done)
        sim.step_graph(n)
        done += n
        w = _state(sim, "witness")
        dr = _state(sim, "drive")
        el = time.perf_counter() - t0
        rec["marks"].append({"step": done, "witness": w,
                             "drive": {k: v for k, v in dr.items() if not k.startswith("slice_")}})
        log(f"p={order} step {done}/{steps} ({el:.0f} s): witness <gamma> {w['mean_gamma']:.2f} "
            f"slice sigma_gamma {w['mean_slice_sigma_gamma']:.4f} eps_nx {w['eps_nx']:.5f} n {w['n']}")
    rec["run_s"] = time.perf_counter() - t0
    rec["ms_per_step"] = rec["run_s"] / steps * 1e3
    ez = sim.get_field(0, "Ez")
    sim.close()
    os.makedirs(outdir, exist_ok=True)
    np.save(os.path.join(outdir, f"ez_p{order}.npy"), ez)
    with open(os.path.join(outdir, f"run_p{order}.json"), "w") as f:
        json.dump(rec, f)
    return rec


def modified_kz(kz, dz: float, order: int):
    """[k_z] of Eq. (5), sum_j alpha_{n,j} sin(k_z j dz) / (j dz) with p = 2n; the
    coefficients of Eq. (3) by their ratio alpha_{n,j+1}/alpha_{n,j} =
    -(n - j)/(n + j + 1) from alpha_{n,1} = 2n/(n + 1).  order 0: k_z itself,
    zero at the Nyquist wavenumber pi/dz (the limit of every finite order)."""
    kz = np.asarray(kz, np.float64)
    if order == 0:
        out = kz.copy()
        out[np.abs(np.abs(kz * dz) - np.pi) <= 1e-12 * np.pi] = 0.0   # Nyquist column
        return out
    n = order // 2
    a = 2.0 * n / (n + 1.0)
    out = np.zeros_like(kz)
    for j in range(1, n + 1):
        out += a * np.sin(kz * j * dz) / (j * dz)
        a *= -(n - j) / (n + j + 1.0)
    return out


def resonance_kz(gamma: float, order: int, dz: float) -> float:
    """On-axis (k_perp = 0) numerical Cherenkov resonance of Eq. (10): the
    smallest k_z in (0, pi/dz) where the numerical phase velocity [k_z]/k_z
    drops to the beam speed; NaN when there is none (infinite order)."""
    beta = np.sqrt(1.0 - 1.0 / gamma ** 2)
    k = np.linspace(1e-6, np.pi / dz * (1.0 - 1e-9), 200_001)   # (0, pi/dz): the Nyquist column itself is excluded
    f = modified_kz(k, dz, order) / k - beta
    idx = np.nonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0]
    if idx.size == 0:
        return float("nan")
    lo, hi = k[idx[0]], k[idx[0] + 1]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if np.sign(modified_kz(np.array([mid]), dz, order)[0] / mid - beta) == np.sign(f[idx[0]]):
            lo = mid
        else:
            hi = mid
    return float(0.5 * (lo + hi))


def ez_excess_peak(ez_f, ez_inf, dz: float, rows: int):
    """k_z at which the z-spectrum of E_z (mode 0, averaged over the first
    `rows` radial rows) most exceeds that of the infinite-order run."""
    sf = np.abs(np.fft.fft(ez_f[:rows], axis=-1)).mean(axis=0)
    si = np.abs(np.fft.fft(ez_inf[:rows], axis=-1)).mean(axis=0)
    nz = ez_f.shape[-1]
    kz = 2.0 * np.pi * np.fft.fftfreq(nz, dz)
    sel = (kz > 0.05 * np.pi / dz)
    ratio = np.where(sel, sf / np.maximum(si, 1e-30 * si.max()), 0.0)
    i = int(np.argmax(ratio))
    return float(kz[i]), float(ratio[i])


def errors(run_f, run_inf, ez_f=None, ez_inf=None, mark=-1):
    a = run_f["marks"][mark]["witness"]
    b = run_inf["marks"][mark]["witness"]
    out = {"order": run_f["order"], "step": run_f["marks"][mark]["step"],
           "err_sigma_gamma": err_sigma_gamma(a["slice_sigma_gamma"], a["slice_count"], b["slice_sigma_gamma"],
                                              b["slice_count"]),
           "err_eps": (a["eps_nx"] - b["eps_nx"]) / b["eps_nx"]}
    if ez_f is not None and ez_inf is not None:
        fa, fb = np.fft.fft2(ez_f), np.fft.fft2(ez_inf)
        out["err_ez"] = float(np.linalg.norm(fa - fb) / np.linalg.norm(fb))
    return out


def report(outdir: str, reference: int = 0):
    """Errors of every other order against the `reference` order's run
    (0 = infinite order, the paper's reference)."""
    runs = {}
    for f in os.listdir(outdir):
        if f.startswith("run_p") and f.endswith(".json"):
            r = json.load(open(os.path.join(outdir, f)))
            runs[r["order"]] = r
    if reference not in runs:
        raise SystemExit(f"no run of the reference order p = {reference} in " + outdir)
    ez = {p: np.load(os.path.join(outdir, f"ez_p{p}.npy")) for p in runs
          if os.path.exists(os.path.join(outdir, f"ez_p{p}.npy"))}
    from workloads import PAPER_DZ, M_E_MEV
    g_drive = 1.0 + 1000.0 / M_E_MEV
    rows = []
    for p in sorted(k for k in runs if k != reference):
        e = errors(runs[p], runs[reference], ez.get(p), ez.get(reference))
        if p and p in ez and reference in ez:
            kpk, ratio = ez_excess_peak(ez[p], ez[reference], PAPER_DZ, ez[p].shape[0] // 8)
            e["ez_excess_kz_dz"] = kpk * PAPER_DZ
            e["ez_excess_ratio"] = ratio
            e["resonance_kz_dz_drive"] = resonance_kz(g_drive, p, PAPER_DZ) * PAPER_DZ
        rows.append(e)
    return {"reference": reference, "rows": rows,
            "final": {p: {k: r["marks"][-1][b][k] for b in ("witness",) for k in
                          ("mean_gamma", "mean_slice_sigma_gamma", "eps_nx", "n")} | {
                          "drive_eps_nx": r["marks"][-1]["drive"]["eps_nx"]} for p, r in runs.items()},
            "ms_per_step": {p: r["ms_per_step"] for p, r in runs.items()}}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--orders", type=int, nargs="*", default=[])
    ap.add_argument("--steps", type=int, default=175_000)
    ap.add_argument("--marks", type=int, default=25_000)
    ap.add_argument("--out", default="accuracy_runs")
    ap.add_argument("--witness-mev", type=float, default=25.0,
                    help="witness kinetic energy (the paper's set-up: 25 MeV)")
    ap.add_argument("--filter", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="binomial J/rho filter passes (pic_config.filter)")
    ap.add_argument("--report", metavar="DIR")
    ap.add_argument("--reference", type=int, default=0, help="reference order of the report (0 = infinite)")
    a = ap.parse_args(argv)
    if a.report:
        print(json.dumps(report(a.report, a.reference), indent=1))
        return
    for p in a.orders:
        run_order(p, a.steps, a.out, a.marks, log=lambda m: print(m, file=sys.stderr, flush=True),
                  witness_mev=a.witness_mev, filter=a.filter)


if __name__ == "__main__":
    main()
