"""Parameter scans: many independent runs of the PIC cycle on one GPU.

Each run is its own context (own workspace and stream).  `run_batched`
advances all of them together as replays of one HIP graph that holds two
steps of every context, each on its own stream (pic_batch_step), so one launch
advances the whole batch and small runs overlap on the GPU; the launch
parameters of each context are first chosen by the library's autotuner.  The scan's figure of merit is the
witness slice energy spread, the quantity the paper tracks against the
stencil order (Sec. "Accurate modeling of plasma accelerators in finite order
PSATD"): the mean over 0.5 um slices within +-3 sigma_z of the slice gamma
spread, relative to the mean gamma.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

from .pic import Simulation, batch_step

SLICE_LEN = 0.02975   # 0.5 um at n0 = 1e23 m^-3, in 1/k_p


def slice_energy_spread(sim: Simulation, species: str = "witness") -> float:
    """Mean slice sigma_gamma / <gamma> of a species (pic_diagnostics); NaN
    when the species has no live particle or no populated slice."""
    d = sim.diagnostics(species, slice_len=SLICE_LEN, allow_nan=True)
    if d["n"] == 0 or d["n_slices"] == 0 or not d["mean_gamma"] > 0:
        return float("nan")
    return d["mean_slice_sigma_gamma"] / d["mean_gamma"]


def run_batched(sims: Sequence[Simulation], steps: int, tune_steps: int = 2) -> Dict[str, object]:
    """Autotune every context (the trial steps count towards `steps`), then
    advance all contexts to `steps` steps in one batch.  Returns the chosen
    tunings, the wall time of everything (tuning included) and of the batch."""
    for s in sims:
        s.sync()
    t_all = time.perf_counter()
    tunings = []
    for s in sims:
        tunings.append(s.autotune(tune_steps) if tune_steps else s.tuning())
    done = [s.state()[1] for s in sims]
    left = min(max(0, steps - d) for d in done)
    # contexts that tuned further than others catch up first
    for s, d in zip(sims, done):
        extra = max(0, steps - d) - left
        if extra:
            s.step_graph(extra)
    for s in sims:
        s.sync()
    t0 = time.perf_counter()
    batch_step(list(sims), left)
    for s in sims:
        s.sync()
    t1 = time.perf_counter()
    return {"tunings": tunings, "total_s": t1 - t_all, "batch_s": t1 - t0, "batch_steps": left}


def run_plain(sim: Simulation, steps: int) -> float:
    """Eager steps (no graph), synchronized; returns the wall time."""
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    return time.perf_counter() - t0


# ---------------------------------------------------------------------------
# finite-order error scan: training data of the order surrogate
# ---------------------------------------------------------------------------
def err_sigma_gamma(sg_f, cnt_f, sg_inf, cnt_inf, min_per_slice: int = 10) -> float:
    """Err_sigma_gamma of Eq. (11): rms over the slices populated in both runs of
    the relative deviation of the finite-order slice rms gamma from the
    infinite-order one.  Slices are matched by their offset from the beam
    centroid (slice k of an n-slice list covers xi in [(k - n/2) L, ...))."""
    import numpy as np
    hf, hi = len(sg_f) // 2, len(sg_inf) // 2
    h = min(hf, hi)
    dev = []
    for off in range(-h, h):
        a, na = sg_f[hf + off], cnt_f[hf + off]
        b, nb = sg_inf[hi + off], cnt_inf[hi + off]
        if na >= min_per_slice and nb >= min_per_slice and b > 0:
            dev.append((a - b) / b)
    return float(np.sqrt(np.mean(np.square(dev)))) if dev else float("nan")


def witness_state(sim: Simulation):
    d, sg, cnt = sim.diagnostics_slices("witness", slice_len=SLICE_LEN, allow_nan=True)
    return {"eps_nx": d["eps_nx"], "eps_ny": d["eps_ny"], "mean_gamma": d["mean_gamma"],
            "mean_slice_sigma_gamma": d["mean_slice_sigma_gamma"], "n": d["n"], "nan_flag": d["nan_flag"],
            "slice_sigma_gamma": [float(v) for v in sg], "slice_count": [int(v) for v in cnt]}


def ncr_error_scan(n_tuples: int, steps: int, seed: int = 1, group: int = 4, log=None,
                   device: str = "cuda:0", first: int = 0) -> Dict[str, object]:
    """Runs every physical tuple of a seeded scan at every stencil order
    (8 ... 64 and infinite), `group` tuples at a time in one batch, and returns
    per tuple the witness state of every run and, per finite order, the
    paper's Err_sigma_gamma (Eq. (11)) and Err_eps (Eq. (12), on eps_n,x)
    against the infinite-order twin.  `first` skips the first tuples of the
    seeded sequence (tuple k is the same set-up whatever the range), so a long
    scan can be run in parts and merged."""
    import numpy as np
    from workloads import scan_instances, scan_workload
    insts = [i for i in scan_instances(n_tuples=first + n_tuples, seed=seed, extra=0) if i.tuple_index >= first]
    by_tuple: Dict[int, list] = {}
    for i in insts:
        by_tuple.setdefault(i.tuple_index, []).append(i)
    tuples = []
    t_run = 0.0
    keys = sorted(by_tuple)
    for g0 in range(0, len(keys), group):
        batch = [i for k in keys[g0:g0 + group] for i in by_tuple[k]]
        sims = []
        for inst in batch:
            wl = scan_workload(inst, steps)
            sims.append(Simulation.from_workload(wl, device=device))
            del wl
        r = run_batched(sims, steps, tune_steps=0)
        t_run += r["batch_s"]
        states = [witness_state(s) for s in sims]
        for s in sims:
            s.close()
        for k in keys[g0:g0 + group]:
            runs = {inst.order: st for inst, st in zip(batch, states) if inst.tuple_index == k}
            inst0 = by_tuple[k][0]
            ref = runs[0]
            errs = {}
            for p, st in runs.items():
                if p == 0:
                    continue
                esg = err_sigma_gamma(st["slice_sigma_gamma"], st["slice_count"], ref["slice_sigma_gamma"],
                                      ref["slice_count"])
                eeps = (st["eps_nx"] - ref["eps_nx"]) / ref["eps_nx"] if ref["eps_nx"] > 0 else float("nan")
                errs[str(p)] = {"err_sigma_gamma": esg, "err_eps": eeps}
            tuples.append({"tuple": k, "nz": inst0.nz, "nr": inst0.nr, "dz": inst0.dz, "dr": inst0.dr,
                           "gamma_w": inst0.gamma_w, "charge_w_pC": inst0.charge_w_C * 1e12,
                           "seed": inst0.seed, "errors": errs,
                           "runs": {str(p): {kk: v for kk, v in st.items() if not kk.startswith("slice_")}
                                    for p, st in runs.items()}})
        if log:
            log(f"tuples {g0 + 1}-{min(g0 + group, len(keys))} of {len(keys)} done ({t_run:.1f} s of batched steps)")
    return {"steps": steps, "seed": seed, "orders": [p for p in sorted({i.order for i in insts}) if p],
            "tuples": tuples, "batched_s": t_run}


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="finite-order error scan (training data of the order surrogate)")
    ap.add_argument("--tuples", type=int, default=48)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--group", type=int, default=4)
    ap.add_argument("--first", type=int, default=0, help="first tuple index of this part of the scan")
    ap.add_argument("--out", required=True)
    ap.add_argument("--merge", nargs="*", default=None, metavar="PART",
                    help="instead of running: merge scan parts (same seed and steps) into --out")
    a = ap.parse_args()
    if a.merge:
        parts = [json.load(open(f)) for f in a.merge]
        assert len({(q["seed"], q["steps"]) for q in parts}) == 1, "parts of different scans"
        tuples = sorted((t for q in parts for t in q["tuples"]), key=lambda t: t["tuple"])
        assert len({t["tuple"] for t in tuples}) == len(tuples), "overlapping parts"
        res = dict(parts[0], tuples=tuples, batched_s=sum(q["batched_s"] for q in parts))
    else:
        res = ncr_error_scan(a.tuples, a.steps, a.seed, a.group, log=lambda m: print(m, file=sys.stderr, flush=True),
                             first=a.first)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {a.out}: {len(res['tuples'])} tuples", file=sys.stderr)
