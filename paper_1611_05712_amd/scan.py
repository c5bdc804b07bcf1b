"""Parameter scans: many independent runs of the PIC cycle on one GPU.

Each run is its own context (own workspace and stream).  `run_batched`
advances all of them together: per context two steps at a time as replays of
its captured HIP graph, interleaved over the contexts' streams so small runs
overlap on the GPU (pic_batch_step); the launch parameters of each context are
first chosen by the library's autotuner.  The scan's figure of merit is the
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
