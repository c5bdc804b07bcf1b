"""Writes the stored expected values of the long oracle runs (FP64 CPU oracle
only; no GPU code is imported).  Run from the repository root:

    python tests/golden/make_oracle_runs.py

c0_oracle.json: the 256 x 64, 2-mode, p = 16 moving-window beam-plasma
workload (seed 0) advanced 50 steps; drive-bunch moments after 1, 10, 25 and
50 steps, the live particle count, and per (mode, component) field L2 norms
after 1 and 50 steps together with 64 sampled nodes after 1 step.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.cycle import OracleSim          # noqa: E402
from oracle.diag import beam_moments        # noqa: E402
from workloads import preset                # noqa: E402

COMPS = ["E+", "E-", "Ez", "B+", "B-", "Bz"]
SLICE = 0.02975    # 0.5 um at n0 = 1e23 m^-3, in 1/k_p


def fields(sim):
    out = {}
    for m in range(sim.M):
        for c, name in enumerate(COMPS):
            F = (sim.E if c < 3 else sim.B)[m, c % 3]
            out[f"{m}:{name}"] = float(np.linalg.norm(F))
    return out


def main():
    wl = preset("c0")
    sim = OracleSim(wl)
    rng = np.random.default_rng(1234)
    idx = np.stack([rng.integers(0, wl.nr, 64), rng.integers(0, wl.nz, 64)], axis=1)
    res = {"workload": "c0", "seed": 0, "steps": {}, "sample_nodes": idx.tolist()}
    t0 = time.time()
    for n in range(1, 51):
        sim.step(1)
        if n in (1, 10, 25, 50):
            s = sim.species_by_name("drive")
            mom = beam_moments(s.x, s.y, s.z, s.ux, s.uy, s.uz, s.w, slice_len=SLICE)
            entry = {"drive": mom,
                     "n_mobile": int(sum(sp.x.size for sp in sim.species if sp.mobile)),
                     "field_norm": fields(sim)}
            if n == 1:
                samples = {}
                for m in range(sim.M):
                    for c, name in enumerate(COMPS):
                        F = (sim.E if c < 3 else sim.B)[m, c % 3]
                        v = F[idx[:, 0], idx[:, 1]]
                        samples[f"{m}:{name}"] = [[float(a.real), float(a.imag)] for a in v]
                entry["samples"] = samples
            res["steps"][str(n)] = entry
            print(f"step {n}: {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c0_oracle.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
