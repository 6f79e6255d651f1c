"""Write configs/<workload>.json: the parameters of every synthetic workload
(grid, species, profile, run parameters), as synth.workloads() defines them.

    python -m synth.write_configs

The files are a readable record of each workload; synth.workloads() is what the
tests and the benchmark use, and tests/test_synth.py checks that the two agree."""
from __future__ import annotations

import dataclasses
import json
import os

from synth import PROF_HARRIS2, PROF_SHOCK_TUBE, PROF_UNIFORM, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "configs")
PROFILES = {PROF_UNIFORM: "uniform", PROF_SHOCK_TUBE: "shock_tube", PROF_HARRIS2: "double_harris"}
BCS = {0: "periodic", 1: "wall", 2: "inflow"}


def config(wl) -> dict:
    d = dataclasses.asdict(wl)
    d = {k: (list(v) if isinstance(v, tuple) else v) for k, v in d.items()}
    d["profile"] = PROFILES.get(wl.profile, wl.profile)
    d["a_mode"] = {0: "light", 1: "bulk"}[wl.a_mode]
    d["x_boundaries"] = [BCS[b] for b in wl.bc]
    del d["bc"]
    d["particles"] = wl.nparticles()
    d["physical_cells"] = wl.nphys
    return d


def render(wl) -> str:
    return json.dumps(config(wl), indent=1, sort_keys=True) + "\n"


def main():
    os.makedirs(OUT, exist_ok=True)
    for name, wl in workloads().items():
        with open(os.path.join(OUT, f"{name}.json"), "w") as f:
            f.write(render(wl))


if __name__ == "__main__":
    main()
