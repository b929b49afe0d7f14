"""Writes the oracle regression fixtures in this folder.

The paper prints no worked numerical example of the substep (its only numbers
are timings, Table "Computational Time of Each Component"), so these fixtures
are produced by the FP64 oracle alone, on seeded synthetic scenes, and pin the
oracle against unintended changes.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from paper_2402_01181_amd import scenes  # noqa: E402

SAMPLE = [0, 1, 777, 4095, 8191]


def cube_50():
    sc = scenes.cube_scene(seed=1, substeps=50)
    sim = orc.Sim(sc.envs[0], sc.dt, bound=sc.bound)
    sim.run(sc.substeps)
    st = sim.state
    return {
        "scene": "cube_scene(seed=1), 8192 particles, 32^3, dt 1e-4, 50 substeps, no tool",
        "flags": int(sim.flags),
        "centroid": st.x.mean(0).tolist(),
        "mean_v": st.v.mean(0).tolist(),
        "sample_ids": SAMPLE,
        "x": st.x[SAMPLE].tolist(),
        "v": st.v[SAMPLE].tolist(),
        "F": st.F[SAMPLE].tolist(),
    }


def slab_small_40():
    sc = scenes.small_slab_scene(seed=17, n_particles=3000, n=32, substeps=40)
    sim = orc.Sim(sc.envs[0], sc.dt, bound=sc.bound)
    sim.run(sc.substeps)
    st = sim.state
    ids = [0, 10, 1500, 2999]
    return {
        "scene": "small_slab_scene(seed=17, 3000 particles, 32^3, 40 substeps), capsule pushing at 0.2 m/s, slip, friction 0.3",
        "flags": int(sim.flags),
        "centroid": st.x.mean(0).tolist(),
        "mean_v": st.v.mean(0).tolist(),
        "tool_T": sim.T[0].tolist(),
        "sample_ids": ids,
        "x": st.x[ids].tolist(),
        "v": st.v[ids].tolist(),
        "F": st.F[ids].tolist(),
    }


if __name__ == "__main__":
    orc.build()
    for name, fn in (("cube_50.json", cube_50), ("slab_small_40.json", slab_small_40)):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
        print("wrote", name)
