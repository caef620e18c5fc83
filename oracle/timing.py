"""Timing of the oracle on host cores (a reported baseline, not a target).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Times a bounded, seeded sample of per-atom solves with every available core
(one BLAS thread per worker process) and scales linearly in N to whole-step
figures; the method's cost is O(n^3 N) at fixed cluster size (Sec. 2), so
per-atom time times N is the step time.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import tb


def time_atom_solves(pos, cell, periodic, p, r_cut, r, n_sample, seed=0,
                     processes=None, seeds="block", group=1):
    N = pos.shape[0]
    rng = np.random.default_rng(seed)
    atoms = sorted(rng.choice(N, size=min(n_sample, N), replace=False).tolist())
    if processes is None:
        processes = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    tb.solve_atoms(atoms, pos, cell, periodic, p, r_cut, r, processes=processes, seeds=seeds, group=group)
    dt = time.perf_counter() - t0
    per_atom = dt / len(atoms)
    return {"n_sample": len(atoms), "seconds": dt, "cores": processes,
            "atom_solves_per_s": len(atoms) / dt,
            "steps_per_s": 1.0 / (per_atom * N)}
