"""Write tests/golden/<workload>_sweep1.npz: one sweep of the FP64 oracle
from the seeded, clamped init of the paper-shape workloads that are too large
for the oracle to run inside a GPU test -- the ICEWS string at 249 x 249 x 20
x 228 (283 M entries) and the Uber string at the 400 x 400 mesh (726 M
entries).  The oracle evaluates them slab by slab along the first mode
(``sweep_slabs``, ``loss_slabs``).  Stored: the factors after the sweep
(float64) and the loss before and after it.  Only the oracle and the seeded
input generator are used.  Run: python tests/golden/make_big_sweeps.py [icews|uber400]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2602_02759_amd import datagen  # noqa: E402

WORKLOADS = {"icews": (datagen.icews_problem, 24), "uber400": (lambda: datagen.uber_problem(mesh=400), 27)}


def run(name):
    make, n_slabs = WORKLOADS[name]
    t0 = time.time()
    p = make()
    print(f"{name}: data {p.Y.shape} in {time.time() - t0:.0f} s", flush=True)
    f0 = [np.maximum(t, np.float32(1e-10)).astype(np.float64) for t in p.init]
    l0 = O.loss_slabs(p.model_str, f0, p.Y, p.M, p.alpha, p.beta, n_slabs)
    f1 = O.sweep_slabs(p.model_str, f0, p.Y, p.M, p.alpha, p.beta, 1e-10, n_slabs)
    l1 = O.loss_slabs(p.model_str, f1, p.Y, p.M, p.alpha, p.beta, n_slabs)
    print(f"{name}: loss {l0:.10e} -> {l1:.10e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, f"{name}_sweep1.npz"), loss0=l0, loss1=l1,
                        **{f"f{i}": f for i, f in enumerate(f1)},
                        source=np.array(f"FP64 oracle sweep_slabs, {n_slabs} slabs, from the seeded init of "
                                        f"paper_2602_02759_amd.datagen ({p.model_str}, {p.sizes}); "
                                        "written by tests/golden/make_big_sweeps.py"))


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        run(name)
