"""Write tests/golden/cp3_targets.json: the FP64 oracle's loss trajectory for the
CP 256^3, R = 32 workload (20 % missing) from its seeded Gamma(1, 1) init.

L* (the time-to-target threshold) is the oracle's loss after 200 plain sweeps
of Algorithm 1.  Only the oracle and the seeded input generator are used;
nothing here touches the GPU library.  Run: python tests/golden/make_targets.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2602_02759_amd import datagen  # noqa: E402

N_SWEEPS = 200
RECORD = (0, 1, 2, 5, 10, 20, 50, 100, 150, 200)


def run(alpha, beta):
    p = datagen.cp3(alpha, beta)
    f = [np.maximum(t, 1e-10).astype(np.float64) for t in p.init]
    trace = {0: O.loss(p.model_str, f, p.Y, p.M, alpha, beta)}
    t0 = time.time()
    for s in range(1, N_SWEEPS + 1):
        f = O.sweep(p.model_str, f, p.Y, p.M, alpha, beta, 1e-10)
        if s in RECORD:
            trace[s] = O.loss(p.model_str, f, p.Y, p.M, alpha, beta)
            print(f"(alpha,beta)=({alpha},{beta}) sweep {s}: loss {trace[s]:.10e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    return trace


def main():
    out = {"_source": "FP64 oracle (oracle/oracle.py), Algorithm 1 from the seeded init of "
                      "paper_2602_02759_amd.datagen.cp3; written by tests/golden/make_targets.py",
           "workload": "CP ir,jr,kr->ijk 256^3 R=32, Poisson(Gamma(0.3,1) CP), 20% missing",
           "eps": 1e-10, "targets": {}}
    for ab in ((1.0, 1.0), (0.5, 1.0)):
        tr = run(*ab)
        out["targets"][f"{ab[0]},{ab[1]}"] = {"loss_by_sweep": {str(k): v for k, v in tr.items()},
                                              "L_star": tr[N_SWEEPS]}
    with open(os.path.join(HERE, "cp3_targets.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
