"""Write tests/golden/cp3_targets.json: the FP64 oracle's loss trajectory for the
CP 256^3, R = 32 workload (20 % missing) from its seeded Gamma(1, 1) init.

Two targets per (alpha, beta):
  L_star  the loss after 200 plain sweeps of Algorithm 1 (the time-to-target
          threshold of the benchmark);
  L_conv  the loss of the state at which the stopping rule of App. B fires
          (relative decrease below 1e-6; cap 5000 sweeps), with that sweep.
Only the oracle and the seeded input generator are used; nothing here touches
the GPU library.  Run: python tests/golden/make_targets.py
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
REL_TOL = 1e-6
CAP = 5000
RECORD = {0, 1, 2, 5, 10, 20, 50, 100, 150, 199, 200}


def run(alpha, beta):
    p = datagen.cp3(alpha, beta)
    f = [np.maximum(t, 1e-10).astype(np.float64) for t in p.init]
    losses = [O.loss(p.model_str, f, p.Y, p.M, alpha, beta)]
    t0 = time.time()
    t = 0
    while True:
        r = O.stop_reason(t, losses, None, 0, REL_TOL, CAP)
        if r is not None and t >= N_SWEEPS:
            break
        f = O.sweep(p.model_str, f, p.Y, p.M, alpha, beta, 1e-10)
        t += 1
        losses.append(O.loss(p.model_str, f, p.Y, p.M, alpha, beta))
        if t in RECORD or t % 50 == 0:
            print(f"(alpha,beta)=({alpha},{beta}) sweep {t}: loss {losses[t]:.10e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    stop = next(s for s in range(len(losses)) if O.stop_reason(s, losses, None, 0, REL_TOL, CAP) is not None)
    rec = {str(k): losses[k] for k in sorted(RECORD | {stop}) if k < len(losses)}
    return {"loss_by_sweep": rec, "L_star": losses[N_SWEEPS], "L_conv": losses[stop],
            "stop_sweep": stop}


def main():
    out = {"_source": "FP64 oracle (oracle/oracle.py), Algorithm 1 from the seeded init of "
                      "paper_2602_02759_amd.datagen.cp3; written by tests/golden/make_targets.py",
           "workload": "CP ir,jr,kr->ijk 256^3 R=32, Poisson(Gamma(0.3,1) CP), 20% missing",
           "eps": 1e-10, "rel_tol": REL_TOL, "targets": {}}
    for ab in ((1.0, 1.0), (0.5, 1.0)):
        out["targets"][f"{ab[0]},{ab[1]}"] = run(*ab)
    with open(os.path.join(HERE, "cp3_targets.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
