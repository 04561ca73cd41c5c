"""Write plummer64k_run.json: the oracle's own block-step run of the
Plummer N = 65536 workload (seed 1002, eps = 1/1024, eta = 0.02,
eta_s = 0.01, dt_max = 1/8, t: 0 -> 1/8), from the oracle only.

Stored: block steps, sum of block sizes, energy (K + W, softened, j != i)
at t = 0 and t = 1/8 and the relative drift per time unit.  The Hermite
scheme of Section 2 with the Aarseth step criterion conserves energy only
to its truncation error, so the GPU run is gated against this float64
run's drift rather than against an absolute bound.

About 2e11 float64 pair interactions (minutes on a few cores).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads.plummer import CONFIGS, plummer  # noqa: E402


def main():
    cfg = CONFIGS["plummer64k"]
    pos, vel, m = plummer(cfg.n, cfg.seed)
    e0 = sum(oracle.energy(pos, vel, m, cfg.eps2))
    s = oracle.init_state(pos, vel, m, cfg.eps2, eta=cfg.eta, eta_s=cfg.eta_s,
                          dt_max=cfg.dt_max)
    t0 = time.time()
    steps, block_sum = oracle.integrate(s, cfg.t_end)
    wall = time.time() - t0
    e1 = sum(oracle.energy(s.x, s.v, m, cfg.eps2))
    out = {
        "workload": "plummer N=65536 seed=1002 eps=1/1024 eta=0.02 eta_s=0.01 "
                    "dt_max=1/8 t_end=1/8",
        "steps": steps,
        "block_sum": block_sum,
        "e0": e0,
        "e1": e1,
        "drift_per_time_unit": abs((e1 - e0) / e0) / cfg.t_end,
        "oracle_seconds": wall,
        "oracle_threads": oracle.num_threads(),
    }
    with open(os.path.join(HERE, "plummer64k_run.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
