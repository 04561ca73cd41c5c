"""Write grad16k_fd.json: FP64 central finite differences of the
differentiable-run loss on 32 seeded coordinates, from the oracle only.

Run: a Plummer sphere N = 16384 (seed 1005), eps = 1/512, 64 shared Hermite
steps of 1/512 (Section 2 predictor and corrector with every particle in
every step).  Loss L = (1/N) sum_i |x_i(T) - x*_i|^2 with the target
x* = x(T) of the same FP64 oracle run + 1e-3 * xi, xi ~ N(0, 1) (seed 2005).
Coordinates: 32 seeded (particle, axis) pairs of the initial positions
(seed 3005); dL/dx0 ~ (L(x0 + h e) - L(x0 - h e)) / 2h with h = 1e-6, and
with h = 5e-7 on the first four coordinates as a stability check.

This needs ~1e12 float64 pair interactions (tens of minutes on a few
cores); the GPU test reads the stored values instead of recomputing them.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads.plummer import CONFIGS, plummer  # noqa: E402


def target_and_coords(cfg, pos, vel, m):
    ex = cfg.extra
    xT = oracle.shared_run(pos, vel, m, cfg.eps2, ex["dt"], ex["steps"])[0]
    xi = np.random.default_rng(ex["target_seed"]).normal(size=xT.shape)
    target = xT + ex["target_sigma"] * xi
    rng = np.random.default_rng(ex["fd_seed"])
    parts = rng.choice(cfg.n, ex["n_coords"], replace=False)
    axes = rng.integers(0, 3, ex["n_coords"])
    return target, [(int(a), int(p)) for a, p in zip(axes, parts)]


def main():
    cfg = CONFIGS["grad16k"]
    ex = cfg.extra
    pos, vel, m = plummer(cfg.n, cfg.seed)
    t0 = time.time()
    target, coords = target_and_coords(cfg, pos, vel, m)

    def loss(p):
        x = oracle.shared_run(p, vel, m, cfg.eps2, ex["dt"], ex["steps"])[0]
        return float(((x - target) ** 2).sum() / cfg.n)

    out = {"_comment": __doc__.strip().splitlines()[0], "config": "grad16k", "coords": []}
    for k, (ax, p) in enumerate(coords):
        row = {"axis": ax, "particle": p}
        for name, h in (("fd", ex["fd_h"]), ("fd_half", ex["fd_h"] / 2)):
            if name == "fd_half" and k >= 4:
                continue
            xp, xm = pos.copy(), pos.copy()
            xp[ax, p] += h
            xm[ax, p] -= h
            row[name] = (loss(xp) - loss(xm)) / (2 * h)
        out["coords"].append(row)
        print("coord %d/%d (%d, %d): %.10e  [%.0f s]" % (k + 1, len(coords), ax, p, row["fd"],
                                                      time.time() - t0), flush=True)
    with open(os.path.join(HERE, "grad16k_fd.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
