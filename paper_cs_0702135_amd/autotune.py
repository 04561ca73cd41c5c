"""Autotuner for the pair-kernel launch shapes.

For a given j-count it times candidate shapes (coordinate form, i-particles
per lane, waves per workgroup, split target) at a ladder of active-block
sizes with HIP events, keeps the fastest per size, and installs the result
as the context's tuning table (nbody_tune_set): each measured size covers
the range up to the geometric midpoint with its neighbours.  Tables are
cached as JSON next to this file, keyed by device name, j-count bucket and
accumulation mode.

Candidates use the float64-difference coordinate form (rep 0); the
float-float form (rep 1) measured slower on gfx950 and is only tried with
`forms=(0, 1)`; the float32-velocity form (rep 2) changes the jerk's
accuracy and is only tried when asked for explicitly.  Small blocks also try
the j-lane layout (layout 1: one j per lane, a few wave-uniform i), and the
table's small-block entry is what the block-step driver launches beside its
i-lane kernel.

The ensemble (nbody_ensemble_run) is calibrated separately
(calibrate_ensemble): every compiled workgroup shape at two occupancies on a
representative launch, with its team-planning model refitted on the measured
per-cluster times, keeping the fastest measured launch.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import ForceShape, force, tune_clear, tune_set

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_DIR = os.path.join(HERE, "tuned")

LADDER = (1, 16, 64, 256, 1024, 4096, 16384, 65536, 262144, 1 << 20, 1 << 22)


def _bucket(n_j: int) -> int:
    return 1 << max(0, int(round(math.log2(max(1, n_j)))))


def cache_path(n_j: int, mode: str) -> str:
    name = torch.cuda.get_device_properties(0).name if torch.cuda.is_available() else "cpu"
    arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", name).split(":")[0] \
        if torch.cuda.is_available() else "cpu"
    return os.path.join(CACHE_DIR, "%s_nj%d_%s.json" % (arch, _bucket(n_j), mode))


JL_MAX_TRY = 512  # largest block given j-lane candidates


def candidates(n_i: int, n_j: int, forms=(0,)):
    out = []
    if n_i <= JL_MAX_TRY:
        # one j per lane, the workgroup's C i-particles shared by all lanes
        for c in (1, 2, 4, 8):
            if c > 1 and c > 2 * n_i:
                continue
            for w in (1, 2, 4):
                for tg in (256, 512, 2048, 8192):
                    out.append(ForceShape(0, c, w, 128, 64, tg, 1))
    for rep in forms:
        for it in (1, 2, 4):
            if n_i <= 64 and it > 1:
                continue
            for w in (1, 2, 4, 8):
                if it == 4 and w == 8:  # not compiled (registers)
                    continue
                for tg in (8192, 32768, 65536, 131072, 262144):
                    out.append(ForceShape(rep, it, w, 128, 64, tg))
    return out


def _time_shape(shape, pos, vel, mass, eps2, act, mode, reps):
    tune_clear()
    tune_set(0, 1 << 62, shape)
    force(pos, vel, mass, eps2, act, mode)  # warm-up (and allocation)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        force(pos, vel, mass, eps2, act, mode)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(pos, vel, mass, eps2, mode="fp32", ladder=None, forms=(0,),
         budget_interactions=4e11, log=None):
    """Measure the ladder of block sizes on the given particles.

    Returns {"n_j": n, "mode": mode, "entries": [[n_i, shape_dict, ms], ...]}.
    """
    n = mass.shape[0]
    ladder = [k for k in (ladder or LADDER) if k <= n]
    if n not in ladder:
        ladder.append(n)
    gen = torch.Generator(device="cpu").manual_seed(12345)
    entries = []
    for n_i in ladder:
        act = None if n_i == n else \
            torch.sort(torch.randperm(n, generator=gen)[:n_i])[0].to(torch.int32).cuda()
        work = float(n_i) * n
        reps = int(max(1, min(20, budget_interactions / 50 / max(work, 1.0))))
        best = None
        for shape in candidates(n_i, n, forms):
            ms = _time_shape(shape, pos, vel, mass, eps2, act, mode, reps)
            if best is None or ms < best[1]:
                best = (shape, ms)
        entries.append([n_i, best[0].asdict(), best[1]])
        if log:
            log("tune n_j=%d n_i=%d: %r %.3f ms (%.3e interactions/s)"
                % (n, n_i, best[0], best[1], work / best[1] * 1e3))
    tune_clear()
    return {"n_j": n, "mode": mode, "entries": entries}


def install(table, dynamic_n_i=None):
    """Install a tuned table into the current device's context.

    Each measured n_i covers [geometric midpoint below, midpoint above).  The
    block-step driver's shape is the one measured closest to `dynamic_n_i`
    (default: the smallest measured size above 1).
    """
    tune_clear()
    ent = sorted(table["entries"], key=lambda e: e[0])
    sizes = [e[0] for e in ent]
    for k, (n_i, shape, _) in enumerate(ent):
        lo = 0 if k == 0 else int(math.sqrt(sizes[k - 1] * n_i)) + 1
        hi = (1 << 62) if k == len(ent) - 1 else int(math.sqrt(n_i * sizes[k + 1])) + 1
        tune_set(lo, hi, ForceShape(**shape))
    if ent:
        target = dynamic_n_i or (sizes[1] if len(sizes) > 1 else sizes[0])
        pick = min(ent, key=lambda e: abs(math.log2(e[0]) - math.log2(max(1, target))))
        tune_set(-1, 0, ForceShape(**pick[1]))
        # the driver's small blocks: the j-lane shape of the largest of the
        # smallest measured sizes that all chose it, up to the midpoint with
        # the next size
        k = 0
        while k < len(ent) and ent[k][1].get("layout", 0) == 1:
            k += 1
        if k > 0 and pick[1].get("layout", 0) == 0:
            jl_max = int(math.sqrt(sizes[k - 1] * sizes[k])) if k < len(ent) else sizes[k - 1]
            tune_set(-2, jl_max, ForceShape(**ent[k - 1][1]))


def load(n_j, mode="fp32"):
    p = cache_path(n_j, mode)
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return None


def save(table):
    os.makedirs(CACHE_DIR, exist_ok=True)
    p = cache_path(table["n_j"], table["mode"])
    with open(p, "w") as f:
        json.dump(table, f, indent=1)
    return p


def load_or_tune(pos, vel, mass, eps2, mode="fp32", log=None, dynamic_n_i=None, **kw):
    n = mass.shape[0]
    table = load(n, mode)
    if table is None:
        table = tune(pos, vel, mass, eps2, mode, log=log, **kw)
        save(table)
    install(table, dynamic_n_i=dynamic_n_i)
    return table


# ---------------------------------------------------------------------------
# Ensemble team-planning model (nbody_ensemble_config), fitted on a
# representative launch: a synthetic ensemble drawn like the workload is run,
# the per-cluster wall times the kernel records are fitted by least squares
# (per-step latency and effective pair rate of a group on single-group
# clusters, the team cost b0 + b1 g on multi-group ones, the block-step and
# interaction laws c N^p on all), the teams are re-planned with the fitted
# model, and the fastest of the measured launches is kept, for every compiled
# shape at 2 and 3 waves per SIMD.

def _ens_mixed_inputs():
    # 256 clusters drawn like the ensemble workload (log-uniform N in
    # [256, 8192], eps = N^(-1/3)/16) but from other seeds
    import numpy as np
    from workloads.plummer import cluster_sizes, plummer
    sizes = cluster_sizes(256, 256, 8192, 4242)
    parts = [plummer(int(n), 5000 + k) for k, n in enumerate(sizes)]
    P = torch.from_numpy(np.concatenate([q[0] for q in parts], axis=1)).cuda()
    V = torch.from_numpy(np.concatenate([q[1] for q in parts], axis=1)).cuda()
    M = torch.from_numpy(np.concatenate([q[2] for q in parts])).cuda()
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps2 = (sizes.astype(np.float64) ** (-1.0 / 3.0) / 16.0) ** 2
    return sizes, P, V, M, off, eps2


def _ens_mixed_run(inp, mode, t_end, dt_max):
    """Time one launch; return (seconds, per-cluster rows (sec, g, N, steps, inter))."""
    from . import ensemble_run, ensemble_timing
    sizes, P, V, M, off, eps2 = inp
    ensemble_run(P, V, M, off, eps2, t_end, dt_max=dt_max, mode=mode)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = ensemble_run(P, V, M, off, eps2, t_end, dt_max=dt_max, mode=mode)
    e1.record()
    torch.cuda.synchronize()
    sec, grp = ensemble_timing(len(sizes))
    rows = list(zip(sec, grp, [int(n) for n in sizes], out["steps"], out["interactions"]))
    return e0.elapsed_time(e1) * 1e-3, rows


def ens_tiles(n_i, n, g, slots, tile, max_split=64):
    """j tiles of the busiest group of a g-group team in a pair pass of n_i
    slots over n particles, under the kernel's split rule: items of `slots`
    block slots by S j ranges, S minimising ceil(nb S / g) / S (the
    smallest on ties), S <= min(64, g) and S <= n / tile."""
    nb = -(-int(n_i) // slots)
    smax = max(1, min(max_split, g, n // tile))
    best, bq = 1, -(-nb // g)
    for S in range(2, smax + 1):
        q = -(-(nb * S) // g)
        if q * best < bq * S:
            best, bq = S, q
    jchunk = -(-n // best)
    return bq * (-(-jchunk // tile))


def _fit_model(rows, cfg, t_end):
    """Least-squares fit of the time model to measured clusters of one launch:
    the block-step and block-size laws on all clusters; per-step latency,
    tile latency and pair rate of one group on single-group clusters; the
    extra per-step cost b0 + b1 g of a team on the others."""
    import numpy as np
    r = np.array(rows, dtype=np.float64)
    sec, g, n, st, it = r.T
    new = dict(cfg)
    ok = st > 0
    p, logc = np.polyfit(np.log(n[ok]), np.log(st[ok] / t_end), 1)
    new["steps_exp"], new["steps_coef"] = float(p), float(np.exp(logc))
    blk = it[ok] / st[ok] / n[ok]
    p, logc = np.polyfit(np.log(n[ok]), np.log(blk), 1)
    new["block_exp"], new["block_coef"] = float(min(max(p, 0.0), 1.0)), float(np.exp(logc))
    slots, tile = 64 * int(cfg["i_per_lane"]), int(cfg["j_tile"])
    # tiles of the busiest group over the run: the initial full pass plus
    # every step at the cluster's mean block
    tiles = np.array([ens_tiles(nn, int(nn), int(gg), slots, tile)
                      + ss * ens_tiles(max(1, round(ii / max(ss, 1) / nn)), int(nn), int(gg),
                                       slots, tile)
                      for nn, gg, ss, ii in zip(n, g, st, it)], dtype=np.float64)
    inter = it + n * n  # the steps' pairs plus the initial full pass
    from scipy.optimize import nnls
    one = g == 1
    if one.sum() >= 4:
        # non-negative least squares, columns scaled to unit norm
        A = np.stack([st[one], tiles[one], inter[one]], axis=1)
        sc = np.linalg.norm(A, axis=0)
        sol, _ = nnls(A / sc, sec[one])
        sol = sol / sc
        if sol[2] > 0:
            new["step_us"] = sol[0] * 1e6
            new["tile_us"] = sol[1] * 1e6
            new["group_rate"] = 1.0 / sol[2]
    many = g > 1
    if many.sum() >= 3:
        rest = (sec[many] - st[many] * new["step_us"] * 1e-6 - tiles[many] * new["tile_us"] * 1e-6
                - inter[many] / (g[many] * new["group_rate"])) / st[many]
        A = np.stack([np.ones(many.sum()), g[many]], axis=1)
        sc = np.linalg.norm(A, axis=0)
        sol, _ = nnls(A / sc, rest)
        sol = sol / sc
        new["barrier_us"] = sol[0] * 1e6
        new["barrier_group_us"] = sol[1] * 1e6
    return {k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in new.items()}


ENS_FIELDS = ("groups_per_cu", "max_team", "step_us", "barrier_us", "barrier_group_us",
              "group_rate", "steps_coef", "steps_exp", "waves", "j_tile", "i_per_lane",
              "tile_us", "block_coef", "block_exp")

# Workgroup shapes of the ensemble kernel the library compiles:
# (waves per group, j records per LDS tile, block slots per lane).
ENS_SHAPES = ((4, 256, 2), (4, 256, 1), (2, 128, 2), (2, 256, 2), (4, 512, 2), (8, 512, 2))


def calibrate_ensemble(mode="fp32", t_end=1.0 / 16, dt_max=1.0 / 16, log=None, rounds=3,
                       shapes=ENS_SHAPES):
    """Choose the ensemble's workgroup shape and fit its team-planning model:
    for every compiled shape at 2 and 3 waves per SIMD, run a representative
    ensemble, refit the model on its per-cluster times, re-plan and run
    again; keep the fastest launch's shape and model."""
    from . import ensemble_get, ensemble_set
    saved = ensemble_get()
    inp = _ens_mixed_inputs()
    best = None
    try:
        for waves, tile, ipl in shapes:
            for wps in (2, 3):  # waves per SIMD
                gpc = max(1, wps * 4 // waves)
                cfg = dict(saved, groups_per_cu=gpc, waves=waves, j_tile=tile, i_per_lane=ipl)
                for k in range(rounds):
                    ensemble_set(**cfg)
                    secs, rows = _ens_mixed_run(inp, mode, t_end, dt_max)
                    if log:
                        log("ensemble calibration shape (%d, %d, %d) gpc=%d round %d: %.4f s"
                            % (waves, tile, ipl, gpc, k, secs))
                    if best is None or secs < best[1]:
                        best = (dict(cfg), secs)
                    cfg = _fit_model(rows, cfg, t_end)
        cfg = best[0]
        if log:
            log("ensemble model: shape (%d waves, tile %d, %d per lane), step %.1f us, tile "
                "%.2f us, barrier %.1f + %.2f g us, group rate %.3e /s, steps %.1f N^%.3f per "
                "time unit, blocks %.3f N^%.3f, %d groups per CU (%.4f s)"
                % (cfg["waves"], cfg["j_tile"], cfg["i_per_lane"], cfg["step_us"],
                   cfg["tile_us"], cfg["barrier_us"], cfg["barrier_group_us"],
                   cfg["group_rate"], cfg["steps_coef"], cfg["steps_exp"], cfg["block_coef"],
                   cfg["block_exp"], cfg["groups_per_cu"], best[1]))
        cfg["calibration_seconds"] = best[1]
        return cfg
    finally:
        ensemble_set(**saved)


def load_or_calibrate_ensemble(mode="fp32", log=None):
    from . import ensemble_set
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    p = os.path.join(CACHE_DIR, "%s_ensemble_%s.json" % (arch, mode))
    if os.path.exists(p):
        with open(p) as f:
            cfg = json.load(f)
    else:
        cfg = calibrate_ensemble(mode, log=log)
        os.makedirs(CACHE_DIR, exist_ok=True)
        with open(p, "w") as f:
            json.dump(cfg, f, indent=1)
    ensemble_set(**{k: v for k, v in cfg.items() if k in ENS_FIELDS})
    return cfg
