#!/usr/bin/env python3
"""Throughput benchmark of the direct-summation Hermite hot path on one GPU.

Workload (the configuration the headline metric is quoted on): a Plummer
sphere of N = 2^20 equal-mass particles in N-body units, softening 1/4096,
seed 1003.  One step is one Hermite block step of the device-resident
driver (nbody_blockstep: schedule -> predict all -> pair sums on the block
-> correct the block) with every particle in the block (shared steps of
2^-12, NBODY_FIXED_DT), i.e. N (N - 1) pair interactions per step.  Inputs
are resident in HBM before the timed region.

Printed: one JSON line with interactions/s, the pair kernel's roofline
(algorithmic flops at 60 per interaction -- the paper's per-interaction
operation count -- over its HIP-event-timed duration, against the MI355X
float32 vector peak), and the FP64 oracle timed on the host cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 60          # the paper's per-interaction operation count
FP32_PEAK_TFLOPS = 157.3            # MI355X float32 vector peak
HBM_PEAK_GBS = 8000.0


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("force.hip", "pairs.hpp", "records.hpp"):
        with open(os.path.join(ROOT, "paper_cs_0702135_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


MIN_FLOPS_PER_INTERACTION = 42     # minimal algorithmic count (28 instructions, FMA = 2)


def measured_valu_mix():
    """Executed float32 flops per interaction of the pair kernel from the
    committed instruction-mix counters (profiles/force_kernel_valu_mix.json),
    or None if the kernel sources have changed since they were taken."""
    p = os.path.join(ROOT, "profiles", "force_kernel_valu_mix.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    return t if t.get("source_sha256") == kernel_source_digest() else None


def measured_traffic():
    """HBM bytes per pair-kernel launch from the committed counter runs
    (profiles/force_kernel_traffic.json), or None if the kernel sources have
    changed since those counters were taken."""
    p = os.path.join(ROOT, "profiles", "force_kernel_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    return t["bytes_per_launch"] if t.get("source_sha256") == kernel_source_digest() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTER_RUNS = {
    # subdirectory of a profiling run -> rocprofv3 counters of that pass
    "pmc_fetch": "FETCH_SIZE",
    "pmc_write": "WRITE_SIZE",
    "pmc_copy_fetch": "FETCH_SIZE",
    "pmc_copy_write": "WRITE_SIZE",
    "pmc_f32": "SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 "
               "SQ_INSTS_VALU_TRANS_F32",
    "pmc_f64": "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 "
               "SQ_INSTS_VALU_CVT",
    "pmc_flops": "SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES "
                 "SQ_LDS_BANK_CONFLICT SQ_INSTS_LDS GRBM_GUI_ACTIVE",
}


def summarize_counters(run_dir):
    """Write profiles/force_kernel_traffic.json and force_kernel_valu_mix.json
    from the rocprofv3 counter passes under run_dir (one subdirectory per
    pass, named as in COUNTER_RUNS; the pair-kernel passes profile
    `bench.py --steps 1 --warmup 0 --no-cpu --no-aux`, the copy passes
    `bench.py --calib-copy`).  The values are those of the last pair-kernel
    dispatch of each pass (the timed block-step launch); FETCH_SIZE and
    WRITE_SIZE are in KiB and are scaled by what they read for the 1 GiB copy."""
    import csv

    def read(sub, kernel_prefix):
        out = {}
        with open(os.path.join(run_dir, sub, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Kernel_Name"].startswith(kernel_prefix):
                    # later dispatches overwrite earlier ones
                    out.setdefault(r["Counter_Name"], {})[int(r["Dispatch_Id"])] = \
                        float(r["Counter_Value"])
        return {k: [v[d] for d in sorted(v)] for k, v in out.items()}

    def cmd(sub, prog):
        return ("rocprofv3 --pmc %s --output-format csv -d %s -o run -- python3 bench.py %s"
                % (COUNTER_RUNS[sub], os.path.join(run_dir, sub), prog))

    pair = "void nb::force_kernel<0, 2, 2, 0>"
    prog = "--steps 1 --warmup 0 --no-cpu --no-aux"
    copy_bytes = float(1 << 30)
    fetch = read("pmc_fetch", pair)["FETCH_SIZE"]
    write = read("pmc_write", pair)["WRITE_SIZE"]
    cf = read("pmc_copy_fetch", "__amd_rocclr_copyBuffer")["FETCH_SIZE"]
    cw = read("pmc_copy_write", "__amd_rocclr_copyBuffer")["WRITE_SIZE"]
    fetch_factor = copy_bytes / (max(cf) * 1024.0)
    write_factor = copy_bytes / (max(cw) * 1024.0)
    traffic = {
        "kernel": pair + "(nb::KArgs)",
        "workload": "plummer N=2^20 shared block step (bench.py), block-step launch (the timed kind)",
        "fetch_kib": fetch, "write_kib": write,
        "fetch_factor": fetch_factor, "write_factor": write_factor,
        "bytes_per_launch": (fetch[-1] * fetch_factor + write[-1] * write_factor) * 1024.0,
        "source_sha256": kernel_source_digest(),
        "commands": [cmd("pmc_fetch", prog), cmd("pmc_write", prog),
                     "calibration: " + cmd("pmc_copy_fetch", "--calib-copy") + " ; "
                     + cmd("pmc_copy_write", "--calib-copy")
                     + " (1 GiB device copy: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB)"
                     % (max(cf), max(cw))],
    }
    counters = {}
    for sub in ("pmc_f32", "pmc_f64", "pmc_flops"):
        for k, v in read(sub, pair).items():
            counters[k] = v[-1]
    inter = float(1 << 20) * ((1 << 20) - 1)
    ex = 64.0 * counters["SQ_INSTS_VALU_FLOPS_FP32"] / inter
    mix = {
        "kernel": pair + "(nb::KArgs)",
        "workload": "plummer N=2^20 shared block step (bench.py), block-step launch",
        "counters_per_launch": counters,
        "executed_f32_flops_per_interaction": round(ex, 3),
        "valu_instructions_per_interaction": round(64.0 * counters["SQ_INSTS_VALU"] / inter, 3),
        "source_sha256": kernel_source_digest(),
        "commands": [cmd(sub, prog) for sub in ("pmc_f32", "pmc_f64", "pmc_flops")],
    }
    for name, obj in (("force_kernel_traffic.json", traffic),
                      ("force_kernel_valu_mix.json", mix)):
        with open(os.path.join(ROOT, "profiles", name), "w") as f:
            json.dump(obj, f, indent=1)
            f.write("\n")
    print(json.dumps({"bytes_per_launch": traffic["bytes_per_launch"],
                      "executed_f32_flops_per_interaction": mix["executed_f32_flops_per_interaction"],
                      "valu_instructions_per_interaction":
                          mix["valu_instructions_per_interaction"]}))


def fit_power_law(x, y):
    """Least-squares fit of y = c x^p in log-log space; returns (c, p)."""
    import numpy as np
    p, lc = np.polyfit(np.log(np.asarray(x, dtype=float)), np.log(np.asarray(y, dtype=float)), 1)
    return float(np.exp(lc)), float(p)


def ensemble_only(args):
    """The batched-ensemble workload alone: 256 Plummer clusters (N
    log-uniform in [256, 8192], eps = N^(-1/3)/16, seed 1004) integrated to
    t = 1/16 in one persistent launch; a warm-up launch, then `steps` timed
    launches.  Prints one JSON line with the block interactions per second
    and the launch's float32 roofline (60 flops per interaction)."""
    import numpy as np
    import torch

    import paper_cs_0702135_amd as nb
    from paper_cs_0702135_amd import autotune
    from workloads.plummer import CONFIGS, ensemble_members, plummer

    ce = CONFIGS["ensemble256"]
    sizes, eps_c, seeds = ensemble_members(ce)
    parts = [plummer(int(nc), int(sd)) for nc, sd in zip(sizes, seeds)]
    EP = torch.from_numpy(np.concatenate([q[0] for q in parts], axis=1)).cuda()
    EV = torch.from_numpy(np.concatenate([q[1] for q in parts], axis=1)).cuda()
    EM = torch.from_numpy(np.concatenate([q[2] for q in parts])).cuda()
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cfg = autotune.load_or_calibrate_ensemble(args.mode, log=log)
    for _ in range(max(1, args.warmup)):
        nb.ensemble_run(EP, EV, EM, off, eps_c ** 2, ce.t_end, dt_max=ce.dt_max, mode=args.mode)
    torch.cuda.synchronize()
    inter, secs = 0, 0.0
    for _ in range(args.steps):
        ta = time.perf_counter()
        res = nb.ensemble_run(EP, EV, EM, off, eps_c ** 2, ce.t_end, dt_max=ce.dt_max,
                              mode=args.mode)
        secs += time.perf_counter() - ta
        inter += sum(res["interactions"])
    achieved = FLOPS_PER_INTERACTION * inter / secs / 1e12
    out = {
        "metric": "block pair interactions/s of the batched ensemble (one persistent launch)",
        "value": inter / secs,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256 Plummer clusters, N log-uniform in [256, 8192], "
                               "eps = N^(-1/3)/16, eta = 0.02, dt_max = 1/16, t: 0 -> 1/16",
                   "accumulation": args.mode, "grid_teams": list(nb.ensemble_info()),
                   "model": cfg},
        "roofline": {"bound": "alu", "kernel": "ensemble_kernel", "achieved": round(achieved, 2),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "flops_per_interaction": FLOPS_PER_INTERACTION},
    }
    print(json.dumps(out), flush=True)


def section5_fit(rows, table4):
    """The Section 5 time model t_step = t_host + t_force + t_comm refitted
    with device terms: the state stays in HBM, so t_comm = 0, and what the
    paper's host did (prediction and correction) runs on the device:
        t_step  = t0 + a N + I / R           (I = n_block N interactions)
        t_pairs = f0 + I / R_k               (pair + reduction kernels only)
    by least squares on the relative error over the protocol's N: t_step
    from the timed window (t: 1/4 -> 1/2, no event timing), t_pairs from the
    pair kernels' HIP events in the first quarter.  The paper's measured
    parameters (its Table 4, other hardware) are returned beside for
    context."""
    import numpy as np
    n = np.array([r["n"] for r in rows], dtype=float)
    y = np.array([r["ms_per_block_step"] for r in rows]) * 1e-3
    inter = np.array([r["mean_block"] for r in rows]) * n
    yk = np.array([r["pair_kernel_us_per_step_0_to_quarter"] for r in rows]) * 1e-6
    inter_k = np.array([r["interactions_per_step_0_to_quarter"] for r in rows])
    A = np.stack([np.ones_like(n), n, inter], axis=1) / y[:, None]
    c, *_ = np.linalg.lstsq(A, np.ones_like(y), rcond=None)
    model = c[0] + c[1] * n + c[2] * inter
    Ak = np.stack([np.ones_like(n), inter_k], axis=1) / yk[:, None]
    ck, *_ = np.linalg.lstsq(Ak, np.ones_like(yk), rcond=None)
    mk = ck[0] + ck[1] * inter_k
    gtx = table4["eta_fe_t_force_s"]["geforce8800gtx"] / table4["n_pipe"]["geforce8800gtx"]
    return {
        "t0_us": float(c[0] * 1e6),
        "a_ns_per_particle": float(c[1] * 1e9),
        "pair_rate_interactions_per_s": float(1.0 / c[2]) if c[2] > 0 else None,
        "rel_residuals": [float(v) for v in (model - y) / y],
        "pair_kernels_f0_us": float(ck[0] * 1e6),
        "pair_kernels_rate_interactions_per_s": float(1.0 / ck[1]) if ck[1] > 0 else None,
        "pair_kernels_rel_residuals": [float(v) for v in (mk - yk) / yk],
        "t_comm": 0.0,
        "paper_table4_context": {
            "t_host_per_particle_s": table4["t_host_per_particle_s"],
            "geforce8800gtx_s_per_interaction": gtx,
            "geforce8800gtx_send_receive_s_per_particle":
                table4["eta_send_t_send_s"]["geforce8800gtx"]
                + table4["eta_rec_t_rec_s"]["geforce8800gtx"],
        },
    }


def small_block_sweep(P, V, M, eps2, cfg, reps=20):
    """Pair sums of small active blocks (seeded subsets of n_i = 1, 16, 64)
    against all N j, both modes, in the installed launch shapes: the call
    time (packing the j records, the pair kernels and the split reduction)
    and the pair kernels' own HIP-event time."""
    import torch

    import paper_cs_0702135_amd as nb
    from workloads.plummer import random_active_set
    n = M.shape[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    small = {}
    for n_i in cfg.extra["n_i_small"]:
        idx = torch.from_numpy(random_active_set(n, n_i, cfg.seed + n_i)).cuda()
        for md in ("fp32", "ds"):
            nb.force(P, V, M, eps2, idx, md)
            torch.cuda.synchronize()
            nb.profile(1)
            e0.record()
            for _ in range(reps):
                nb.force(P, V, M, eps2, idx, md)
            e1.record()
            torch.cuda.synchronize()
            f_ms, r_ms, nl = nb.profile(0)
            small["%s_n_i_%d" % (md, n_i)] = {
                "call_us": e0.elapsed_time(e1) / reps * 1e3,
                "pair_kernel_us": f_ms / max(1, nl) * 1e3,
                "reduce_us": r_ms / max(1, nl) * 1e3,
                "shape": nb.tune_get(n_i).asdict()}
            log("small blocks: n_i=%d %s: call %.1f us, pair kernel %.1f us"
                % (n_i, md, small["%s_n_i_%d" % (md, n_i)]["call_us"],
                   small["%s_n_i_%d" % (md, n_i)]["pair_kernel_us"]))
    return small


def valu_issue_bound(mix, kernel_ms):
    """The pair kernel's VALU issue bound: the wave-instructions of each kind
    its loop executes (the committed counter run of this launch) divided by
    the issue rate of that kind measured now on this device
    (nbody_valu_rates), summed, against this run's kernel time.  The
    `rsq_coissued` figures leave the reciprocal square roots out of the sum,
    as if the transcendental unit issued them beside the other instructions."""
    import paper_cs_0702135_amd as nb
    c = mix["counters_per_launch"]
    count = {"v_fmac_f32": c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"],
             "v_mul_f32": c["SQ_INSTS_VALU_MUL_F32"],
             "v_add_f64": c["SQ_INSTS_VALU_ADD_F64"],
             "v_cvt_f32_f64": c["SQ_INSTS_VALU_CVT"],
             "v_rsq_f32": c["SQ_INSTS_VALU_TRANS_F32"]}
    rate = nb.valu_rates(8)
    t_all = sum(count[k] / rate[k] for k in count)
    t_co = t_all - count["v_rsq_f32"] / rate["v_rsq_f32"]
    return {
        "wave_instr_per_launch": {k: float("%.4g" % count[k]) for k in count},
        "wave_instr_per_s": {k: float("%.4g" % rate[k]) for k in count},
        "bound_ms": round(t_all * 1e3, 2),
        "bound_ms_rsq_coissued": round(t_co * 1e3, 2),
        "frac": round(t_all * 1e3 / kernel_ms, 4),
        "frac_rsq_coissued": round(t_co * 1e3 / kernel_ms, 4),
    }


def plummer64k_run(mode):
    """Plummer N = 65536, eps = 1/1024, built-in launch shapes: the full-N
    force-only throughput, then the block-step run to t = 1/8 (wall time,
    steps, energy drift)."""
    import torch

    import paper_cs_0702135_amd as nb
    from workloads.plummer import CONFIGS, plummer
    c2 = CONFIGS["plummer64k"]
    p2, v2, m2 = (torch.from_numpy(a).cuda() for a in plummer(c2.n, c2.seed))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    nb.force(p2, v2, m2, c2.eps2, None, mode)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        nb.force(p2, v2, m2, c2.eps2, None, mode)
    e1.record()
    torch.cuda.synchronize()
    out["plummer64k_force_only_interactions_per_s"] = 5 * c2.n * (c2.n - 1.0) / (
        e0.elapsed_time(e1) * 1e-3)
    s2 = nb.System(p2, v2, m2, c2.eps2, eta=c2.eta, dt_max=c2.dt_max, mode=mode)
    e_0 = s2.energy()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    steps2 = s2.run(c2.t_end)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    e_1 = s2.energy()
    out["plummer64k_run_seconds"] = tb - ta
    out["plummer64k_block_steps"] = steps2
    out["plummer64k_run_interactions_per_s"] = s2.interactions / (tb - ta)
    out["plummer64k_energy_drift_per_time_unit"] = abs((e_1 - e_0) / e_0) / c2.t_end
    log("plummer64k: %d block steps in %.4f s" % (steps2, tb - ta))
    return out


def small_blocks_only(args):
    """Only the small-block sweep at N = 2^20 (the tuned table installed as
    the default run installs it); one JSON line."""
    import torch

    from paper_cs_0702135_amd import autotune
    from workloads.plummer import CONFIGS, plummer
    cfg = CONFIGS["plummer1m"]
    pos, vel, m = plummer(cfg.n, cfg.seed)
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, m))
    autotune.load_or_tune(P, V, M, cfg.eps2, args.mode, log=log, dynamic_n_i=cfg.n)
    out = {"metric": "pair sums of small active blocks at N = 2^20 (us per call)",
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "plummer N=2^20 eps=1/4096 seed=1003, seeded active "
                                  "subsets n_i = 1, 16, 64"},
           "rows": small_block_sweep(P, V, M, cfg.eps2, cfg)}
    print(json.dumps(out), flush=True)


def host_cpu():
    """The host the oracle ran on: CPU model, logical CPUs, CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def paper_table(args):
    """The Section 4 results-table protocol on one GPU: for each N, one
    seeded Plummer realisation, eps = 1/256, eta = 0.02, dt_max = 1/8,
    block steps from t = 0 to 1/4 (untimed), then timed from 1/4 to 1/2.
    Prints one JSON line with a row per N (seconds, block steps, mean block
    size, interactions/s, energy drift) next to the paper's printed seconds
    for its GeForce 8800GTX and GRAPE-6Af (other hardware: context only),
    and power-law fits of the block statistics next to the paper's."""
    import numpy as np
    import torch

    import paper_cs_0702135_amd as nb
    from workloads.plummer import CONFIGS, plummer, table_protocol_seed

    cfg = CONFIGS["table_protocol"]
    t_from = cfg.extra["timed_from"]
    with open(os.path.join(ROOT, "tests", "golden", "paper_fits.json")) as f:
        gold = json.load(f)
    paper = gold["results_table_seconds"]
    nb.tune_clear()
    rows = []
    for n in cfg.extra["n_list"]:
        if n > args.table_max_n:
            break
        pos, vel, m = plummer(n, table_protocol_seed(n))
        P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, m))
        s = nb.System(P, V, M, cfg.eps2, eta=cfg.eta, eta_s=cfg.eta_s, dt_max=cfg.dt_max,
                      mode=args.mode)
        e0 = s.energy()
        # the untimed first part carries the pair-kernel event timing (and
        # gives the per-step terms of the Section 5 model fit)
        nb.profile(1)
        torch.cuda.synchronize()
        t00 = time.perf_counter()
        steps0 = s.run(t_from)
        torch.cuda.synchronize()
        t01 = time.perf_counter()
        force_ms, reduce_ms, launches = nb.profile(0)
        inter0 = s.interactions
        ta = time.perf_counter()
        steps1 = s.run(cfg.t_end)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        inter1 = s.interactions - inter0
        e1 = s.energy()
        k = paper["n"].index(n)
        row = {
            "n": n,
            "seconds": tb - ta,
            "block_steps": steps1,
            "block_steps_0_to_quarter": steps0,
            "mean_block": inter1 / max(1, steps1) / n,
            "interactions_per_s": inter1 / (tb - ta),
            "ms_per_block_step": (tb - ta) / max(1, steps1) * 1e3,
            "energy_drift_per_time_unit": abs((e1 - e0) / e0) / cfg.t_end,
            "pair_kernel_tflops_0_to_quarter": FLOPS_PER_INTERACTION * inter0 / (force_ms * 1e-3) / 1e12,
            "pair_kernel_frac_0_to_quarter": FLOPS_PER_INTERACTION * inter0 / (force_ms * 1e-3) / 1e12
            / FP32_PEAK_TFLOPS,
            "pair_kernel_launches_0_to_quarter": launches,
            "step_us_0_to_quarter": (t01 - t00) / max(1, steps0) * 1e6,
            "pair_kernel_us_per_step_0_to_quarter": (force_ms + reduce_ms) / max(1, steps0) * 1e3,
            "interactions_per_step_0_to_quarter": inter0 / max(1, steps0),
            "paper_8800gtx_seconds": paper["geforce8800gtx"][k],
            "paper_grape6af_seconds": paper["grape6af"][k],
        }
        rows.append(row)
        log("table: N=%d %.4f s, %d block steps (mean block %.1f), drift/unit %.2e"
            % (n, row["seconds"], steps1, row["mean_block"], row["energy_drift_per_time_unit"]))
        del s, P, V, M
    ns = [r["n"] for r in rows]
    fits = {}
    if len(rows) >= 2:
        window = cfg.t_end - t_from
        fits["mean_block"] = fit_power_law(ns, [r["mean_block"] for r in rows])
        fits["block_steps_per_time_unit"] = fit_power_law(
            ns, [r["block_steps"] / window for r in rows])
        fits["paper_mean_block"] = (gold["n_block"]["coef"], gold["n_block"]["exp"])
        fits["paper_block_steps_per_time_unit"] = (gold["n_steps_per_time_unit"]["coef"],
                                                   gold["n_steps_per_time_unit"]["exp"])
        fits["section5_model"] = section5_fit(rows, gold["model_parameters_table4"])
    out = {
        "metric": "wall-clock seconds of t = 1/4 -> 1/2 (Section 4 results-table protocol)",
        "unit": "s",
        "higher_is_better": False,
        "n_gpus": 1,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer N=256..524288 (one seeded realisation per N), "
                               "eps=1/256, eta=0.02, dt_max=1/8, block steps t: 0 -> 1/2, "
                               "timed over 1/4 -> 1/2", "accumulation": args.mode},
        "rows": rows,
        "fits": fits,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=("fp32", "ds"), default="fp32")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-aux", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the per-cluster driver ablation of the ensemble (many launches)")
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--paper-table", action="store_true",
                    help="run the Section 4 results-table protocol instead of the default step")
    ap.add_argument("--ensemble", action="store_true",
                    help="run only the batched-ensemble workload")
    ap.add_argument("--small-blocks", action="store_true",
                    help="run only the small-block pair-sum sweep at N = 2^20")
    ap.add_argument("--plummer64k", action="store_true",
                    help="run only the Plummer N = 65536 block-step run to t = 1/8")
    ap.add_argument("--table-max-n", type=int, default=1 << 19,
                    help="largest N of the results-table protocol")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run one plain device copy of 1 GiB (HBM-counter calibration)")
    ap.add_argument("--summarize-counters", metavar="RUN_DIR",
                    help="write the pair kernel's traffic and instruction-mix summaries under "
                         "profiles/ from the counter passes in RUN_DIR (no GPU)")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return

    if args.calib_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": src.numel() * 8}), flush=True)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path "
              "(the j-parallel sharding is a design note only); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.paper_table:
        paper_table(args)
        return
    if args.ensemble:
        ensemble_only(args)
        return
    if args.small_blocks:
        small_blocks_only(args)
        return
    if args.plummer64k:
        nb_cfg = {"metric": "Plummer N = 65536 block-step run to t = 1/8",
                  "n_gpus": 1, "data": "synthetic",
                  "config": {"workload": "plummer N=65536 eps=1/1024 seed=1002 eta=0.02 "
                                         "dt_max=1/8, built-in launch shapes",
                             "accumulation": args.mode}}
        nb_cfg.update(plummer64k_run(args.mode))
        print(json.dumps(nb_cfg), flush=True)
        return

    import numpy as np
    import torch

    import paper_cs_0702135_amd as nb
    from paper_cs_0702135_amd import autotune
    from workloads.plummer import CONFIGS, plummer

    cfg = CONFIGS["plummer1m"]
    n = args.n
    eps2 = cfg.eps2
    log("bench: building Plummer N=%d" % n)
    pos, vel, m = plummer(n, cfg.seed)
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, m))

    if args.retune:
        table = autotune.tune(P, V, M, eps2, args.mode, log=log)
        autotune.save(table)
    table = autotune.load_or_tune(P, V, M, eps2, args.mode, log=log, dynamic_n_i=n)
    shape = nb.tune_get(-1)
    log("bench: block-step pair-kernel shape %r" % (shape,))

    h = 2.0 ** -12
    sysg = nb.System(P, V, M, eps2, dt_max=h, mode=args.mode, fixed_dt=True)
    for _ in range(args.warmup):
        assert sysg.step(1) == 1
    torch.cuda.synchronize()
    # HIP events around every pair-kernel launch, read back after each step
    # (each step synchronises anyway): average and median per launch
    per_launch, force_ms, reduce_ms, launches = [], 0.0, 0.0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        nb.profile(1)
        assert sysg.step(1) == 1
        f_ms, r_ms, nl = nb.profile(0)
        force_ms, reduce_ms, launches = force_ms + f_ms, reduce_ms + r_ms, launches + nl
        per_launch.append(f_ms / max(1, nl))
        log("bench: step %d done (pair kernel %.1f ms)" % (k + 1, per_launch[-1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    inter_step = float(n) * (n - 1)
    value = args.steps * inter_step / wall
    ms_step = wall / args.steps * 1e3

    k_ms = force_ms / max(1, launches)
    k_med = float(np.median(per_launch))
    achieved = FLOPS_PER_INTERACTION * inter_step / (k_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": "force_kernel",
        "achieved": round(achieved, 2),
        "peak": FP32_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
        "traffic": measured_traffic(),
        "kernel_ms": round(k_ms, 3),
        "kernel_ms_median": round(k_med, 3),
        "flops_per_interaction": FLOPS_PER_INTERACTION,
        "reduce_ms": round(reduce_ms / max(1, launches), 3),
        # the same launch at the minimal algorithmic count, and at the float32
        # flops the counters saw it execute (FMA = 2, rsq = 1)
        "frac_at_42_flops": round(MIN_FLOPS_PER_INTERACTION * inter_step / (k_ms * 1e-3) / 1e12
                                  / FP32_PEAK_TFLOPS, 4),
    }
    mix = measured_valu_mix()
    if mix is not None:
        ex = mix["executed_f32_flops_per_interaction"]
        roofline["executed_f32_flops_per_interaction"] = ex
        roofline["frac_executed"] = round(ex * inter_step / (k_ms * 1e-3) / 1e12
                                          / FP32_PEAK_TFLOPS, 4)
        roofline["valu_issue"] = valu_issue_bound(mix, k_ms)

    out = {
        "metric": "pairwise acc+jerk interactions/s (Hermite block step, all N active)",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plummer N=2^20 eps=1/4096 seed=1003, shared Hermite block step "
                        "h=2^-12 (all N active), pair arithmetic f32 on f64-formed "
                        "relative coordinates, f64 integrator",
            "n": n, "eps": 1.0 / 4096, "accumulation": args.mode,
            "shape": shape.asdict(),
        },
        "roofline": roofline,
    }

    if not args.no_aux:
        aux = {}
        # the other accumulation mode on the same state, pair kernel only
        other = "ds" if args.mode == "fp32" else "fp32"
        nb.force(P, V, M, eps2, None, other)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.force(P, V, M, eps2, None, other)
        e1.record()
        torch.cuda.synchronize()
        aux["force_only_%s_interactions_per_s" % other] = inter_step / (e0.elapsed_time(e1) * 1e-3)
        # cost of the compensated mode (float64 pair terms): its n_i = N call
        # over the float32 pair kernel's launch time
        aux["%s_call_over_%s_pair_kernel" % (other, args.mode)] = e0.elapsed_time(e1) / k_ms
        # force-only sweep at N = 2^20 over active-block sizes, both modes;
        # small blocks also with the pair kernels' own event time (the call
        # time includes packing the 2^20 j records and the launches)
        from workloads.plummer import random_active_set
        sweep = {}
        aux["plummer1m_small_blocks"] = small_block_sweep(P, V, M, eps2, cfg)
        for n_i in cfg.extra["n_i"]:
            idx = None if n_i == n else torch.from_numpy(
                random_active_set(n, n_i, cfg.seed + n_i)).cuda()
            reps = max(1, int(3e10 // (n_i * (n - 1))))
            for md in ("fp32", "ds"):
                nb.force(P, V, M, eps2, idx, md)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    nb.force(P, V, M, eps2, idx, md)
                e1.record()
                torch.cuda.synchronize()
                sweep["%s_n_i_%d" % (md, n_i)] = reps * n_i * (n - 1.0) / (
                    e0.elapsed_time(e1) * 1e-3)
        aux["plummer1m_force_sweep_interactions_per_s"] = sweep
        # energy drift of the block-step integrator, Plummer N=1024 to t=1/4
        # (built-in shapes: the tuned table above is for N = 2^20)
        nb.tune_clear()
        c1 = CONFIGS["plummer1k"]
        p1, v1, m1 = plummer(c1.n, c1.seed)
        s1 = nb.System(*(torch.from_numpy(a).cuda() for a in (p1, v1, m1)), c1.eps2,
                       eta=c1.eta, dt_max=c1.dt_max, mode=args.mode)
        e_0 = s1.energy()
        ta = time.perf_counter()
        steps1 = s1.run(c1.t_end)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        e_1 = s1.energy()
        aux["plummer1k_energy_drift_per_time_unit"] = abs((e_1 - e_0) / e_0) / c1.t_end
        aux["plummer1k_block_steps"] = steps1
        aux["plummer1k_ms_per_block_step"] = (tb - ta) / max(1, steps1) * 1e3

        # cost of the smallest-first float32 sums (Section 6) against the
        # float32 mode on the same full-N call, N = 1024 and N = 8192
        sorted_cost = {}
        for n_s in (1024, 8192):
            ps, vs, ms = (torch.from_numpy(a).cuda() for a in plummer(n_s, c1.seed))
            row = {}
            for key, fn in (("sorted_ms", lambda: nb.force_sorted(ps, vs, ms, c1.eps2)),
                            ("fp32_ms", lambda: nb.force(ps, vs, ms, c1.eps2, None, "fp32"))):
                fn()
                torch.cuda.synchronize()
                e0.record()
                for _ in range(3):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                row[key] = e0.elapsed_time(e1) / 3
            row["ratio"] = row["sorted_ms"] / row["fp32_ms"]
            sorted_cost["n%d" % n_s] = row
        aux["smallest_first_sorted_cost"] = sorted_cost

        aux.update(plummer64k_run(args.mode))

        # batched ensemble: 256 clusters, N log-uniform in [256, 8192], to t = 1/16,
        # one persistent launch (inputs resident before timing; second run timed)
        from workloads.plummer import ensemble_members
        ce = CONFIGS["ensemble256"]
        sizes, eps_c, seeds = ensemble_members(ce)
        parts = [plummer(int(nc), int(sd)) for nc, sd in zip(sizes, seeds)]
        EP = torch.from_numpy(np.concatenate([q[0] for q in parts], axis=1)).cuda()
        EV = torch.from_numpy(np.concatenate([q[1] for q in parts], axis=1)).cuda()
        EM = torch.from_numpy(np.concatenate([q[2] for q in parts])).cuda()
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        ens_cfg = autotune.load_or_calibrate_ensemble(args.mode, log=log)
        aux["ensemble_model"] = ens_cfg
        nb.ensemble_run(EP, EV, EM, off, eps_c ** 2, ce.t_end, dt_max=ce.dt_max, mode=args.mode)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        res = nb.ensemble_run(EP, EV, EM, off, eps_c ** 2, ce.t_end, dt_max=ce.dt_max,
                              mode=args.mode)
        tb = time.perf_counter()
        grid, teams = nb.ensemble_info()
        aux["ensemble256_seconds"] = tb - ta
        aux["ensemble256_interactions_per_s"] = float(sum(res["interactions"])) / (tb - ta)
        aux["ensemble256_block_steps"] = int(sum(res["steps"]))
        aux["ensemble256_grid_teams"] = [grid, teams]
        # ablation: the same clusters integrated one after the other, each
        # with the single-system block-step driver (several launches per step)
        if not args.no_ablation:
            ta = time.perf_counter()
            abl_inter = 0
            for c in range(len(sizes)):
                lo_, hi_ = int(off[c]), int(off[c + 1])
                sc = nb.System(EP[:, lo_:hi_].contiguous(), EV[:, lo_:hi_].contiguous(),
                               EM[lo_:hi_].contiguous(), float(eps_c[c]) ** 2,
                               eta=ce.eta, dt_max=ce.dt_max, mode=args.mode)
                sc.run(ce.t_end)
                abl_inter += sc.interactions
            torch.cuda.synchronize()
            tb = time.perf_counter()
            aux["ensemble256_per_cluster_driver_seconds"] = tb - ta
            aux["ensemble256_per_cluster_driver_interactions_per_s"] = abl_inter / (tb - ta)

        # differentiable run: N = 16384, eps = 1/512, 64 shared steps of 1/512,
        # checkpoints every 8 steps; forward + backward through the HIP adjoint
        from paper_cs_0702135_amd.autograd import shared_run
        cg = CONFIGS["grad16k"]
        gp, gv, gm = plummer(cg.n, cg.seed)
        GP, GV, GM = (torch.from_numpy(q).cuda() for q in (gp, gv, gm))
        with torch.no_grad():
            xT = shared_run(GP, GV, GM, cg.eps2, cg.extra["dt"], cg.extra["steps"])[0]
        tgt = xT + cg.extra["target_sigma"] * torch.randn(xT.shape, dtype=xT.dtype,
                                                          device=xT.device,
                                                          generator=torch.Generator("cuda").manual_seed(2005))
        # one untimed forward + backward (the first backward allocates the
        # library's workspace), then the median of three timed ones
        fb = []
        for rep in range(4):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            P0 = GP.clone().requires_grad_(True)
            xf = shared_run(P0, GV, GM, cg.eps2, cg.extra["dt"], cg.extra["steps"],
                            checkpoint_every=cg.extra["ckpt"])[0]
            loss = ((xf - tgt) ** 2).sum() / cg.n
            loss.backward()
            torch.cuda.synchronize()
            if rep > 0:
                fb.append(time.perf_counter() - ta)
        aux["grad16k_forward_backward_seconds"] = float(np.median(fb))
        # adjoint pair kernel alone on the N=16384 state (both roles of every pair)
        gb = torch.ones_like(GP)
        nb.force_adjoint(GP, GV, GM, cg.eps2, gb, gb)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            nb.force_adjoint(GP, GV, GM, cg.eps2, gb, gb)
        e1.record()
        torch.cuda.synchronize()
        aux["grad16k_adjoint_pairs_per_s"] = 5 * cg.n * (cg.n - 1.0) / (
            e0.elapsed_time(e1) * 1e-3)
        del GP, GV, GM, P0, xf, tgt, xT

        # beyond 2^20: N = 9e6 pair sums of seeded active subsets (both
        # accumulations); N = 2^22 initialisation and a few block steps
        c9 = CONFIGS["plummer9m"]
        p9 = [torch.from_numpy(a).cuda() for a in plummer(c9.n, c9.seed)]
        big = {}
        for n_i in c9.extra["n_i"]:
            idx = torch.from_numpy(random_active_set(c9.n, n_i, c9.seed + n_i)).cuda()
            for md in ("fp32", "ds"):
                nb.force(*p9, c9.eps2, idx, md)
                torch.cuda.synchronize()
                e0.record()
                nb.force(*p9, c9.eps2, idx, md)
                e1.record()
                torch.cuda.synchronize()
                big["%s_n_i_%d" % (md, n_i)] = n_i * (c9.n - 1.0) / (e0.elapsed_time(e1) * 1e-3)
        aux["plummer9m_force_interactions_per_s"] = big
        del p9
        c4 = CONFIGS["plummer4m"]
        p4 = [torch.from_numpy(a).cuda() for a in plummer(c4.n, c4.seed)]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        s4 = nb.System(*p4, c4.eps2, eta=c4.eta, dt_max=c4.dt_max, mode=args.mode)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        steps4 = s4.step(8)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        aux["plummer4m_init_seconds"] = tb - ta
        aux["plummer4m_block_steps"] = steps4
        aux["plummer4m_ms_per_block_step"] = (tc - tb) / max(1, steps4) * 1e3
        aux["plummer4m_mean_block"] = s4.interactions / max(1, steps4) / c4.n
        aux["plummer4m_block_step_interactions_per_s"] = s4.interactions / (tc - tb)
        del s4, p4
        out["aux"] = aux

    if not args.no_cpu:
        import oracle
        cores = oracle.num_threads()
        rng = np.random.default_rng(cfg.seed + 7)
        # calibrate on a small sample, then size the sample to ~cpu_seconds
        probe = np.sort(rng.choice(n, 256, replace=False)).astype(np.int32)
        ta = time.perf_counter()
        oracle.force(pos, vel, m, eps2, active=probe)
        rate0 = 256 * (n - 1) / (time.perf_counter() - ta)
        n_s = int(max(256, min(n, args.cpu_seconds * rate0 / (n - 1))))
        sample = np.sort(rng.choice(n, n_s, replace=False)).astype(np.int32)
        log("bench: oracle sample of %d i-particles (%d threads)" % (n_s, cores))
        ta = time.perf_counter()
        oracle.force(pos, vel, m, eps2, active=sample)
        dt_cpu = time.perf_counter() - ta
        out["cpu_baseline"] = {
            "value": n_s * (n - 1) / dt_cpu,
            "unit": "interactions/s",
            "cores": cores,
            "kind": "oracle",
            "sample": "FP64 oracle pair sums for %d seeded i-particles against all %d j "
                      "(%.2e interactions, %.1f s)" % (n_s, n, n_s * (n - 1.0), dt_cpu),
        }
        # the same oracle on one host core, over a proportionally smaller
        # sample (about a third of the multi-core sample's wall time)
        n_1 = int(max(64, n_s / max(1, cores) / 3))
        one = sample[:n_1]
        oracle.set_num_threads(1)
        try:
            ta = time.perf_counter()
            oracle.force(pos, vel, m, eps2, active=one)
            dt_1 = time.perf_counter() - ta
        finally:
            oracle.set_num_threads(cores)
        out["cpu_host"] = host_cpu()
        out["cpu_baseline_one_core"] = {
            "value": n_1 * (n - 1) / dt_1,
            "unit": "interactions/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "the first %d of the same i-particles (%.1f s)" % (n_1, dt_1),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
