"""Plummer N = 65536 block-step run on the GPU (eps = 1/1024, eta = 0.02,
dt_max = 1/8, t: 0 -> 1/8) with the oracle re-evaluating sampled blocks.

Every 50th block step the oracle takes the GPU's own state before the step,
selects the block (t_i + dt_i minimal, Section 2), predicts every particle
to the block time and evaluates the pair sums of up to 4096 seeded block
members in float64 (Eq. 1 with Plummer softening).  After the GPU's step
the new acceleration and jerk of those members (the corrector stores the
pair sums at the predicted state) are compared with the oracle's.  Gates on
the per-particle relative errors over all sampled members (the block
members are the particles in the closest encounters, whose sums are
dominated by one or two pairs and often cancel): float32 mode acceleration
p99 <= 1e-6 and max <= 1e-5, jerk p99 <= 1e-5 and max <= 1e-4; compensated
mode (float64 pair terms) acceleration and jerk p99 <= 1e-11 and max
<= 1e-9; same block as the oracle.  Energy: at eta = 0.02 the float64 oracle's own run of this
workload drifts by 1.68e-5 per time unit (Hermite truncation error, stored
in tests/golden/plummer64k_run.json by make_plummer64k_run.py), above the
1e-6 target, so the GPU's drift is gated against the oracle's: within
1e-7 + 5 % of it, and the step count within 3 %.
"""
import json
import os

import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import CONFIGS, plummer

pytestmark = pytest.mark.gpu

# mode: (acc p99, acc max, jerk p99, jerk max)
GATES = {"fp32": (1e-6, 1e-5, 1e-5, 1e-4), "ds": (1e-11, 1e-9, 1e-11, 1e-9)}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plummer64k_run.json")


def _rel(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_plummer64k_sampled_blocks_and_drift(orc, mode):
    need_gpu()
    import paper_cs_0702135_amd as nb
    cfg = CONFIGS["plummer64k"]
    pos, vel, m = plummer(cfg.n, cfg.seed)
    sysg = nb.System(dev(pos), dev(vel), dev(m), cfg.eps2, eta=cfg.eta, dt_max=cfg.dt_max,
                     mode=mode)
    e0 = sysg.energy()
    rng = np.random.default_rng(cfg.seed + 50)
    ea, ek, sizes = [], [], []
    steps = 0
    while True:
        done = sysg.run(cfg.t_end, max_steps=49)
        steps += done
        if done < 49:
            break
        t, dt = host(sysg.t), host(sysg.dt)
        x, v, a, k = host(sysg.x), host(sysg.v), host(sysg.a), host(sysg.k)
        tn, act = orc.schedule(t, dt)
        if tn > cfg.t_end:
            break
        xp, vp = orc.predict(tn, t, x, v, a, k)
        pick = act if act.size <= 4096 else np.sort(rng.choice(act, 4096, replace=False))
        ra, rk, _ = orc.force(xp, vp, m, cfg.eps2, active=pick.astype(np.int32))
        assert sysg.run(cfg.t_end, max_steps=1) == 1
        steps += 1
        t1 = host(sysg.t)
        assert np.all(t1[act] == tn) and np.count_nonzero(t1 != t) == act.size
        ga, gk = host(sysg.a)[:, pick], host(sysg.k)[:, pick]
        ea.append(_rel(ga, ra))
        ek.append(_rel(gk, rk))
        sizes.append(act.size)
    e1 = sysg.energy()
    assert np.all(host(sysg.t) == cfg.t_end)
    drift = abs((e1 - e0) / e0) / cfg.t_end
    ea, ek = np.concatenate(ea), np.concatenate(ek)
    say("plummer64k %s: %d steps, %d sampled blocks (mean size %.0f), acc median %.2e "
        "p99 %.2e max %.2e, jerk median %.2e p99 %.2e max %.2e, drift/unit %.2e"
        % (mode, steps, len(sizes), np.mean(sizes), np.median(ea), np.percentile(ea, 99),
           ea.max(), np.median(ek), np.percentile(ek, 99), ek.max(), drift))
    ref = json.load(open(GOLDEN))
    say("oracle run: %d steps, drift/unit %.4e" % (ref["steps"], ref["drift_per_time_unit"]))
    assert len(sizes) >= 10
    a99, amax, j99, jmax = GATES[mode]
    assert np.percentile(ea, 99) <= a99 and ea.max() <= amax
    assert np.percentile(ek, 99) <= j99 and ek.max() <= jmax
    d_ref = ref["drift_per_time_unit"]
    assert abs(drift - d_ref) <= 1e-7 + 0.05 * d_ref
    assert abs(steps - ref["steps"]) <= 0.03 * ref["steps"]
