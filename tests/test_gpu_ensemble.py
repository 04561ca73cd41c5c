"""GPU batched ensemble (one persistent launch) against per-cluster oracle runs.

Each cluster is integrated by the FP64 oracle from the same initial state
with the same block-step rules.  float32 pair sums can flip a rare step-size
decision, so trajectories are compared with a tolerance: same end time for
every particle, block-step counts within a few percent, final positions
within 1e-6, and the same energy drift as the oracle's run of the cluster
(the drift itself is the integrator's truncation error at eta = 0.02, which
can exceed 1e-6 per time unit for the largest clusters in both).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import CONFIGS, ensemble_members, plummer

pytestmark = pytest.mark.gpu


def _build(sizes, seeds):
    ps, vs, ms = [], [], []
    for n, sd in zip(sizes, seeds):
        p, v, m = plummer(int(n), int(sd))
        ps.append(p), vs.append(v), ms.append(m)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return (np.concatenate(ps, axis=1), np.concatenate(vs, axis=1), np.concatenate(ms), off)


def _run(sizes, seeds, t_end=1.0 / 16, dt_max=1.0 / 16, mode="fp32"):
    import paper_cs_0702135_amd as nb
    pos, vel, m, off = _build(sizes, seeds)
    eps = np.asarray(sizes, dtype=np.float64) ** (-1.0 / 3.0) / 16.0
    out = nb.ensemble_run(dev(pos), dev(vel), dev(m), off, eps * eps, t_end, dt_max=dt_max,
                          mode=mode)
    return pos, vel, m, off, eps * eps, out


def _check_cluster(orc, pos, vel, m, off, eps2, out, c, t_end, dt_max):
    a, b = off[c], off[c + 1]
    s = orc.init_state(pos[:, a:b], vel[:, a:b], m[a:b], eps2[c], dt_max=dt_max)
    e0 = sum(orc.energy(s.x, s.v, s.m, s.eps2))
    steps, _ = orc.integrate(s, t_end)
    e_ref = sum(orc.energy(s.x, s.v, s.m, s.eps2))
    x = host(out["x"])[:, a:b]
    v = host(out["v"])[:, a:b]
    t = host(out["t"])[a:b]
    assert np.all(t == t_end), "cluster %d did not end at t_end" % c
    dx = np.abs(x - s.x).max()
    e1 = sum(orc.energy(x, v, m[a:b], eps2[c]))
    drift = abs((e1 - e0) / e0) / t_end
    drift_ref = abs((e_ref - e0) / e0) / t_end
    say("  cluster %d: drift/unit GPU %.3e, oracle %.3e" % (c, drift, drift_ref))
    assert abs(drift - drift_ref) <= 1e-7 + 0.05 * drift_ref
    return steps, out["steps"][c], dx, drift


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_small_mixed_ensemble(orc, mode):
    need_gpu()
    sizes = [2, 64, 100, 256, 300, 513, 1024]
    seeds = [11, 12, 13, 14, 15, 16, 17]
    pos, vel, m, off, eps2, out = _run(sizes, seeds, mode=mode)
    for c in range(len(sizes)):
        rs, gs, dx, drift = _check_cluster(orc, pos, vel, m, off, eps2, out, c, 1 / 16, 1 / 16)
        say("cluster %d N=%d: steps GPU %d oracle %d, max|dx| %.2e, drift/unit %.2e"
            % (c, sizes[c], gs, rs, dx, drift))
        assert abs(gs - rs) <= max(2, 0.03 * rs)
        assert dx < 1e-6


def test_multi_group_team(orc):
    # one large cluster among small ones gets a team of several groups
    need_gpu()
    import paper_cs_0702135_amd as nb
    saved = nb.ensemble_get()
    nb.ensemble_set(groups_per_cu=1, max_team=32)
    try:
        sizes = [3000] + [128] * 20
        seeds = list(range(100, 121))
        pos, vel, m, off, eps2, out = _run(sizes, seeds)
        grid, teams = nb.ensemble_info()
        say("grid %d groups, %d teams" % (grid, teams))
        assert teams < grid  # at least one team has more than one group
        for c in (0, 1, 20):
            rs, gs, dx, drift = _check_cluster(orc, pos, vel, m, off, eps2, out, c, 1 / 16, 1 / 16)
            say("cluster %d N=%d: steps GPU %d oracle %d, max|dx| %.2e, drift/unit %.2e"
                % (c, sizes[c], gs, rs, dx, drift))
            assert abs(gs - rs) <= max(2, 0.03 * rs)
            assert dx < 1e-6
    finally:
        nb.ensemble_set(**saved)


def test_full_ensemble_workload(orc):
    # 256 clusters, N log-uniform in [256, 8192], eps = N^(-1/3)/16, to t = 1/16
    need_gpu()
    cfg = CONFIGS["ensemble256"]
    sizes, eps, seeds = ensemble_members(cfg)
    pos, vel, m, off, eps2, out = _run(sizes, seeds, cfg.t_end, cfg.dt_max)
    say("ensemble of %d clusters, %d particles, %.3e interactions"
        % (len(sizes), off[-1], float(sum(out["interactions"]))))
    assert np.all(host(out["t"]) == cfg.t_end)
    order = np.argsort(sizes)
    for c in list(order[:3]) + list(order[-2:]):
        rs, gs, dx, drift = _check_cluster(orc, pos, vel, m, off, eps2, out, c, cfg.t_end,
                                           cfg.dt_max)
        say("cluster %d N=%d: steps GPU %d oracle %d, max|dx| %.2e, drift/unit %.2e"
            % (c, sizes[c], gs, rs, dx, drift))
        assert abs(gs - rs) <= max(2, 0.03 * rs)
        assert dx < 1e-6
