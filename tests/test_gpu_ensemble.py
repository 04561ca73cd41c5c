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


@pytest.mark.parametrize("shape", [(4, 256, 1), (2, 128, 2), (2, 256, 2), (4, 512, 2),
                                   (8, 512, 2)])
def test_every_compiled_shape(orc, shape):
    # the workgroup shapes the autotuner chooses among integrate like the
    # default one: same steps as the oracle's runs, final positions within
    # 1e-6 of the oracle's and of the default shape's (only the order of the
    # float64 combination of wave and split sums differs)
    need_gpu()
    import paper_cs_0702135_amd as nb
    saved = nb.ensemble_get()
    waves, tile, ipl = shape
    sizes = [64, 100, 300, 1024, 2000]
    seeds = [21, 22, 23, 24, 25]
    try:
        for mode in ("fp32", "ds"):
            nb.ensemble_set(waves=4, j_tile=256, i_per_lane=2, groups_per_cu=3)
            ref = host(_run(sizes, seeds, mode=mode)[-1]["x"])
            nb.ensemble_set(waves=waves, j_tile=tile, i_per_lane=ipl,
                            groups_per_cu=max(1, 12 // waves))
            pos, vel, m, off, eps2, out = _run(sizes, seeds, mode=mode)
            d_default = np.abs(host(out["x"]) - ref).max()
            say("shape %r %s: max |x - x(default shape)| %.2e" % (shape, mode, d_default))
            assert d_default < 1e-6
            for c in range(len(sizes)):
                rs, gs, dx, drift = _check_cluster(orc, pos, vel, m, off, eps2, out, c, 1 / 16,
                                                   1 / 16)
                say("shape %r %s cluster %d N=%d: steps GPU %d oracle %d, max|dx| %.2e"
                    % (shape, mode, c, sizes[c], gs, rs, dx))
                assert abs(gs - rs) <= max(2, 0.03 * rs)
                assert dx < 1e-6
    finally:
        nb.ensemble_set(**saved)


def _rel(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_ensemble_force_accuracy_per_cluster(orc, mode):
    # Per-cluster acceleration and jerk errors of the ensemble's pair sums
    # against the oracle, for the smallest and largest clusters of the
    # 256-cluster workload: at the initial state (a launch to t_end = 0 only
    # initialises), and at an evolved state (the clusters integrated to
    # t = 1/32 with dt_max = 1/32, so that every particle ends at 1/32, then
    # initialised again there).  Gates per cluster: float32 mode
    # acceleration p99 <= 1e-6 and max <= 1e-5, jerk p99 <= 1e-5 and max <=
    # 1e-4 (float32 pair terms); compensated mode (float64 pair terms and
    # sums) p99 <= 1e-12 and max <= 1e-10 for both.
    need_gpu()
    import paper_cs_0702135_amd as nb
    cfg = CONFIGS["ensemble256"]
    sizes, eps, seeds = ensemble_members(cfg)
    pos, vel, m, off = _build(sizes, seeds)
    eps2 = eps * eps
    order = np.argsort(sizes)
    pick = list(order[:3]) + list(order[-3:])
    for label, t_mid in (("initial", None), ("t=1/32", 1.0 / 32)):
        P, V = dev(pos), dev(vel)
        if t_mid is not None:
            st = nb.ensemble_run(P, V, dev(m), off, eps2, t_mid, dt_max=t_mid, mode=mode)
            assert np.all(host(st["t"]) == t_mid)
            P, V = st["x"], st["v"]
        out = nb.ensemble_run(P, V, dev(m), off, eps2, 0.0, dt_max=cfg.dt_max, mode=mode)
        x, v = host(P), host(V)
        for c in pick:
            a, b = off[c], off[c + 1]
            ra, rk, _ = orc.force(x[:, a:b], v[:, a:b], m[a:b], eps2[c])
            ea = _rel(host(out["a"])[:, a:b], ra)
            ek = _rel(host(out["k"])[:, a:b], rk)
            say("ensemble %s %s cluster %d N=%d: acc p99 %.2e max %.2e | jerk p99 %.2e max %.2e"
                % (label, mode, c, sizes[c], np.percentile(ea, 99), ea.max(),
                   np.percentile(ek, 99), ek.max()))
            a99, amax, k99, kmax = {"fp32": (1e-6, 1e-5, 1e-5, 1e-4),
                                    "ds": (1e-12, 1e-10, 1e-12, 1e-10)}[mode]
            assert np.percentile(ea, 99) <= a99 and ea.max() <= amax
            assert np.percentile(ek, 99) <= k99 and ek.max() <= kmax
