"""N beyond 2^20 on the GPU, checked against the oracle on sampled particles.

* N = 9,000,000 (the number of particles the paper says its GPU's memory
  holds), eps = 1/4096: pair sums of a seeded active subset of 1024
  particles against all 9e6, both modes, against the oracle evaluating the
  same 1024 particles in float64.  Gates over all 1024: float32 mode
  acceleration p99 <= 1e-7, max <= 1e-6, jerk p99 <= 5e-6, max <= 1e-5;
  compensated mode (float64 pair terms) acceleration and jerk p99 <= 1e-12,
  max <= 1e-11.
* N = 2^22, eps = 1/4096: initialisation (pair sums of every particle) and
  three block steps of the device-resident driver; the initial and the new
  acceleration and jerk of up to 1024 seeded block members are compared
  with the oracle's pair sums at the same (GPU-predicted) state.  Gates for
  the float32 driver: at initialisation as for N = 9e6; for the block
  members (the particles with the smallest |a|/|jerk|, whose acceleration
  sums cancel most) acceleration max <= 1e-5 and jerk max <= 1e-5; the
  block, new times and step sizes must be valid.
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import CONFIGS, plummer, random_active_set

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.fixture(scope="module")
def nine_million():
    cfg = CONFIGS["plummer9m"]
    return cfg, plummer(cfg.n, cfg.seed)


GATES = {"fp32": (1e-7, 1e-6, 5e-6, 1e-5), "ds": (1e-12, 1e-11, 1e-12, 1e-11)}


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_nine_million_sampled_force(orc, nine_million, mode):
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    cfg, (pos, vel, m) = nine_million
    act = random_active_set(cfg.n, cfg.extra["n_sample"], cfg.seed + 1)
    acc, jerk, pot = nb.force(dev(pos), dev(vel), dev(m), cfg.eps2,
                              dev(act, torch.int32), mode)
    ra, rk, rp = orc.force(pos, vel, m, cfg.eps2, active=act)
    ea, ek = _rel(host(acc), ra), _rel(host(jerk), rk)
    ep = np.abs(host(pot) - rp) / np.abs(rp)
    say("N=9e6 %s: acc p50 %.2e p99 %.2e max %.2e | jerk p99 %.2e max %.2e | pot p99 %.2e"
        % (mode, np.median(ea), np.percentile(ea, 99), ea.max(), np.percentile(ek, 99), ek.max(),
           np.percentile(ep, 99)))
    a99, amax, j99, jmax = GATES[mode]
    assert np.percentile(ea, 99) <= a99 and ea.max() <= amax
    assert np.percentile(ek, 99) <= j99 and ek.max() <= jmax


def test_four_million_block_steps(orc):
    need_gpu()
    import paper_cs_0702135_amd as nb
    cfg = CONFIGS["plummer4m"]
    pos, vel, m = plummer(cfg.n, cfg.seed)
    rng = np.random.default_rng(cfg.seed + 2)
    k = cfg.extra["n_sample"]
    sysg = nb.System(dev(pos), dev(vel), dev(m), cfg.eps2, eta=cfg.eta, dt_max=cfg.dt_max)
    pick = np.sort(rng.choice(cfg.n, k, replace=False)).astype(np.int32)
    ra, rk, _ = orc.force(pos, vel, m, cfg.eps2, active=pick)
    ea = _rel(host(sysg.a)[:, pick], ra)
    ek = _rel(host(sysg.k)[:, pick], rk)
    say("N=2^22 init: acc p99 %.2e max %.2e, jerk p99 %.2e max %.2e"
        % (np.percentile(ea, 99), ea.max(), np.percentile(ek, 99), ek.max()))
    a99, amax, j99, jmax = GATES["fp32"]
    assert np.percentile(ea, 99) <= a99 and ea.max() <= amax
    assert np.percentile(ek, 99) <= j99 and ek.max() <= jmax
    for step in range(cfg.extra["steps"]):
        t, dt = host(sysg.t), host(sysg.dt)
        x, v, a, kk = host(sysg.x), host(sysg.v), host(sysg.a), host(sysg.k)
        tn, act = orc.schedule(t, dt)
        xp, vp = orc.predict(tn, t, x, v, a, kk)
        sel = act if act.size <= k else np.sort(rng.choice(act, k, replace=False))
        ra, rk, _ = orc.force(xp, vp, m, cfg.eps2, active=sel.astype(np.int32))
        assert sysg.step(1) == 1
        t1, dt1 = host(sysg.t), host(sysg.dt)
        assert np.all(t1[act] == tn) and np.count_nonzero(t1 != t) == act.size
        # new steps are powers of two that divide the new time
        d = dt1[act]
        assert np.all(np.frexp(d)[0] == 0.5) and np.all(np.fmod(t1[act], d) == 0)
        ea = _rel(host(sysg.a)[:, sel], ra)
        ek = _rel(host(sysg.k)[:, sel], rk)
        say("N=2^22 step %d: block %d at t=%.6g, acc p50 %.2e max %.2e, jerk p50 %.2e max %.2e"
            % (step, act.size, tn, np.median(ea), ea.max(), np.median(ek), ek.max()))
        assert ea.max() <= 1e-5
        assert ek.max() <= 1e-5
