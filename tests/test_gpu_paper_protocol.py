"""The Section 4 results-table protocol on the GPU against the oracle.

For N = 1024 and 4096 (the protocol's own seeded realisations; eps = 1/256,
eta = 0.02, dt_max = 1/8) the GPU block-step driver and the float64 oracle
both integrate from t = 0 to 1/4 (the untimed part) and on to 1/2 (the
timed part).  Gates: block steps in each part within 1 % of the oracle's,
every particle at t = 1/2, the same mean block size within 1 %, and the
relative energy drift per time unit within 1e-7 + 5 % of the oracle's.
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import CONFIGS, plummer, table_protocol_seed

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1024, 4096])
def test_table_protocol_matches_oracle(orc, n):
    need_gpu()
    import paper_cs_0702135_amd as nb
    cfg = CONFIGS["table_protocol"]
    t_from = cfg.extra["timed_from"]
    pos, vel, m = plummer(n, table_protocol_seed(n))
    sysg = nb.System(dev(pos), dev(vel), dev(m), cfg.eps2, eta=cfg.eta, eta_s=cfg.eta_s,
                     dt_max=cfg.dt_max)
    e0 = sysg.energy()
    g0 = sysg.run(t_from)
    i0 = sysg.interactions
    g1 = sysg.run(cfg.t_end)
    gi = sysg.interactions - i0
    e1 = sysg.energy()
    assert np.all(host(sysg.t) == cfg.t_end)
    g_drift = abs((e1 - e0) / e0) / cfg.t_end

    s = orc.init_state(pos, vel, m, cfg.eps2, eta=cfg.eta, eta_s=cfg.eta_s, dt_max=cfg.dt_max)
    r0, _ = orc.integrate(s, t_from)
    r1, rb = orc.integrate(s, cfg.t_end)
    assert np.all(s.t == cfg.t_end)
    r_drift = abs((sum(orc.energy(s.x, s.v, m, cfg.eps2)) - sum(orc.energy(pos, vel, m, cfg.eps2)))
                  / sum(orc.energy(pos, vel, m, cfg.eps2))) / cfg.t_end
    g_block, r_block = gi / g1 / n, rb / r1
    say("protocol N=%d: steps GPU %d + %d, oracle %d + %d; mean block GPU %.2f oracle %.2f; "
        "drift/unit GPU %.3e oracle %.3e" % (n, g0, g1, r0, r1, g_block, r_block, g_drift,
                                            r_drift))
    assert abs(g0 - r0) <= 0.01 * r0 and abs(g1 - r1) <= 0.01 * r1
    assert abs(g_block - r_block) <= 0.01 * r_block
    assert abs(g_drift - r_drift) <= 1e-7 + 0.05 * r_drift
