"""Checks of the seeded input generators (Plummer spheres, ensembles).

Plummer sampling: Aarseth, Henon & Wielen (1974), cited in Section 4 for the
paper's initial conditions; N-body units (G = M = 1, E = -1/4).
"""
import math

import numpy as np
from scipy import stats

from workloads.plummer import (CONFIGS, ensemble_members, plummer,
                               random_active_set)


def test_plummer_is_deterministic_and_centred():
    p1, v1, m1 = plummer(2048, 5)
    p2, v2, m2 = plummer(2048, 5)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(v1, v2)
    assert np.abs(p1.mean(axis=1)).max() < 1e-15
    assert np.abs(v1.mean(axis=1)).max() < 1e-15
    assert np.all(m1 == 1 / 2048)


def test_plummer_mass_profile_ks():
    # M(<r) = r^3 / (r^2 + b^2)^(3/2) with b = 3 pi / 16, truncated at 0.999
    p, _, _ = plummer(20000, 6)
    r = np.sqrt((p ** 2).sum(0))
    b = 3 * math.pi / 16

    def cdf(x):
        return np.minimum(x ** 3 / (x * x + b * b) ** 1.5 / 0.999, 1.0)

    assert stats.kstest(r, cdf).pvalue > 0.01


def test_plummer_virial_energy(orc):
    # kinetic 1/4 and potential -1/2 in N-body units, statistically
    p, v, m = plummer(8192, 7)
    K, W = orc.energy(p, v, m, 0.0)
    assert abs(K - 0.25) < 0.01
    assert abs(W + 0.5) < 0.02
    assert abs(2 * K / abs(W) - 1) < 0.05


def test_ensemble_members():
    sizes, eps, seeds = ensemble_members()
    assert sizes.shape == (256,) and sizes.min() >= 256 and sizes.max() <= 8192
    np.testing.assert_allclose(eps, sizes ** (-1 / 3) / 16)
    assert len(set(seeds.tolist())) == 256
    # log-uniform: about half the clusters below the geometric midpoint
    assert 0.35 < (sizes < math.sqrt(256 * 8192)).mean() < 0.65


def test_active_sets_and_configs():
    a = random_active_set(1000, 100, 1)
    assert a.dtype == np.int32 and np.all(np.diff(a) > 0)
    assert CONFIGS["plummer1m"].n == 1 << 20
    assert CONFIGS["plummer1k"].eps2 == (1 / 256) ** 2


def test_table_protocol_config():
    from workloads.plummer import CONFIGS, table_protocol_seed
    cfg = CONFIGS["table_protocol"]
    assert cfg.extra["n_list"][0] == 256 and cfg.extra["n_list"][-1] == 524288
    assert cfg.eps == 1.0 / 256 and cfg.dt_max == 0.125 and cfg.t_end == 0.5
    assert cfg.extra["timed_from"] == 0.25
    seeds = [table_protocol_seed(n) for n in cfg.extra["n_list"]]
    assert len(set(seeds)) == len(seeds)


def test_power_law_fit_recovers_exact_law():
    import bench
    x = [256 << k for k in range(8)]
    c, p = bench.fit_power_law(x, [0.2 * v ** 0.81 for v in x])
    assert abs(c - 0.2) < 1e-9 and abs(p - 0.81) < 1e-12
