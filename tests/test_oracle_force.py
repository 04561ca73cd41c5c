"""Pins of the oracle's pair sums (acceleration, jerk, potential).

Each check compares the oracle with something that does not come from the
oracle's own formula: closed forms of symmetric configurations, exact
conservation laws of the pairwise force, and derivative identities (jerk is
the time derivative of the acceleration, acceleration minus the gradient of
the potential) evaluated by finite differences.

Force law: Section 2, Eq. (1), softened as in the Appendix A listing.
"""
import math

import numpy as np
import pytest

from workloads.plummer import plummer, random_active_set


def _binary(m1, m2, d, eps):
    M = m1 + m2
    s = d * d + eps * eps
    om = math.sqrt(M / s ** 1.5)
    pos = np.array([[-m2 * d / M, m1 * d / M], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [-m2 * d * om / M, m1 * d * om / M], [0.0, 0.0]])
    return pos, vel, np.array([m1, m2]), om, s


@pytest.mark.parametrize("eps", [0.0, 0.05, 0.3])
def test_circular_binary_closed_form(orc, eps):
    # softened circular orbit: omega^2 = M / (d^2+eps^2)^(3/2), a = -omega^2 x,
    # k = -omega^2 v, phi_1 = -m_2 / sqrt(d^2 + eps^2)
    pos, vel, m, om, s = _binary(0.3, 0.7, 1.3, eps)
    acc, jerk, pot = orc.force(pos, vel, m, eps * eps)
    np.testing.assert_allclose(acc, -om * om * pos, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(jerk, -om * om * vel, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(pot, [-m[1] / math.sqrt(s), -m[0] / math.sqrt(s)],
                               rtol=1e-15)


@pytest.mark.parametrize("eps", [0.0, 0.1])
def test_equilateral_triangle(orc, eps):
    # three equal masses on a triangle of side L: each acceleration points to
    # the centroid with magnitude sqrt(3) m L / (L^2 + eps^2)^(3/2)
    L, m = 0.8, 0.25
    R = L / math.sqrt(3.0)
    ang = np.array([0.3, 0.3 + 2 * math.pi / 3, 0.3 + 4 * math.pi / 3])
    pos = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(3)])
    vel = np.zeros((3, 3))
    acc, jerk, pot = orc.force(pos, vel, np.full(3, m), eps * eps)
    mag = math.sqrt(3.0) * m * L / (L * L + eps * eps) ** 1.5
    np.testing.assert_allclose(acc, -mag * pos / R, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(jerk, 0.0, atol=1e-15)
    np.testing.assert_allclose(pot, -2 * m / math.sqrt(L * L + eps * eps), rtol=1e-15)


def _random_system(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    pos = rng.normal(0, spread, (3, n))
    vel = rng.normal(0, 0.5, (3, n))
    m = rng.uniform(0.5, 1.5, n) / n
    return pos, vel, m


def test_jerk_is_time_derivative_of_acceleration(orc):
    # k_i = d/dt a_i along straight-line motion x(t) = x + t v (the pair sums
    # depend on time only through the positions): central differences
    pos, vel, m = _random_system(16, 7)
    eps2 = 0.01 ** 2
    tau = 1e-5
    ap, _, _ = orc.force(pos + tau * vel, vel, m, eps2)
    am, _, _ = orc.force(pos - tau * vel, vel, m, eps2)
    _, jerk, _ = orc.force(pos, vel, m, eps2)
    fd = (ap - am) / (2 * tau)
    np.testing.assert_allclose(jerk, fd, rtol=1e-7, atol=1e-8 * np.abs(jerk).max())


def test_acceleration_is_minus_gradient_of_potential(orc):
    # phi_i as a function of x_i alone: a_i = -grad_{x_i} phi_i
    pos, vel, m = _random_system(12, 8)
    eps2 = 0.02 ** 2
    acc, _, _ = orc.force(pos, vel, m, eps2)
    h = 1e-6
    for i in range(12):
        for c in range(3):
            p1 = pos.copy()
            p1[c, i] += h
            p2 = pos.copy()
            p2[c, i] -= h
            f1 = orc.force(p1, vel, m, eps2, active=[i])[2][0]
            f2 = orc.force(p2, vel, m, eps2, active=[i])[2][0]
            g = (f1 - f2) / (2 * h)
            assert abs(-g - acc[c, i]) <= 1e-7 * max(1.0, abs(acc[c, i]))


def test_newton_third_law_and_angular_momentum(orc):
    # pairwise antisymmetric forces: sum m a = sum m k = 0 and, for central
    # forces, sum m x cross a = 0, in exact arithmetic
    pos, vel, m = plummer(512, 11)
    acc, jerk, _ = orc.force(pos, vel, m, 1e-4)
    scale_a = (m * np.abs(acc)).sum()
    scale_k = (m * np.abs(jerk)).sum()
    assert np.abs((m * acc).sum(axis=1)).max() < 1e-13 * scale_a
    assert np.abs((m * jerk).sum(axis=1)).max() < 1e-13 * scale_k
    torque = np.cross(pos.T, acc.T) * m[:, None]
    assert np.abs(torque.sum(axis=0)).max() < 1e-13 * (m * np.abs(pos).sum(0) * np.abs(acc).sum(0)).sum()


def test_active_subset_matches_full_set(orc):
    pos, vel, m = plummer(300, 12)
    full = orc.force(pos, vel, m, 1e-3)
    act = random_active_set(300, 37, 5)
    sub = orc.force(pos, vel, m, 1e-3, active=act)
    for f, s in zip(full, sub):
        np.testing.assert_array_equal(f[..., act], s)


def test_plummer_mean_field(orc):
    # a large Plummer sample feels, on average, the smooth Plummer field
    # a(r) = -r / (r^2 + b^2)^(3/2), b = 3 pi / 16 in N-body units
    pos, vel, m = plummer(16384, 21)
    act = random_active_set(16384, 512, 22)
    acc, _, pot = orc.force(pos, vel, m, (1.0 / 4096) ** 2, active=act)
    r = np.sqrt((pos[:, act] ** 2).sum(0))
    b = 3 * math.pi / 16
    a_model = r / (r * r + b * b) ** 1.5
    a_rad = (acc * pos[:, act]).sum(0) / r
    ratio = -a_rad / a_model
    assert abs(np.median(ratio) - 1.0) < 0.03
    phi_model = -1.0 / np.sqrt(r * r + b * b)
    assert abs(np.median(pot / phi_model) - 1.0) < 0.02


def test_self_pair_excluded_by_index(orc):
    # eps = 0 with distinct positions is finite (the self pair is skipped)
    pos, vel, m, om, s = _binary(0.5, 0.5, 1.0, 0.0)
    acc, jerk, pot = orc.force(pos, vel, m, 0.0)
    assert np.isfinite(acc).all() and np.isfinite(pot).all()
