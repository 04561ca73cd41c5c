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


# ---- float32 sums in index order and smallest force first (Section 6) ----

def test_sum32_single_term_is_rounded_exact_term(orc):
    # two particles: each sum has one term, so both orders give the float32
    # rounding of the float64 term
    pos = np.array([[0.0, 0.3], [0.0, -0.2], [0.0, 0.1]])
    vel = np.array([[0.1, -0.05], [0.0, 0.2], [0.3, 0.0]])
    m = np.array([0.25, 0.75])
    ra, rk, rp = orc.force(pos, vel, m, 1e-3)
    for order in ("index", "sorted"):
        a, k, p = orc.force_sum32(pos, vel, m, 1e-3, order=order)
        np.testing.assert_array_equal(a, ra.astype(np.float32).astype(np.float64))
        np.testing.assert_array_equal(k, rk.astype(np.float32).astype(np.float64))
        np.testing.assert_array_equal(p, rp.astype(np.float32).astype(np.float64))


def test_sorted_sum32_keeps_small_forces_that_index_order_drops(orc):
    # particle 0 at the origin, particle 1 close by (one large force), then
    # 4000 distant particles whose forces are each below half an ulp of the
    # large one: added after it in index order they are all lost; added
    # first (smallest first) they survive, so the sorted float32 sum is
    # within an ulp of the float64 sum.
    k = 4000
    x = np.zeros((3, k + 2))
    x[0, 1] = 0.01
    rng = np.random.default_rng(5)
    x[0, 2:] = 100.0 + rng.uniform(0, 1, k)
    m = np.full(k + 2, 1e-3)
    v = np.zeros_like(x)
    ra, _, _ = orc.force(x, v, m, 0.0, active=np.array([0], np.int32))
    ai, _, _ = orc.force_sum32(x, v, m, 0.0, active=np.array([0], np.int32), order="index")
    asd, _, _ = orc.force_sum32(x, v, m, 0.0, active=np.array([0], np.int32), order="sorted")
    exact = ra[0, 0]
    ulp = np.spacing(np.float32(exact))
    assert abs(asd[0, 0] - exact) <= ulp
    assert abs(ai[0, 0] - exact) > 100 * ulp
    # the index-order float32 sum equals the large term alone
    assert ai[0, 0] == float(np.float32(np.float32(1e-3 / 0.01 ** 2)))


def test_sorted_sum32_does_not_depend_on_particle_order(orc):
    pos, vel, m = plummer(700, 41)
    m = m * (1.0 + 0.5 * np.random.default_rng(42).uniform(size=m.shape))  # distinct keys
    perm = np.random.default_rng(43).permutation(700)
    a0, k0, p0 = orc.force_sum32(pos, vel, m, 1e-4, order="sorted")
    a1, k1, p1 = orc.force_sum32(pos[:, perm], vel[:, perm], m[perm], 1e-4, order="sorted")
    inv = np.argsort(perm)
    np.testing.assert_array_equal(a1[:, inv], a0)
    np.testing.assert_array_equal(k1[:, inv], k0)
    np.testing.assert_array_equal(p1[inv], p0)
    # index order does depend on it (float32 addition is not associative)
    b0 = orc.force_sum32(pos, vel, m, 1e-4, order="index")[0]
    b1 = orc.force_sum32(pos[:, perm], vel[:, perm], m[perm], 1e-4, order="index")[0]
    assert not np.array_equal(b1[:, inv], b0)


def test_sum32_orders_close_to_float64_sum(orc):
    # both float32 sums stay within float32 accumulation error of the exact
    # sum on a small Plummer sphere
    pos, vel, m = plummer(2048, 44)
    ra, _, _ = orc.force(pos, vel, m, 1e-4)
    for order in ("index", "sorted"):
        a, _, _ = orc.force_sum32(pos, vel, m, 1e-4, order=order)
        err = np.linalg.norm(a - ra, axis=0) / np.linalg.norm(ra, axis=0)
        assert np.percentile(err, 99) < 2e-5


def test_sorted_sum32_orders_by_force_not_distance(orc):
    # particle 0 at the origin; a massive distant particle (m = 1e4 at
    # x = 100) and a light near one (m = 1 at x = -1) pull with forces +1
    # and -1; 1000 particles at x ~ 10 add 4e-8 each (4e-5 in all), each
    # below half an ulp of 1.  Smallest force first, the 4e-5 is summed
    # before the two unit forces and survives their cancellation; ordered
    # by distance instead, the far unit force would come first and swallow
    # every small term.
    k = 1000
    x = np.zeros((3, k + 3))
    x[0, 1], x[0, 2] = 100.0, -1.0
    x[0, 3:] = 10.0 + np.random.default_rng(6).uniform(0, 1e-3, k)
    m = np.full(k + 3, 4e-6)
    m[1], m[2] = 1e4, 1.0
    v = np.zeros_like(x)
    one = np.array([0], np.int32)
    exact = orc.force(x, v, m, 0.0, active=one)[0][0, 0]
    got = orc.force_sum32(x, v, m, 0.0, active=one, order="sorted")[0][0, 0]
    assert 3.9e-5 < exact < 4.1e-5
    assert abs(got - exact) <= 1e-2 * exact
