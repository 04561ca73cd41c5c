"""Pins of the oracle's Hermite integrator, block scheduler and energy.

Predictor and corrector: Section 2 (the printed Taylor forms).  They are
checked against polynomial trajectories on which they must be exact, and the
whole scheme against fourth-order convergence on a Kepler orbit.  The time
step criterion (a reading: Aarseth's, the paper does not state it) is pinned
by its closed form on a circular orbit; block statistics are compared with
the fits printed in Section 5 (a loose band only).
"""
import json
import math
import os

import numpy as np
import pytest

from workloads.plummer import plummer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_fits.json")


def test_predictor_exact_on_cubics(orc):
    # x(t) = x0 + v0 t + a0 t^2/2 + k0 t^3/6 is reproduced exactly
    rng = np.random.default_rng(3)
    n = 50
    x0, v0, a0, k0 = (rng.normal(size=(3, n)) for _ in range(4))
    t = rng.uniform(0, 1, n)
    h = rng.uniform(0, 0.3, n)
    xp, vp = orc.predict(0.0, t - 0.0, x0, v0, a0, k0)  # dt = -t
    for c in range(3):
        for i in range(n):
            d = -t[i]
            X = np.polynomial.polynomial.polyval(d, [x0[c, i], v0[c, i], a0[c, i] / 2, k0[c, i] / 6])
            V = np.polynomial.polynomial.polyval(d, [v0[c, i], a0[c, i], k0[c, i] / 2])
            assert abs(xp[c, i] - X) <= 1e-14 * (1 + abs(X))
            assert abs(vp[c, i] - V) <= 1e-14 * (1 + abs(V))
    # dt = 0 is the identity
    xp, vp = orc.predict(0.5, np.full(n, 0.5), x0, v0, a0, k0)
    np.testing.assert_array_equal(xp, x0)
    np.testing.assert_array_equal(vp, v0)
    del h


def test_corrector_exact_on_quintics(orc):
    # If x(t) is a quintic, a(t) is a cubic and the Hermite interpolant of
    # (a, k) at both ends is exact, so the corrected x, v are exact.
    rng = np.random.default_rng(4)
    n = 40
    c = rng.normal(size=(6, 3, n))  # x = sum c_p t^p / p!
    h = 2.0 ** -3
    fact = [math.factorial(p) for p in range(6)]

    def deriv(order, t):
        return sum(c[p] * t ** (p - order) / fact[p - order] for p in range(order, 6))

    x0, v0, a0, k0 = deriv(0, 0.0), deriv(1, 0.0), deriv(2, 0.0), deriv(3, 0.0)
    t = np.zeros(n)
    xp, vp = orc.predict(h, t, x0, v0, a0, k0)
    a1, k1 = deriv(2, h), deriv(3, h)
    x, v, a, k = x0.copy(), v0.copy(), a0.copy(), k0.copy()
    dt = np.full(n, h)
    rc = orc.correct(None, xp, vp, a1, k1, 0.02, 1.0, 2.0 ** -40, t, dt, x, v, a, k,
                     fixed_dt=True)
    assert rc == 0
    np.testing.assert_allclose(x, deriv(0, h), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(v, deriv(1, h), rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(a, a1)
    np.testing.assert_array_equal(t, h)
    # a scheme that drops the third-derivative term is visibly off
    assert np.abs(x - (xp + (-3 * (a0 - a1) - (2 * k0 + k1) * h) / 12 * h * h)).max() > 1e-8


def _kepler(e=0.5):
    # relative orbit with a = 1, M = 1, started at pericentre; equal masses
    M, a = 1.0, 1.0
    rp = a * (1 - e)
    vp = math.sqrt(M * (1 + e) / rp)
    m = np.array([0.5, 0.5])
    pos = np.array([[-rp / 2, rp / 2], [0, 0], [0, 0]], dtype=float)
    vel = np.array([[0, 0], [-vp / 2, vp / 2], [0, 0]], dtype=float)
    return pos, vel, m, 2 * math.pi * math.sqrt(a ** 3 / M)


def test_fourth_order_convergence_kepler(orc):
    # one period with shared steps: the position error falls ~16x per halving
    pos, vel, m, P = _kepler()
    errs = []
    for nst in (256, 512, 1024):
        x, v, a, k = orc.shared_run(pos, vel, m, 0.0, P / nst, nst)
        errs.append(np.abs(x - pos).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, (errs, r1, r2)


def _circular_state(om, R, t):
    x = np.array([[R * math.cos(om * t)], [R * math.sin(om * t)], [0.0]])
    v = np.array([[-R * om * math.sin(om * t)], [R * om * math.cos(om * t)], [0.0]])
    return x, v, -om * om * x, -om * om * v


@pytest.mark.parametrize("ratio,h_exp,t0,expect_exp", [
    (0.85, -6, 0.0, -7),          # dt_crit < dt: halve
    (1.15, -6, 0.0, -6),          # dt <= dt_crit < 2 dt: keep
    (1.85, -6, 2.0 ** -6, -6),    # 2 dt > dt_crit: keep
    (2.15, -6, 2.0 ** -6, -5),    # 2 dt <= dt_crit and t_new = 2^-5: double
    (2.15, -6, 0.0, -6),          # t_new = 2^-6 is not a multiple of 2^-5: keep
    (4.5, -6, 2.0 ** -6, -5),     # doubles once only
])
def test_aarseth_step_closed_form_on_circular_orbit(orc, ratio, h_exp, t0, expect_exp):
    # On a circle |a| = w^2 R, |k| = w^3 R, |a''| = w^4 R, |a'''| = w^5 R, so
    # the criterion gives dt_crit = sqrt(eta) / w independently of R.
    eta = 0.02
    target = ratio * 2.0 ** -6
    om = math.sqrt(eta) / target
    h = 2.0 ** h_exp
    R = 0.7
    x0, v0, a0, k0 = _circular_state(om, R, t0)
    x1, v1, a1, k1 = _circular_state(om, R, t0 + h)
    t = np.array([t0])
    dt = np.array([h])
    xp, vp = orc.predict(t0 + h, t, x0, v0, a0, k0)
    x, v, a, k = x0.copy(), v0.copy(), a0.copy(), k0.copy()
    rc = orc.correct(None, xp, vp, a1, k1, eta, 0.125, 2.0 ** -40, t, dt, x, v, a, k)
    assert rc == 0
    assert dt[0] == 2.0 ** expect_exp


def test_step_criterion_uses_end_of_step_derivatives(orc):
    # a(t) cubic, so the corrector's a2, a3 are exact.  Chosen (in units of
    # the step h) so that the end-of-step derivatives |a| = 900,
    # |k| h = 0.375, |d2a/dt2| h^2 = 0.59, |d3a/dt3| h^3 = 0.59 give
    # dt_crit ~ 4.3 h (the step may double), while the start-of-step second
    # derivative (exactly zero here) would give dt_crit ~ 0.11 h.
    eta, h, t0 = 0.02, 2.0 ** -6, 2.0 ** -6
    A, K, S, T = 900.0, -0.375 / h, -0.59 / h ** 2, -0.59 / h ** 3

    def vec(q):
        return np.array([[q], [0.0], [0.0]])

    a1, k1 = vec(A), vec(K)
    a0 = vec(A - K * h + S * h * h / 2 - T * h ** 3 / 6)
    k0 = vec(K - S * h + T * h * h / 2)
    x0, v0 = vec(0.3), vec(-0.2)
    t = np.array([t0])
    dt = np.array([h])
    xp, vp = orc.predict(t0 + h, t, x0, v0, a0, k0)
    x, v, a, k = x0.copy(), v0.copy(), a0.copy(), k0.copy()
    rc = orc.correct(None, xp, vp, a1, k1, eta, 0.125, 2.0 ** -40, t, dt, x, v, a, k)
    assert rc == 0
    assert dt[0] == 2 * h


def test_initial_step_power_of_two(orc):
    rng = np.random.default_rng(9)
    a = rng.normal(size=(3, 200))
    k = rng.normal(size=(3, 200)) * 10 ** rng.uniform(-2, 3, 200)
    dt, rc = orc.initial_dt(0.0, a, k, 0.01, 0.125, 2.0 ** -40)
    assert rc == 0
    want = 0.01 * np.linalg.norm(a, axis=0) / np.linalg.norm(k, axis=0)
    e = np.log2(dt)
    assert np.all(e == np.round(e))
    assert np.all(dt <= np.minimum(want, 0.125))
    assert np.all(np.minimum(2 * dt, 0.25) > np.minimum(want, 0.125))
    # a restart at t0 = 3/8 also needs t0 to be a multiple of the step
    dt2, rc = orc.initial_dt(0.375, a, k, 0.01, 0.125, 2.0 ** -40)
    assert rc == 0 and np.all(np.fmod(0.375, dt2) == 0)


def test_initial_step_flags_nonfinite_norms(orc):
    # a NaN or infinite |a| or |k| gives no step: dt_min, reported; zero
    # jerk alone is finite and sets no limit (dt_max)
    a = np.ones((3, 4))
    k = np.ones((3, 4))
    k[1, 0] = np.nan
    a[2, 1] = np.inf
    k[:, 2] = 0.0
    dt, rc = orc.initial_dt(0.0, a, k, 0.01, 0.125, 2.0 ** -40)
    assert rc == orc.E_NONFINITE
    assert dt[0] == 2.0 ** -40 and dt[1] == 2.0 ** -40
    assert dt[2] == 0.125
    e = np.log2(dt[3])
    assert e == np.round(e) and dt[3] <= 0.01


@pytest.mark.parametrize("fixed_dt", [False, True])
def test_corrector_reports_nonfinite_state(orc, fixed_dt):
    # a NaN in the new force of one particle: reported, its step kept; the
    # other particle is corrected as usual
    n = 2
    rng = np.random.default_rng(12)
    x, v, a, k = (rng.normal(size=(3, n)) for _ in range(4))
    t = np.zeros(n)
    dt = np.full(n, 1.0 / 64)
    an, kn = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    an[1, 0] = np.nan
    rc = orc.correct(None, x.copy(), v.copy(), an, kn, 0.02, 0.125, 2.0 ** -40, t, dt, x, v, a,
                     k, fixed_dt=fixed_dt)
    assert rc == orc.E_NONFINITE
    assert dt[0] == 1.0 / 64 and np.all(t == 1.0 / 64)
    assert np.all(np.isfinite(x[:, 1])) and np.all(np.isfinite(v[:, 1]))


def test_scheduler_definition(orc):
    rng = np.random.default_rng(10)
    n = 1000
    e = rng.integers(3, 12, n)
    dt = 2.0 ** -e
    t = np.floor(rng.uniform(0, 1, n) / dt) * dt
    tn, act = orc.schedule(t, dt)
    assert tn == (t + dt).min()
    np.testing.assert_array_equal(act, np.nonzero(t + dt == tn)[0])


def test_two_body_energy_closed_form(orc):
    m = np.array([0.2, 0.8])
    pos = np.array([[0.1, -0.4], [0.3, 0.2], [-0.2, 0.5]])
    vel = np.array([[0.5, -0.1], [0.0, 0.3], [0.2, 0.1]])
    eps = 0.1
    K, W = orc.energy(pos, vel, m, eps * eps)
    d2 = ((pos[:, 0] - pos[:, 1]) ** 2).sum()
    assert abs(K - 0.5 * (m * (vel ** 2).sum(0)).sum()) < 1e-16
    assert abs(W - (-m[0] * m[1] / math.sqrt(d2 + eps * eps))) < 1e-16


def test_block_invariants_each_step(orc):
    pos, vel, m = plummer(256, 31)
    s = orc.init_state(pos, vel, m, (1 / 256) ** 2)
    for _ in range(150):
        n_i, tn, act = orc.blockstep(s)
        assert n_i > 0
        assert np.all(s.t[act] == tn)
        e = np.log2(s.dt)
        assert np.all(e == np.round(e)) and np.all(s.dt <= 0.125)
        assert np.all(np.fmod(s.t, s.dt) == 0)
        assert (s.t + s.dt).min() > tn
    # all particles meet at the next multiple of dt_max
    orc.integrate(s, 0.125)
    assert np.all(s.t == 0.125)


def test_plummer_energy_conservation_and_block_statistics(orc):
    # Plummer N = 1024, eps = 1/256, eta = 0.02, dt_max = 1/8, to t = 1/4
    fits = json.load(open(GOLDEN))
    n = 1024
    pos, vel, m = plummer(n, 1001)
    eps2 = (1 / 256) ** 2
    s = orc.init_state(pos, vel, m, eps2)
    e0 = sum(orc.energy(s.x, s.v, m, eps2))
    steps, blk = orc.integrate(s, 0.25)
    e1 = sum(orc.energy(s.x, s.v, m, eps2))
    drift_per_unit = abs((e1 - e0) / e0) / 0.25
    assert drift_per_unit < 1e-6
    nb = fits["n_block"]
    ns = fits["n_steps_per_time_unit"]
    mean_block = blk / steps
    steps_per_unit = steps / 0.25
    assert 0.5 < mean_block / (nb["coef"] * n ** nb["exp"]) < 2.0
    assert 0.5 < steps_per_unit / (ns["coef"] * n ** ns["exp"]) < 2.0
