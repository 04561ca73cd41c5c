"""Pins of the oracle's adjoint of the pair sums and of the Hermite chain.

The adjoint is not in the paper; it is derived from the Appendix A force law.
It is pinned by the defining identity of a transpose (the dot-product test
against central finite differences of the forward oracle), by translation
invariance (the force depends on differences only), and by homogeneity in the
masses (a, k, phi are linear in m).
"""
import numpy as np
import pytest

from workloads.plummer import plummer


def _loss(orc, pos, vel, m, eps2, ab, kb, pb):
    a, k, p = orc.force(pos, vel, m, eps2)
    return (ab * a).sum() + (kb * k).sum() + (pb * p).sum()


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_dot_product_identity(orc, eps):
    rng = np.random.default_rng(41)
    n = 10
    pos = rng.normal(size=(3, n))
    vel = rng.normal(size=(3, n))
    m = rng.uniform(0.5, 1.5, n) / n
    ab, kb = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    pb = rng.normal(size=n)
    dx, dv, dm = rng.normal(size=(3, n)), rng.normal(size=(3, n)), rng.normal(size=n)
    xb, vb, mb = orc.force_adjoint(pos, vel, m, eps * eps, ab, kb, pb)
    h = 1e-6
    fd = (_loss(orc, pos + h * dx, vel + h * dv, m + h * dm, eps * eps, ab, kb, pb) -
          _loss(orc, pos - h * dx, vel - h * dv, m - h * dm, eps * eps, ab, kb, pb)) / (2 * h)
    adj = (xb * dx).sum() + (vb * dv).sum() + (mb * dm).sum()
    assert abs(fd - adj) <= 1e-7 * abs(adj)


def test_translation_invariance_and_mass_homogeneity(orc):
    pos, vel, m = plummer(128, 42)
    rng = np.random.default_rng(43)
    ab, kb = rng.normal(size=(3, 128)), rng.normal(size=(3, 128))
    pb = rng.normal(size=128)
    eps2 = 1e-3
    xb, vb, mb = orc.force_adjoint(pos, vel, m, eps2, ab, kb, pb)
    assert np.abs(xb.sum(axis=1)).max() < 1e-12 * np.abs(xb).sum()
    assert np.abs(vb.sum(axis=1)).max() < 1e-12 * np.abs(vb).sum()
    L = _loss(orc, pos, vel, m, eps2, ab, kb, pb)
    assert abs((m * mb).sum() - L) < 1e-12 * abs(L)


def test_shared_chain_adjoint_matches_finite_differences(orc):
    # L = 1/2 |x(T) - x*|^2 after 8 shared Hermite steps
    pos, vel, m = plummer(24, 44)
    eps2 = (1 / 64) ** 2
    h, nst = 1.0 / 64, 8
    rng = np.random.default_rng(45)
    target = orc.shared_run(pos, vel, m, eps2, h, nst)[0] + 1e-2 * rng.normal(size=(3, 24))

    def L(p, v, mm):
        x = orc.shared_run(p, v, mm, eps2, h, nst)[0]
        return 0.5 * ((x - target) ** 2).sum()

    xT = orc.shared_run(pos, vel, m, eps2, h, nst)[0]
    gx, gv, gm = orc.shared_chain_adjoint(pos, vel, m, eps2, h, nst, xT - target,
                                          np.zeros_like(xT))
    e = 1e-6
    for (c, i) in [(0, 3), (1, 7), (2, 11), (0, 20)]:
        p1, p2 = pos.copy(), pos.copy()
        p1[c, i] += e
        p2[c, i] -= e
        fd = (L(p1, vel, m) - L(p2, vel, m)) / (2 * e)
        assert abs(fd - gx[c, i]) <= 1e-6 * abs(gx).max()
        v1, v2 = vel.copy(), vel.copy()
        v1[c, i] += e
        v2[c, i] -= e
        fd = (L(pos, v1, m) - L(pos, v2, m)) / (2 * e)
        assert abs(fd - gv[c, i]) <= 1e-6 * abs(gv).max()
    m1, m2 = m.copy(), m.copy()
    m1[5] += e
    m2[5] -= e
    fd = (L(pos, vel, m1) - L(pos, vel, m2)) / (2 * e)
    assert abs(fd - gm[5]) <= 1e-6 * abs(gm).max()
