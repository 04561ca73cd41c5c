"""Edge cases of the GPU path, each against the oracle or a closed form.

* eps2 = 0 (legal for distinct positions, the self pair excluded by index):
  a circular Kepler binary through the pair kernel (closed form), the
  block-step driver and the ensemble (its masked self-pair path), the last
  two against the oracle's run of the same binary.
* Ragged and degenerate sizes: one particle (no pairs: zero sums), an empty
  active set, active sets that end inside a tile.
* Errors reported, not trapped: an active index out of range (status word,
  raised at the next synchronisation), a non-finite state in the block-step
  driver, a bad ensemble description (rejected on the host).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import plummer

pytestmark = pytest.mark.gpu


def _binary(d=1.0, m1=0.5, m2=0.5):
    # circular orbit of separation d about the centre of mass, in the x-y plane
    mt = m1 + m2
    om = np.sqrt(mt / d ** 3)
    r1, r2 = d * m2 / mt, d * m1 / mt
    pos = np.array([[r1, -r2], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [om * r1, -om * r2], [0.0, 0.0]])
    return pos, vel, np.array([m1, m2]), om


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_kepler_binary_force_eps0(mode):
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m, om = _binary(0.75, 0.3, 0.7)
    a, k, p = (host(q) for q in nb.force(dev(pos), dev(vel), dev(m), 0.0, None, mode))
    # a_i = -om^2 r_i, k_i = -om^2 v_i, phi_i = -m_other / d
    np.testing.assert_allclose(a, -om ** 2 * pos, rtol=2e-6, atol=1e-12)
    np.testing.assert_allclose(k, -om ** 2 * vel, rtol=2e-6, atol=1e-12)
    np.testing.assert_allclose(p, [-0.7 / 0.75, -0.3 / 0.75], rtol=2e-6)


def test_kepler_binary_blockstep_and_ensemble_eps0(orc):
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m, om = _binary()
    t_end, dt_max = 0.5, 0.125
    s = orc.init_state(pos, vel, m, 0.0, dt_max=dt_max)
    r_steps, _ = orc.integrate(s, t_end)
    sysg = nb.System(dev(pos), dev(vel), dev(m), 0.0, dt_max=dt_max)
    g_steps = sysg.run(t_end)
    # closed-form phase: the binary turns by om * t
    ang = np.arctan2(host(sysg.x)[1, 0], host(sysg.x)[0, 0])
    say("Kepler eps=0: steps GPU %d oracle %d, phase error %.2e"
        % (g_steps, r_steps, abs(ang - om * t_end)))
    assert abs(g_steps - r_steps) <= 1
    assert np.abs(host(sysg.x) - s.x).max() < 5e-8
    assert abs(ang - om * t_end) < 1e-6
    # the same binary as one ensemble cluster (plus a softened Plummer one)
    p2, v2, m2 = plummer(100, 7)
    P = np.concatenate([pos, p2], axis=1)
    V = np.concatenate([vel, v2], axis=1)
    M = np.concatenate([m, m2])
    off = np.array([0, 2, 102], dtype=np.int64)
    out = nb.ensemble_run(dev(P), dev(V), dev(M), off, np.array([0.0, 1e-4]), t_end,
                          dt_max=dt_max)
    assert abs(out["steps"][0] - r_steps) <= 1
    assert np.abs(host(out["x"])[:, :2] - s.x).max() < 5e-8


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_masked_self_pair_eps0_both_modes(orc, mode):
    # eps = 0: the self pair must be masked by index (s = 0 otherwise), in
    # the driver's pair kernels and in the ensemble's float32 and float64
    # pair bodies; the compensated mode follows the float64 oracle closely
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m, om = _binary()
    t_end, dt_max = 0.5, 0.125
    s = orc.init_state(pos, vel, m, 0.0, dt_max=dt_max)
    r_steps, _ = orc.integrate(s, t_end)
    tol = {"fp32": 5e-8, "ds": 1e-11}[mode]
    sysg = nb.System(dev(pos), dev(vel), dev(m), 0.0, dt_max=dt_max, mode=mode)
    g_steps = sysg.run(t_end)
    dx_drv = np.abs(host(sysg.x) - s.x).max()
    p2, v2, m2 = plummer(100, 7)
    P = np.concatenate([pos, p2], axis=1)
    V = np.concatenate([vel, v2], axis=1)
    M = np.concatenate([m, m2])
    off = np.array([0, 2, 102], dtype=np.int64)
    out = nb.ensemble_run(dev(P), dev(V), dev(M), off, np.array([0.0, 1e-4]), t_end,
                          dt_max=dt_max, mode=mode)
    dx_ens = np.abs(host(out["x"])[:, :2] - s.x).max()
    say("eps=0 binary %s: steps driver %d ensemble %d oracle %d, |dx| driver %.2e ensemble %.2e"
        % (mode, g_steps, out["steps"][0], r_steps, dx_drv, dx_ens))
    assert abs(g_steps - r_steps) <= 1 and abs(out["steps"][0] - r_steps) <= 1
    assert dx_drv < tol and dx_ens < tol


def test_single_particle_and_empty_active_set():
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = (np.array([[0.1], [0.2], [0.3]]), np.array([[1.0], [0.0], [0.0]]),
                   np.array([1.0]))
    a, k, p = nb.force(dev(pos), dev(vel), dev(m), 1e-4)
    assert torch.count_nonzero(a) == 0 and torch.count_nonzero(k) == 0
    assert torch.count_nonzero(p) == 0
    pos, vel, m = plummer(100, 3)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    a, k, p = nb.force(dev(pos), dev(vel), dev(m), 1e-4, empty)
    assert a.shape == (3, 0) and p.shape == (0,)


@pytest.mark.parametrize("n_i", [1, 63, 65, 127, 129, 255, 257])
def test_ragged_active_sets(orc, n_i):
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = plummer(1000, 8)
    act = np.sort(np.random.default_rng(n_i).choice(1000, n_i, replace=False)).astype(np.int32)
    a, k, p = nb.force(dev(pos), dev(vel), dev(m), 1e-4, dev(act, torch.int32))
    ra, rk, rp = orc.force(pos, vel, m, 1e-4, active=act)
    err = np.linalg.norm(host(a) - ra, axis=0) / np.linalg.norm(ra, axis=0)
    assert err.max() < 1e-5


def test_out_of_range_index_is_reported():
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = plummer(200, 4)
    bad = torch.tensor([3, 200, 7], dtype=torch.int32, device="cuda")
    nb.force(dev(pos), dev(vel), dev(m), 1e-4, bad)
    with pytest.raises(nb.NBodyError):
        nb.context().sync_status()
    nb.context().sync_status()  # the status word is cleared once reported


def test_nonfinite_state_is_reported():
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m = plummer(256, 5)
    # a NaN velocity: every initial step is non-finite, reported by the
    # initialisation (which synchronises) before any step is taken
    bad = vel.copy()
    bad[0, 17] = np.nan
    with pytest.raises(nb.NBodyError):
        nb.System(dev(pos), dev(bad), dev(m), 1e-4)
    # a NaN injected into a valid state: one block step, then reported
    sysg = nb.System(dev(pos), dev(vel), dev(m), 1e-4)
    sysg.x[0, 17] = float("nan")
    with pytest.raises(nb.NBodyError):
        sysg.step(1)


def test_bad_ensemble_description_rejected():
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m = plummer(100, 6)
    # offsets that do not end at n: rejected by the binding
    with pytest.raises(ValueError):
        nb.ensemble_run(dev(pos), dev(vel), dev(m), np.array([0, 60, 50], dtype=np.int64),
                        np.array([1e-4, 1e-4]), 0.0625)
    # an empty cluster and a negative eps2: rejected by the library on the host
    for off, e2 in (([0, 60, 60, 100], [1e-4, 1e-4, 1e-4]), ([0, 60, 100], [1e-4, -1.0])):
        with pytest.raises(nb.NBodyError):
            nb.ensemble_run(dev(pos), dev(vel), dev(m), np.array(off, dtype=np.int64),
                            np.array(e2), 0.0625)
