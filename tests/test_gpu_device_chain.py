"""The device-counted entry points chained without host reads.

nbody_schedule -> nbody_predict_dev -> nbody_force_dev -> nbody_correct_dev
(Section 2: select the block, predict every particle, pair sums of the
block, correct the block) reads the block time and size from device memory.
From the same initialised state, K such chained steps must equal K steps of
the device-resident driver (nbody_blockstep) bitwise: the same predictor,
the same launch shapes of the pair kernels and the same corrector.  Sizes on
both sides of the driver's single-workgroup threshold (2048) and of the
small-block kernel's (8192).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import plummer

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["fp32", "ds"])
@pytest.mark.parametrize("n", [1500, 3001, 20011])
def test_chained_device_steps_equal_the_driver(n, mode):
    need_gpu()
    import torch

    import paper_cs_0702135_amd as nb
    nb.tune_clear()
    pos, vel, m = plummer(n, 4000 + n)
    eps2 = (1 / 512) ** 2
    drv = nb.System(dev(pos), dev(vel), dev(m), eps2, mode=mode)
    t, dt = drv.t.clone(), drv.dt.clone()
    x, v, a, k = drv.x.clone(), drv.v.clone(), drv.a.clone(), drv.k.clone()
    K = 12
    for step in range(K):
        act, n_i, tn = nb.schedule_async(t, dt)
        xp, vp = nb.predict_dev(tn, t, x, v, a, k)
        an, kn, _ = nb.force_dev(xp, vp, drv.m, eps2, act, n_i, n, mode)
        nb.correct_dev(act, n_i, n, xp, vp, an, kn, drv.eta, drv.dt_max, drv.dt_min, t, dt, x,
                       v, a, k)
    torch.cuda.synchronize()
    assert drv.step(K) == K
    for name, got, ref in (("t", t, drv.t), ("dt", dt, drv.dt), ("x", x, drv.x), ("v", v, drv.v),
                           ("a", a, drv.a), ("k", k, drv.k)):
        np.testing.assert_array_equal(host(got), host(ref), err_msg=name)
    say("n=%d %s: %d chained device steps equal the driver's bitwise (t = %.6g)"
        % (n, mode, K, float(host(t).max())))


def test_device_block_size_above_capacity_is_reported():
    # a device block size beyond the stated capacity is clamped (no write
    # past the outputs) and reported as an index error at the next sync
    need_gpu()
    import torch

    import paper_cs_0702135_amd as nb
    n = 300
    pos, vel, m = plummer(n, 5)
    P, V, M = dev(pos), dev(vel), dev(m)
    act = torch.arange(n, dtype=torch.int32, device=P.device)
    n_i = torch.tensor([n], dtype=torch.int64, device=P.device)
    acc, jerk, _ = nb.force_dev(P, V, M, 1e-4, act, n_i, 100)
    ref = nb.force(P, V, M, 1e-4, act[:100].contiguous())
    torch.cuda.synchronize()
    np.testing.assert_allclose(host(acc), host(ref[0]), rtol=1e-6, atol=0)
    t = torch.zeros(n, dtype=torch.float64, device=P.device)
    dt = torch.full((n,), 1.0 / 64, dtype=torch.float64, device=P.device)
    a, k = torch.zeros_like(P), torch.zeros_like(P)
    x, v = P.clone(), V.clone()
    nb.correct_dev(act, n_i, 100, P, V, acc, jerk, 0.02, 0.125, 2.0 ** -40, t, dt, x, v, a, k)
    with pytest.raises(nb.NBodyError):
        nb.context(P.device).sync_status()
