"""nbody_force_noalloc (pair sums with static scratch, no allocation)
against nbody_force, through the C ABI.

Two calls in a row on one device, the second with a smaller input: an
active subset of 3000 particles of N = 50000, then every particle of
N = 20000 (both share the static array; the second must not see the
first's records or partial sums).  A third call at the size limit,
n_j = NBODY_NOALLOC_MAX_NJ, with a 2048-particle active subset.  Each is
compared per particle with nbody_force on the same inputs: the j split can
differ (it is capped so that the partials fit next to the records), so the
float32 mode agrees to the float32 sums' accuracy (relative 1e-6 per
particle; both are within ~1e-7 of the float64 oracle) and the compensated
mode (float64 pair terms) to 1e-12.  Outputs are preallocated, so the
binding allocates nothing either.  A size above the limit is rejected on
the host with NBODY_E_INVAL.
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, rel_vec_err, say
from workloads.plummer import plummer, random_active_set

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-6, "ds": 1e-12}


def _compare(n, n_i, seed, mode, eps2=(1 / 1024) ** 2):
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = plummer(n, seed)
    P, V, M = dev(pos), dev(vel), dev(m)
    A = None if n_i == n else dev(random_active_set(n, n_i, seed + 1), torch.int32)
    out = (torch.empty((3, n_i), dtype=torch.float64, device=P.device),
           torch.empty((3, n_i), dtype=torch.float64, device=P.device),
           torch.empty((n_i,), dtype=torch.float64, device=P.device))
    torch.cuda.synchronize()
    say("no-alloc: n=%d n_i=%d mode=%s" % (n, n_i, mode))
    ga, gk, gp = nb.force_noalloc(P, V, M, eps2, A, mode, out=out)
    ra, rk, rp = nb.force(P, V, M, eps2, A, mode)
    ga, gk, gp, ra, rk, rp = map(host, (ga, gk, gp, ra, rk, rp))
    ea, ek = rel_vec_err(ga, ra), rel_vec_err(gk, rk)
    ep = np.abs(gp - rp) / np.abs(rp)
    say("no-alloc n=%d n_i=%d %s: acc max %.2e jerk max %.2e pot max %.2e"
        % (n, n_i, mode, ea.max(), ek.max(), ep.max()))
    assert np.isfinite(ga).all() and np.isfinite(gk).all() and np.isfinite(gp).all()
    assert ea.max() <= TOL[mode] and ep.max() <= TOL[mode]
    assert ek.max() <= 10 * TOL[mode]


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_noalloc_two_calls_second_smaller(mode):
    need_gpu()
    _compare(50000, 3000, 21, mode)
    _compare(20000, 20000, 22, mode)


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_noalloc_at_the_size_limit(mode):
    need_gpu()
    import paper_cs_0702135_amd._lib as L
    _compare(L.NBODY_NOALLOC_MAX_NJ, 2048, 23, mode, eps2=(1 / 4096) ** 2)


def test_noalloc_rejects_sizes_above_the_limit():
    need_gpu()
    import paper_cs_0702135_amd as nb
    import paper_cs_0702135_amd._lib as L
    n = L.NBODY_NOALLOC_MAX_NJ + 1
    pos, vel, m = np.zeros((3, n)), np.zeros((3, n)), np.full(n, 1.0 / n)
    with pytest.raises(nb.NBodyError) as e:
        nb.force_noalloc(dev(pos), dev(vel), dev(m), 1e-6)
    assert e.value.code == L.NBODY_E_INVAL
    say("no-alloc limit: %s" % e.value)
