"""Smallest-first float32 pair sums on the GPU (Section 6), against the oracle.

nbody_force_sorted evaluates each pair term in float64, rounds it once to
float32, orders a particle's terms by the float64 pair-acceleration
magnitude (ties by j) and adds them in float32 in that order.  The oracle's
force_sum32(order="sorted") does the same arithmetic on the CPU with
correctly rounded float64 operations and no contraction; the kernel's
float64 division and square root are correctly rounded too and it is
compiled without contraction, so both sides take the same keys, the same
order and the same float32 additions: the bar is bitwise equality.

Accuracy is then placed against the float64 oracle next to the GPU's
float32 and compensated modes and the oracle's index-order float32 sum, on
the N = 1024 Plummer workload and on ensemble-sized clusters.
"""
import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, rel_vec_err, say
from workloads.plummer import CONFIGS, ensemble_members, plummer, random_active_set

pytestmark = pytest.mark.gpu


def _sorted_gpu(pos, vel, m, eps2, act=None):
    import paper_cs_0702135_amd as nb
    import torch
    A = None if act is None else dev(act, torch.int32)
    a, k, p = nb.force_sorted(dev(pos), dev(vel), dev(m), eps2, A)
    torch.cuda.synchronize()
    return host(a), host(k), host(p)


@pytest.mark.parametrize("n,n_i,seed", [
    (1, None, 11), (2, None, 12), (3, None, 13), (255, None, 14), (257, None, 15),
    (1024, None, 1001), (1000, 37, 16), (4097, 300, 17), (8192, 256, 18)])
def test_sorted_bitwise_vs_oracle(orc, n, n_i, seed):
    need_gpu()
    pos, vel, m = plummer(n, seed)
    eps2 = (1.0 / 256) ** 2
    act = None if n_i is None else random_active_set(n, n_i, seed + 7)
    say("sorted parity n=%d n_i=%s seed=%d" % (n, n_i, seed))
    a, k, p = _sorted_gpu(pos, vel, m, eps2, act)
    ra, rk, rp = orc.force_sum32(pos, vel, m, eps2, active=act, order="sorted")
    assert np.array_equal(a, ra)
    assert np.array_equal(k, rk)
    assert np.array_equal(p, rp)


def test_sorted_unequal_masses_and_ties(orc):
    """Unequal and negative masses (|m| in the key) and exact key ties (a
    lattice, where many pairs share one distance): the order of equal keys
    is fixed by j on both sides."""
    need_gpu()
    rng = np.random.default_rng(21)
    g = np.arange(8, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()]) * 0.125
    n = pos.shape[1]
    vel = rng.standard_normal((3, n)) * 0.1
    m = np.full(n, 1.0 / n)
    a, k, p = _sorted_gpu(pos, vel, m, 1e-4)
    ra, rk, rp = orc.force_sum32(pos, vel, m, 1e-4, order="sorted")
    assert np.array_equal(a, ra) and np.array_equal(k, rk) and np.array_equal(p, rp)
    m2 = rng.uniform(-1.0, 2.0, n) / n
    a, k, p = _sorted_gpu(pos, vel, m2, 1e-4)
    ra, rk, rp = orc.force_sum32(pos, vel, m2, 1e-4, order="sorted")
    assert np.array_equal(a, ra) and np.array_equal(k, rk) and np.array_equal(p, rp)


def test_sorted_out_of_range_index_is_reported():
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = plummer(300, 9)
    bad = torch.tensor([5, 300, 8], dtype=torch.int32, device="cuda")
    nb.force_sorted(dev(pos), dev(vel), dev(m), 1e-4, bad)
    with pytest.raises(nb.NBodyError):
        nb.context().sync_status()
    nb.context().sync_status()  # cleared once reported


def test_sorted_rejects_large_n():
    need_gpu()
    import paper_cs_0702135_amd as nb
    pos, vel, m = plummer(8193, 5)
    with pytest.raises(nb.NBodyError):
        nb.force_sorted(dev(pos), dev(vel), dev(m), 1e-4)


def _members():
    sizes, eps, seeds = ensemble_members()
    order = np.argsort(sizes)
    picks = [order[0], order[len(order) // 2], order[-1]]
    return [(int(sizes[q]), float(eps[q]), int(seeds[q])) for q in picks]


@pytest.mark.parametrize("label,n,eps,seed", [("plummer1k", 1024, 1.0 / 256, 1001)] +
                         [("ensemble", n, e, s) for n, e, s in _members()])
def test_sorted_accuracy_and_cost(orc, label, n, eps, seed):
    """Acceleration and jerk errors against the float64 oracle at the median
    and 99th percentile for: GPU smallest-first float32, GPU float32 mode,
    GPU compensated mode, oracle index-order float32.  Gates: the GPU
    compensated mode is the most accurate, and smallest-first is no worse
    than index order at the 99th percentile."""
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    pos, vel, m = plummer(n, seed)
    eps2 = eps * eps
    ra, rk, _ = orc.force(pos, vel, m, eps2)
    P, V, M = dev(pos), dev(vel), dev(m)
    res, cost = {}, {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    out, cost["GPU sorted"] = timed(lambda: nb.force_sorted(P, V, M, eps2))
    res["GPU sorted"] = (host(out[0]), host(out[1]))
    for mode in ("fp32", "ds"):
        out, cost["GPU " + mode] = timed(lambda: nb.force(P, V, M, eps2, None, mode))
        res["GPU " + mode] = (host(out[0]), host(out[1]))
    a, k, _ = orc.force_sum32(pos, vel, m, eps2, order="index")
    res["oracle float32 index"] = (a, k)
    stats = {}
    for key, (a, k) in res.items():
        ea, ek = rel_vec_err(a, ra), rel_vec_err(k, rk)
        stats[key] = (np.median(ea), np.percentile(ea, 99), np.median(ek),
                      np.percentile(ek, 99))
        say("%s N=%d %-21s acc med %.2e p99 %.2e  jerk med %.2e p99 %.2e  %s" % (
            label, n, key, *stats[key],
            ("%.3f ms/call" % cost[key]) if key in cost else ""))
    assert stats["GPU ds"][1] < min(v[1] for q, v in stats.items() if q != "GPU ds")
    assert stats["GPU sorted"][1] <= stats["oracle float32 index"][1]
