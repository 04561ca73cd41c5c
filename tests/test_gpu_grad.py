"""GPU adjoint and differentiable-run checks against the FP64 oracle.

* nbody_force_adjoint vs the oracle's adjoint (itself pinned on the CPU by
  the dot-product identity against finite differences).
* The checkpointed shared-step run's gradient (autograd through
  HermiteStep / NBodyForce) vs the oracle's float64 chain adjoint on every
  coordinate, and vs central finite differences of the oracle's forward run.
* The full differentiable-run workload (N = 16384, eps = 1/512, 64 steps of
  1/512, checkpoints every 8 steps) vs the stored float64 finite differences
  of tests/golden/grad16k_fd.json on 32 coordinates.
Gates (float32 pair arithmetic forward and backward): median per-coordinate
relative error <= 1e-4 and maximum <= 1e-3 (reading; the target states no
tolerance for gradients).
"""
import json
import os

import numpy as np
import pytest

from tests.gpu_util import dev, host, need_gpu, say
from workloads.plummer import CONFIGS, plummer

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "grad16k_fd.json")


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_force_adjoint_matches_oracle(orc, mode):
    need_gpu()
    import paper_cs_0702135_amd as nb
    n = 1500
    pos, vel, m = plummer(n, 61)
    rng = np.random.default_rng(62)
    ab, kb, pb = rng.normal(size=(3, n)), rng.normal(size=(3, n)), rng.normal(size=n)
    eps2 = (1 / 256) ** 2
    xb, vb, mb = nb.force_adjoint(dev(pos), dev(vel), dev(m), eps2, dev(ab), dev(kb), dev(pb),
                                  mode)
    rx, rv, rm = orc.force_adjoint(pos, vel, m, eps2, ab, kb, pb)
    for got, ref, name in ((host(xb), rx, "pos"), (host(vb), rv, "vel"), (host(mb), rm, "mass")):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        gl = np.sqrt(((got - ref) ** 2).sum() / (ref ** 2).sum())
        say("adjoint %s %s: max err / max |ref| %.2e, global %.2e" % (mode, name, err, gl))
        assert err < 1e-5 and gl < 1e-5


def test_force_adjoint_accumulates():
    need_gpu()
    import paper_cs_0702135_amd as nb
    import torch
    n = 300
    pos, vel, m = plummer(n, 63)
    rng = np.random.default_rng(64)
    ab, kb = dev(rng.normal(size=(3, n))), dev(rng.normal(size=(3, n)))
    P, V, M = dev(pos), dev(vel), dev(m)
    x1, v1, m1 = nb.force_adjoint(P, V, M, 1e-4, ab, kb)
    base = (torch.ones_like(x1), torch.ones_like(v1), torch.ones_like(m1))
    x2, v2, m2 = nb.force_adjoint(P, V, M, 1e-4, ab, kb, out=base)
    assert torch.equal(x2, x1 + 1) and torch.equal(v2, v1 + 1) and torch.equal(m2, m1 + 1)


def _loss_grad_gpu(pos, vel, m, eps2, h, steps, target, ckpt, mode="ds"):
    import torch
    from paper_cs_0702135_amd.autograd import shared_run
    P = dev(pos).requires_grad_(True)
    V = dev(vel).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    x, v, a, k = shared_run(P, V, M, eps2, h, steps, checkpoint_every=ckpt, mode=mode)
    loss = ((x - dev(target)) ** 2).sum() / m.shape[0]
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), host(P.grad), host(V.grad), host(M.grad), host(x.detach())


def test_shared_run_gradient_matches_oracle_adjoint(orc):
    need_gpu()
    n, h, steps = 1024, 1.0 / 512, 16
    pos, vel, m = plummer(n, 65)
    eps2 = (1 / 256) ** 2
    xT = orc.shared_run(pos, vel, m, eps2, h, steps)[0]
    target = xT + 1e-3 * np.random.default_rng(66).normal(size=xT.shape)
    L, gx, gv, gm, x_gpu = _loss_grad_gpu(pos, vel, m, eps2, h, steps, target, 8)
    assert np.abs(x_gpu - xT).max() < 1e-8  # forward agrees with the float64 run
    rx, rv, rm = orc.shared_chain_adjoint(pos, vel, m, eps2, h, steps, 2 * (xT - target) / n,
                                          np.zeros_like(xT))
    for got, ref, name in ((gx, rx, "x0"), (gv, rv, "v0"), (gm, rm, "m")):
        rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        gl = np.sqrt(((got - ref) ** 2).sum() / (ref ** 2).sum())
        say("grad %s: median rel %.2e, max rel %.2e, global %.2e" % (name, np.median(rel),
                                                                     rel.max(), gl))
        assert np.median(rel) <= 1e-4 and rel.max() <= 1e-3


def test_checkpointing_does_not_change_the_gradient():
    need_gpu()
    n, h, steps = 512, 1.0 / 512, 12
    pos, vel, m = plummer(n, 67)
    target = pos + 0.01
    eps2 = 1e-4
    g1 = _loss_grad_gpu(pos, vel, m, eps2, h, steps, target, 4)
    g2 = _loss_grad_gpu(pos, vel, m, eps2, h, steps, target, 0)
    for a, b in zip(g1[1:4], g2[1:4]):
        np.testing.assert_array_equal(a, b)


def test_full_run_gradient_vs_stored_finite_differences(orc):
    # N = 16384, eps = 1/512, 64 shared steps of 1/512, checkpoints every 8
    need_gpu()
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/grad16k_fd.json not generated")
    cfg = CONFIGS["grad16k"]
    ex = cfg.extra
    gold = json.load(open(GOLDEN))
    pos, vel, m = plummer(cfg.n, cfg.seed)
    xT = orc.shared_run(pos, vel, m, cfg.eps2, ex["dt"], ex["steps"])[0]
    xi = np.random.default_rng(ex["target_seed"]).normal(size=xT.shape)
    target = xT + ex["target_sigma"] * xi
    L, gx, gv, gm, _ = _loss_grad_gpu(pos, vel, m, cfg.eps2, ex["dt"], ex["steps"], target,
                                      ex["ckpt"])
    rel = []
    for c in gold["coords"]:
        fd = c["fd"]
        g = gx[c["axis"], c["particle"]]
        rel.append(abs(g - fd) / abs(fd))
        if "fd_half" in c:  # the finite differences themselves are stable
            assert abs(c["fd_half"] - fd) <= 1e-5 * abs(fd)
    rel = np.array(rel)
    say("grad16k: %d coordinates, median rel err %.2e, max %.2e" % (rel.size, np.median(rel),
                                                                   rel.max()))
    assert np.median(rel) <= 1e-4 and rel.max() <= 1e-3


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_native_chain_matches_per_step_autograd(mode):
    # the native chain runs the same entry points as the per-step autograd
    # composition: identical forward state, gradients equal up to the order
    # in which the mass cotangents of the steps are added
    need_gpu()
    import torch
    from paper_cs_0702135_amd.autograd import shared_run, shared_run_steps
    n, h, steps = 600, 1.0 / 256, 11
    pos, vel, m = plummer(n, 69)
    eps2 = 1e-4
    rng = np.random.default_rng(70)
    wx, wv, wa = (dev(rng.normal(size=(3, n))) for _ in range(3))
    res = []
    for fn in (shared_run, shared_run_steps):
        P = dev(pos).requires_grad_(True)
        V = dev(vel).requires_grad_(True)
        M = dev(m).requires_grad_(True)
        x, v, a, k = fn(P, V, M, eps2, h, steps, checkpoint_every=4, mode=mode)
        loss = (wx * x).sum() + (wv * v).sum() + (wa * a).sum()
        loss.backward()
        torch.cuda.synchronize()
        res.append((host(x.detach()), host(P.grad), host(V.grad), host(M.grad)))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    for got, ref in zip(res[0][1:], res[1][1:]):
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("mode", ["fp32", "ds"])
def test_differentiable_run_forward_force_accuracy(orc, mode):
    # Forward pair sums of the differentiable run (Plummer N = 16384,
    # eps = 1/512, shared steps of 1/512): the acceleration and jerk left by
    # step 8 are the pair sums at the state predicted from the state after
    # step 7 (the corrector stores them), checked against the oracle's pair
    # sums at that predicted state.  Gates: float32 mode acceleration p99
    # <= 1e-6 and max <= 1e-5, jerk p99 <= 1e-5 and max <= 1e-4;
    # compensated mode (float64 pair terms) p99 <= 1e-12 and max <= 1e-10.
    need_gpu()
    from paper_cs_0702135_amd.autograd import shared_run
    cfg = CONFIGS["grad16k"]
    pos, vel, m = plummer(cfg.n, cfg.seed)
    h = cfg.extra["dt"]
    P, V, M = dev(pos), dev(vel), dev(m)
    x7, v7, a7, k7 = (host(q) for q in shared_run(P, V, M, cfg.eps2, h, 7, 0, mode))
    x8, v8, a8, k8 = (host(q) for q in shared_run(P, V, M, cfg.eps2, h, 8, 0, mode))
    t = np.zeros(cfg.n)
    xp, vp = orc.predict(h, t, x7, v7, a7, k7)
    ra, rk, _ = orc.force(xp, vp, m, cfg.eps2)
    ea = np.linalg.norm(a8 - ra, axis=0) / np.linalg.norm(ra, axis=0)
    ek = np.linalg.norm(k8 - rk, axis=0) / np.linalg.norm(rk, axis=0)
    say("differentiable run %s, step 8: acc p50 %.2e p99 %.2e max %.2e | jerk p50 %.2e p99 %.2e "
        "max %.2e" % (mode, np.median(ea), np.percentile(ea, 99), ea.max(), np.median(ek),
                      np.percentile(ek, 99), ek.max()))
    gates = {"fp32": (1e-6, 1e-5, 1e-5, 1e-4), "ds": (1e-12, 1e-10, 1e-12, 1e-10)}[mode]
    assert np.percentile(ea, 99) <= gates[0] and ea.max() <= gates[1]
    assert np.percentile(ek, 99) <= gates[2] and ek.max() <= gates[3]
