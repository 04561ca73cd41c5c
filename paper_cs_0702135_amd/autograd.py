"""Differentiable shared-step Hermite runs (torch.autograd over the C ABI).

* NBodyForce: forward = nbody_force on the full set; backward = the
  hand-written adjoint nbody_force_adjoint.
* HermiteStep: one shared step h of Section 2 (predict every particle, pair
  sums at the predicted state, correct every particle); backward = the
  corrector transpose, the pair-sum adjoint at the predicted state and the
  predictor transpose (nbody_correct_adjoint, nbody_force_adjoint,
  nbody_predict_adjoint).  Every arithmetic step, forward and backward, runs
  in the library's kernels; this module only allocates and wires tensors.
* shared_run: the same run as one Function over the library's native chain
  (nbody_shared_run / nbody_shared_run_adjoint): the initial force plus
  `steps` shared steps, the state checkpointed every `checkpoint_every`
  steps and each segment recomputed in the backward pass; no Python work
  per step.
* shared_run_steps: the same run composed from HermiteSteps under
  torch.utils.checkpoint (per-step autograd nodes, e.g. for hooks).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

import ctypes

from . import (_mode, _ptr, _sca, _vec, context, correct, correct_adjoint, force,
               force_adjoint, predict, predict_adjoint)


def _zeros_if_none(g, like):
    return torch.zeros_like(like) if g is None else g.contiguous()


class NBodyForce(torch.autograd.Function):
    """(acc, jerk, pot) = pair sums of every particle; differentiable in
    pos, vel and mass."""

    @staticmethod
    def forward(ctx, pos, vel, mass, eps2, mode="fp32"):
        acc, jerk, pot = force(pos, vel, mass, eps2, None, mode)
        ctx.save_for_backward(pos, vel, mass)
        ctx.eps2, ctx.mode = eps2, mode
        return acc, jerk, pot

    @staticmethod
    def backward(ctx, g_acc, g_jerk, g_pot):
        pos, vel, mass = ctx.saved_tensors
        ga = _zeros_if_none(g_acc, pos)
        gk = _zeros_if_none(g_jerk, pos)
        gp = None if g_pot is None else g_pot.contiguous()
        xb, vb, mb = force_adjoint(pos, vel, mass, ctx.eps2, ga, gk, gp, ctx.mode)
        return xb, vb, mb, None, None


class HermiteStep(torch.autograd.Function):
    """(x, v, a, k) at t -> (x, v, a, k) at t + h, every particle advanced."""

    @staticmethod
    def forward(ctx, x, v, a, k, mass, eps2, h, mode="fp32"):
        n = mass.shape[0]
        t = torch.zeros(n, dtype=torch.float64, device=x.device)
        xp, vp = predict(h, t, x, v, a, k)
        a1, k1, _ = force(xp, vp, mass, eps2, None, mode)
        x1 = torch.empty_like(x)
        v1 = torch.empty_like(v)
        a_io = a.clone()
        k_io = k.clone()
        dt = torch.full((n,), float(h), dtype=torch.float64, device=x.device)
        correct(None, xp, vp, a1, k1, 1.0, h, h, t, dt, x1, v1, a_io, k_io, fixed_dt=True)
        ctx.save_for_backward(xp, vp, mass)
        ctx.eps2, ctx.h, ctx.mode = eps2, h, mode
        return x1, v1, a_io, k_io

    @staticmethod
    def backward(ctx, g_x1, g_v1, g_a1, g_k1):
        xp, vp, mass = ctx.saved_tensors
        h = ctx.h
        x1b = _zeros_if_none(g_x1, xp)
        v1b = _zeros_if_none(g_v1, xp)
        a1b = _zeros_if_none(g_a1, xp).clone()
        k1b = _zeros_if_none(g_k1, xp).clone()
        xpb = torch.zeros_like(xp)
        vpb = torch.zeros_like(xp)
        a0b = torch.zeros_like(xp)
        k0b = torch.zeros_like(xp)
        correct_adjoint(h, x1b, v1b, xpb, vpb, a0b, k0b, a1b, k1b)
        mb = torch.zeros_like(mass)
        force_adjoint(xp, vp, mass, ctx.eps2, a1b, k1b, None, ctx.mode, out=(xpb, vpb, mb))
        xb = torch.zeros_like(xp)
        vb = torch.zeros_like(xp)
        predict_adjoint(h, xpb, vpb, xb, vb, a0b, k0b)
        return xb, vb, a0b, k0b, mb, None, None, None


def _segment(x, v, a, k, mass, eps2, h, n_steps, mode):
    for _ in range(n_steps):
        x, v, a, k = HermiteStep.apply(x, v, a, k, mass, eps2, h, mode)
    return x, v, a, k


class SharedRun(torch.autograd.Function):
    """(x, v, a, k) after the initial force and `steps` shared steps of h."""

    @staticmethod
    def forward(ctx, pos, vel, mass, eps2, h, steps, checkpoint_every, mode="fp32"):
        n = mass.shape[0]
        _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
        ck = int(checkpoint_every) if checkpoint_every else max(int(steps), 1)
        x = torch.empty_like(pos)
        v = torch.empty_like(vel)
        a = torch.empty_like(pos)
        k = torch.empty_like(pos)
        keep = any(ctx.needs_input_grad[:3]) and steps > 0
        ckpt = (torch.empty((((steps + ck - 1) // ck) * 12 * n,), dtype=torch.float64,
                            device=pos.device) if keep else None)
        c = context(pos.device)
        c.check(c.lib.nbody_shared_run(c.bind(), n, _ptr(mass), float(eps2), float(h), int(steps),
                                       ck, _ptr(pos), _ptr(vel), _ptr(x), _ptr(v), _ptr(a),
                                       _ptr(k), _ptr(ckpt), _mode(mode)))
        ctx.save_for_backward(pos, vel, mass, ckpt if keep else torch.empty(0))
        ctx.eps2, ctx.h, ctx.steps, ctx.ck, ctx.mode = float(eps2), float(h), int(steps), ck, mode
        return x, v, a, k

    @staticmethod
    def backward(ctx, g_x, g_v, g_a, g_k):
        pos, vel, mass, ckpt = ctx.saved_tensors
        gx = _zeros_if_none(g_x, pos)
        gv = _zeros_if_none(g_v, pos)
        ga = _zeros_if_none(g_a, pos)
        gk = _zeros_if_none(g_k, pos)
        xb = torch.empty_like(pos)
        vb = torch.empty_like(vel)
        mb = torch.empty_like(mass)
        c = context(pos.device)
        c.check(c.lib.nbody_shared_run_adjoint(
            c.bind(), mass.shape[0], _ptr(mass), ctx.eps2, ctx.h, ctx.steps, ctx.ck, _ptr(pos),
            _ptr(vel), _ptr(ckpt) if ckpt.numel() else None, _ptr(gx), _ptr(gv), _ptr(ga),
            _ptr(gk), _ptr(xb), _ptr(vb), _ptr(mb), _mode(ctx.mode)))
        return xb, vb, mb, None, None, None, None, None


def shared_run(pos, vel, mass, eps2, h, steps, checkpoint_every=8, mode="fp32"):
    """Initial force at t = 0, then `steps` shared Hermite steps of h, in the
    library's native chain (checkpoints every `checkpoint_every` steps;
    0 keeps one segment).

    Returns (x, v, a, k) at t = steps * h, differentiable in pos, vel, mass.
    """
    return SharedRun.apply(pos, vel, mass, eps2, h, steps, checkpoint_every, mode)


def shared_run_steps(pos, vel, mass, eps2, h, steps, checkpoint_every=8, mode="fp32"):
    """As shared_run, composed from per-step autograd nodes (HermiteStep)
    recomputed under torch.utils.checkpoint."""
    a, k, _ = NBodyForce.apply(pos, vel, mass, eps2, mode)
    x, v = pos, vel
    done = 0
    while done < steps:
        n_seg = min(checkpoint_every or steps, steps - done)
        if checkpoint_every and torch.is_grad_enabled():
            x, v, a, k = checkpoint(_segment, x, v, a, k, mass, eps2, h, n_seg, mode,
                                    use_reentrant=False)
        else:
            x, v, a, k = _segment(x, v, a, k, mass, eps2, h, n_seg, mode)
        done += n_seg
    return x, v, a, k
