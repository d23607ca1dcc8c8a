"""torch.autograd wrappers around the HIP rollout and its hand-written adjoint.

``rollout`` advances a batch by n_steps (forward: ``orchard_step`` with checkpoints
every ``ckpt_every`` steps; backward: ``orchard_step_backward``, which recomputes each
checkpoint segment and runs the adjoint kernels with every discrete switch of the
forward frozen).  Differentiable inputs: per-joint stiffness kp and damping kd, the
per-step apple forces, and the continuous initial state.  ``tips`` returns segment tip
positions with their adjoint.
"""
from __future__ import annotations

import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, state, n_steps, ckpt_every, kp, kd, aforce, q0, qd0, ax0, av0):
        n_ck = -(-n_steps // ckpt_every)
        ckpt = torch.empty(n_ck * model.ckpt_words, dtype=torch.float32, device=kp.device)
        state.q.copy_(q0)
        state.qd.copy_(qd0)
        state.apple[0:3].copy_(ax0)
        state.apple[3:6].copy_(av0)
        af = aforce.contiguous() if aforce is not None else None
        model.step(state, kp.contiguous(), kd.contiguous(), n_steps, aforce=af, ckpt=ckpt, ckpt_every=ckpt_every)
        ctx.model, ctx.n_steps, ctx.ckpt_every = model, n_steps, ckpt_every
        ctx.has_force = aforce is not None
        ctx.save_for_backward(kp, kd, af if af is not None else torch.empty(0, device=kp.device), ckpt)
        return state.q.clone(), state.qd.clone(), state.apple[0:3].clone(), state.apple[3:6].clone()

    @staticmethod
    def backward(ctx, gq, gqd, gax, gav):
        kp, kd, af, ckpt = ctx.saved_tensors
        m = ctx.model
        z = lambda t, shape: (t.contiguous().clone() if t is not None else torch.zeros(shape, device=kp.device))
        adj = dict(q=z(gq, (m.n_seg, 2)), qd=z(gqd, (m.n_seg, 2)), ax=z(gax, (3, m.n_apple)), av=z(gav, (3, m.n_apple)))
        gkp = torch.zeros_like(kp)
        gkd = torch.zeros_like(kd)
        gF = torch.zeros_like(af) if ctx.has_force else None
        m.step_backward(ckpt, ctx.ckpt_every, ctx.n_steps, kp.contiguous(), kd.contiguous(), adj, gkp, gkd, gF,
                        aforce=af if ctx.has_force else None)
        return (None, None, None, None, gkp, gkd, gF, adj["q"], adj["qd"], adj["ax"], adj["av"])


def rollout(model, state, kp, kd, n_steps: int, ckpt_every: int, aforce=None, q0=None, qd0=None, ax0=None, av0=None):
    """Differentiable rollout.  ``state`` supplies the discrete part of the initial state
    (flags, counters, step counter) and receives the final state; the continuous initial
    state defaults to the one in ``state``.  Returns (q, qd, apple_x, apple_v) after the
    rollout.  aforce: [n_steps, n_apple, 3] (internal order) or None."""
    q0 = state.q.clone() if q0 is None else q0
    qd0 = state.qd.clone() if qd0 is None else qd0
    ax0 = state.apple[0:3].clone() if ax0 is None else ax0
    av0 = state.apple[3:6].clone() if av0 is None else av0
    return _Rollout.apply(model, state, n_steps, ckpt_every, kp, kd, aforce, q0, qd0, ax0, av0)


class _Tips(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, node, q):
        q = q.contiguous()
        ctx.model = model
        ctx.save_for_backward(node, q)
        return model.tips(q, node)

    @staticmethod
    def backward(ctx, gout):
        node, q = ctx.saved_tensors
        gq = torch.zeros_like(q)
        ctx.model.tips_backward(q, node, gout.contiguous(), gq)
        return None, None, gq


def tips(model, q, node):
    """Tip positions p_b + R_b (0, 0, l_b) of internal segments ``node`` (int32 tensor)."""
    return _Tips.apply(model, node, q)
