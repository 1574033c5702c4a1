"""torch.autograd binding of the MPA reverse pass.

``propagate(plan, field, z0, z1, sigma, beta2, beta3)`` marches `field`
(complex CUDA tensor of the plan's precision) from z0 to z1 with the plan and
is differentiable with respect to the field and, optionally, the per-span
coefficients sigma, beta2 and beta3 of the plan's map.  The forward keeps one
checkpoint per map period (mpa_propagate_checkpointed); the backward runs
mpa_adjoint, which recomputes each period from its checkpoint.  The map
coefficients are baked into the plan's tables, so the tensors passed must
hold the plan's values; their gradients are returned as FP64.

`plan` may also be an MPABatchPlan: `field` is then the instances'
concatenated fields, and the coefficient gradients are those of the map the
instances share (each instance's sigma is the map's times its scale).
"""
from __future__ import annotations

import torch


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field, sigma, beta2, beta3, plan, z0, z1, store_steps):
        out = field.detach().contiguous().clone()
        ckpt = plan.propagate_checkpointed(out, z0, z1)
        ctx.plan, ctx.z0, ctx.z1, ctx.store_steps = plan, z0, z1, store_steps
        ctx.param_devices = [None if t is None else (t.device, t.dtype) for t in (sigma, beta2, beta3)]
        ctx.save_for_backward(ckpt)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (ckpt,) = ctx.saved_tensors
        grad = grad_out.detach().contiguous().clone()
        pg = ctx.plan.adjoint(ckpt, grad, ctx.z0, ctx.z1, ctx.store_steps)
        outs = []
        for q, spec in enumerate(ctx.param_devices):
            outs.append(None if spec is None else pg[q].to(device=spec[0], dtype=spec[1]))
        return (grad, *outs, None, None, None, None)


def propagate(plan, field, z0, z1, sigma=None, beta2=None, beta3=None, store_steps=0):
    """Differentiable mpa_propagate (see the module docstring)."""
    for q, t in enumerate((sigma, beta2, beta3)):
        if t is None:
            continue
        want = plan.coefficients[q]
        got = tuple(float(v) for v in t.detach().cpu().reshape(-1).tolist())
        if got != want:
            raise ValueError(f"coefficient tensor {('sigma', 'beta2', 'beta3')[q]} = {got} differs from the "
                             f"plan's map {want}; build a plan for these values")
    return _Propagate.apply(field, sigma, beta2, beta3, plan, float(z0), float(z1), int(store_steps))
