"""torch.autograd.Function over the hand-written adjoint of libswiftcl.

ClFunction.apply(plan, inputs, pk, bias, nz, D_z) -> C [B, max_ell, npairs]
with gradients for pk [B, n_k], bias [B, T], nz [B, T, n_zs] and D_z [B, n_zg] (float64
tensors).  `inputs` supplies the remaining device inputs (tracer and multipole counts,
kinds, chi(z), Omega_m); the four differentiable tensors replace their entries.  Both
directions run in the library's HIP kernels; torch provides memory and the stream.
"""
from __future__ import annotations

import torch


class ClFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, inputs, pk, bias, nz, D_z):
        t = dict(inputs)
        t.update(pk=pk.detach().contiguous(), bias=bias.detach().contiguous(), nz=nz.detach().contiguous(),
                 D_z=D_z.detach().contiguous())
        C = plan.cl(t)
        ctx.plan = plan
        ctx.t = t
        ctx.token = plan.state_token
        # torch checks at backward time that none of these was modified in place since
        ctx.save_for_backward(pk, bias, nz, D_z)
        return C

    @staticmethod
    def backward(ctx, dC):
        want = [name for name, need in zip(("pk", "bias", "nz", "D"), ctx.needs_input_grad[2:]) if need]
        if not want:
            return None, None, None, None, None, None
        ctx.saved_tensors  # raises if an input was modified in place after the forward call
        # no other forward on this plan since ours: its assembly and FFTLog state are still ours
        reuse = ctx.plan.state_token is ctx.token
        g = ctx.plan.backward(ctx.t, dC.to(ctx.plan.out_dtype).contiguous(), want=tuple(want), reuse_forward=reuse)
        return None, None, g.get("pk"), g.get("bias"), g.get("nz"), g.get("D")


def cl(plan, inputs, pk, bias, nz, D_z):
    """Differentiable C_l (see ClFunction)."""
    return ClFunction.apply(plan, inputs, pk, bias, nz, D_z)


class ClLimberFunction(torch.autograd.Function):
    """The Limber limit (swiftcl_cl_limber) with its hand-written adjoint
    (swiftcl_cl_limber_backward); same arguments and gradients as ClFunction."""

    @staticmethod
    def forward(ctx, plan, inputs, pk, bias, nz, D_z):
        t = dict(inputs)
        t.update(pk=pk.detach().contiguous(), bias=bias.detach().contiguous(), nz=nz.detach().contiguous(),
                 D_z=D_z.detach().contiguous())
        C = plan.cl_limber(t)
        ctx.plan = plan
        ctx.t = t
        ctx.save_for_backward(pk, bias, nz, D_z)
        return C

    @staticmethod
    def backward(ctx, dC):
        want = [name for name, need in zip(("pk", "bias", "nz", "D"), ctx.needs_input_grad[2:]) if need]
        if not want:
            return None, None, None, None, None, None
        ctx.saved_tensors
        g = ctx.plan.limber_backward(ctx.t, dC.to(ctx.plan.out_dtype).contiguous(), want=tuple(want))
        return None, None, g.get("pk"), g.get("bias"), g.get("nz"), g.get("D")


def cl_limber(plan, inputs, pk, bias, nz, D_z):
    """Differentiable Limber C_l (see ClLimberFunction)."""
    return ClLimberFunction.apply(plan, inputs, pk, bias, nz, D_z)


class ClKgrowthFunction(torch.autograd.Function):
    """Scale-dependent growth (swiftcl_cl_kgrowth) with its hand-written adjoint
    (swiftcl_cl_kgrowth_backward): gradients for pk [B, n_k] and bias [B, T]; D_kz [B, n_interp,
    n_zg] is an input without gradient."""

    @staticmethod
    def forward(ctx, plan, inputs, D_kz, pk, bias):
        t = dict(inputs)
        t.update(pk=pk.detach().contiguous(), bias=bias.detach().contiguous())
        D = D_kz.detach().contiguous()
        C = plan.cl_kgrowth(t, D)
        ctx.plan = plan
        ctx.t = t
        ctx.D = D
        ctx.save_for_backward(pk, bias, C)
        return C

    @staticmethod
    def backward(ctx, dC):
        if ctx.needs_input_grad[2]:
            raise RuntimeError("the scale-dependent growth adjoint has no gradient with respect to D(k, z)")
        want = [name for name, need in zip(("pk", "bias"), ctx.needs_input_grad[3:]) if need]
        if not want:
            return None, None, None, None, None
        _, _, C = ctx.saved_tensors
        g = ctx.plan.kgrowth_backward(ctx.t, ctx.D, C, dC.to(ctx.plan.out_dtype).contiguous(), want=tuple(want))
        return None, None, None, g.get("pk"), g.get("bias")


def cl_kgrowth(plan, inputs, D_kz, pk, bias):
    """Differentiable C_l with scale-dependent growth (see ClKgrowthFunction)."""
    return ClKgrowthFunction.apply(plan, inputs, D_kz, pk, bias)
