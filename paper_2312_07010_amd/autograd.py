"""torch.autograd binding of the library's checkpointed reverse sweep.

ACEStep.apply(phi0, eps2, solver, nsteps, ckpt_every) runs nsteps steps of
the scheme from phi0 (a CUDA float64 tensor) with interface width
sqrt(eps2) and returns phi^T.  Its backward calls the library's transposed
step (ace_backward): checkpoints every ckpt_every steps are kept on the GPU
during the forward, each segment is recomputed in the reverse sweep, and the
gradients with respect to phi0 and eps2 come back in one pass.  All work runs
on torch's current stream.

One solver handle holds the checkpoints of one forward pass.  When a graph
holds several passes on the same handle (two terms of one loss, or a pass
with another eps2), a later forward replaces the checkpoints of an earlier
one; the earlier node's backward sees that from the handle's checkpoint
generation and first repeats its own forward from its saved phi0 and eps2.
"""
import torch

from . import ace as _ace


def _forward(solver, phi0, e2, nsteps, ckpt_every):
    solver.use_torch_stream()
    solver.set_eps(e2 ** 0.5)
    solver.forward_ckpt(phi0, int(nsteps), int(ckpt_every))
    return solver.ckpt_generation


class ACEStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, eps2, solver, nsteps, ckpt_every):
        if not (phi0.is_cuda and phi0.dtype == torch.float64):
            raise ValueError("phi0 must be a CUDA float64 tensor")
        e2 = float(eps2.detach().item()) if torch.is_tensor(eps2) else float(eps2)
        if not e2 > 0.0:
            raise ValueError("eps2 must be positive")
        p0 = phi0.detach().contiguous()
        gen = _forward(solver, p0, e2, nsteps, ckpt_every)
        out = torch.empty_like(phi0)
        solver.get_phi(out)
        ctx.solver = solver
        ctx.gen = gen
        ctx.e2 = e2
        ctx.nsteps = int(nsteps)
        ctx.ckpt_every = int(ckpt_every)
        ctx.save_for_backward(p0)
        ctx.eps2_is_tensor = torch.is_tensor(eps2)
        ctx.eps2_like = eps2 if torch.is_tensor(eps2) else None
        return out

    @staticmethod
    def backward(ctx, grad_out):
        solver = ctx.solver
        (p0,) = ctx.saved_tensors
        solver.use_torch_stream()
        if solver.ckpt_generation != ctx.gen:
            # another forward on this handle replaced the checkpoints
            ctx.gen = _forward(solver, p0, ctx.e2, ctx.nsteps, ctx.ckpt_every)
        g0 = torch.empty_like(grad_out)
        try:
            _, geps2 = solver.backward(grad_out.contiguous(), g0)
        except _ace.AceError as e:
            if e.code != _ace.ACE_E_STATE:
                raise
            # the field or eps changed since the forward: repeat it
            ctx.gen = _forward(solver, p0, ctx.e2, ctx.nsteps, ctx.ckpt_every)
            _, geps2 = solver.backward(grad_out.contiguous(), g0)
        ge = None
        if ctx.eps2_is_tensor:
            ge = torch.tensor(geps2, dtype=ctx.eps2_like.dtype, device=ctx.eps2_like.device)
        return g0, ge, None, None, None


def ace_evolve(phi0, eps2, solver, nsteps, ckpt_every=32):
    """phi^T after nsteps steps, differentiable in phi0 and eps2."""
    return ACEStep.apply(phi0, eps2, solver, nsteps, ckpt_every)
