"""Receiver traces as a differentiable function of per-voxel lam and mu.

The forward runs the HIP stepper from rest with checkpointing; the backward is the
library's discrete adjoint (``ovfem_adjoint``): the adjoint recursion of the central-
difference scheme stepped backward with the incoming trace gradient injected at the
receivers, checkpoint segments recomputed forward, per-element gradients accumulated
on the GPU.  This module only marshals tensors.

The adjoint reads the checkpoints and the material the solver holds when backward runs,
so a graph is tied to its forward run: backward raises if the solver has been
re-modelled, reset or stepped since (the solver's run generation changed), and lam / mu
are saved so that in-place edits of them after the forward are caught by autograd.
"""
import torch


class _Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, solver, rho, solid, nt, ckpt_every):
        solver.set_model(lam.detach().cpu().numpy(), mu.detach().cpu().numpy(), rho, solid)
        solver.set_dt(solver.dt)
        solver.set_checkpointing(ckpt_every, nt)
        solver.step(nt)
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.save_for_backward(lam, mu)
        return solver.get_traces().clone()

    @staticmethod
    def backward(ctx, grad_traces):
        ctx.saved_tensors  # raises if lam or mu were modified in place since the forward
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError("the solver was re-modelled, reset or stepped after this forward run; its "
                               "checkpoints belong to a later run (run the forward again before backward)")
        g_lam, g_mu = ctx.solver.adjoint(grad_traces.contiguous())
        return g_lam, g_mu, None, None, None, None, None


def traces(solver, lam, mu, rho, solid=None, nt=None, ckpt_every=50):
    """Traces [shot][receiver][3][nt] of a run of nt steps from rest for material (lam, mu).

    lam, mu: CUDA float64 tensors shaped (nz, ny, nx); rho, solid: host arrays.  The
    solver's dt, fixed nodes, sources and receivers must be set (receivers recording
    at least nt steps).  Backward must run before the solver is used for another run.
    ckpt_every = 1 keeps every state ((nt + 2) nodal vectors per shot of device memory) and the
    backward then recomputes nothing; larger intervals trade recompute for memory.
    """
    nt = solver.rec_nt if nt is None else int(nt)
    return _Traces.apply(lam, mu, solver, rho, solid, nt, int(ckpt_every))
