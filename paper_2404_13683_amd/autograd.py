"""Receiver traces as a differentiable function of per-voxel lam and mu.

The forward runs the HIP stepper from rest with checkpointing; the backward is the
library's discrete adjoint (``ovfem_adjoint``): the adjoint recursion of the central-
difference scheme stepped backward with the incoming trace gradient injected at the
receivers, checkpoint segments recomputed forward, per-element gradients accumulated
on the GPU.  This module only marshals tensors.
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
        return solver.get_traces().clone()

    @staticmethod
    def backward(ctx, grad_traces):
        g_lam, g_mu = ctx.solver.adjoint(grad_traces.contiguous())
        return g_lam, g_mu, None, None, None, None, None


def traces(solver, lam, mu, rho, solid=None, nt=None, ckpt_every=50):
    """Traces [shot][receiver][3][nt] of a run of nt steps from rest for material (lam, mu).

    lam, mu: CUDA float64 tensors shaped (nz, ny, nx); rho, solid: host arrays.  The
    solver's dt, fixed nodes, sources and receivers must be set (receivers recording
    at least nt steps).
    """
    nt = solver.rec_nt if nt is None else int(nt)
    return _Traces.apply(lam, mu, solver, rho, solid, nt, int(ckpt_every))
