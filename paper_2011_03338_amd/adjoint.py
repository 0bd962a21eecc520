"""Reverse-mode differentiation of an SSP-RK3 evolution through the library's
adjoint kernels, as a torch.autograd.Function.

The differentiated map is the frozen one: the blending factors, squeezing
parameters and step sizes of every stage are those of the forward evolution
(the paper gives the forward scheme only).  Memory is bounded by checkpointing:
the forward keeps the state at the start of every segment of `every` steps;
the backward replays one segment at a time from its checkpoint with the logged
step sizes, recording a tape per step (the three stage states with their
blending factors, squeezing parameters, face states, means and scales,
bit-identical to the forward since the same kernels run on the same inputs),
then walks the segment backwards with the transposed RK3 step.  Peak extra memory: one checkpoint per segment plus
`every` tapes.

Every arithmetic step runs in the library (sedg_rk_step, sedg_rk_step_tape,
sedg_adjoint_rk_step, and sedg_rk_step_frozen for the frozen forward map); this
module only sequences the calls.
"""
from __future__ import annotations

import torch

from . import sedg


def _segment_dt(solver, every, device):
    # one step-size buffer per forward call keeps the library's captured step graph
    # (keyed by the state and log buffers) the same for every segment
    return torch.zeros(every, dtype=torch.float64, device=device)


class RK3Evolve(torch.autograd.Function):
    """u_T = `nsteps` SSP-RK3 steps of u0 with CFL step sizes (state layout of
    sedg_state_len, float64 on the GPU)."""

    @staticmethod
    def forward(ctx, u0, solver: sedg.Solver, nsteps: int, every: int = 20):
        if nsteps < 0 or every < 1:
            raise ValueError("nsteps >= 0 and every >= 1 required")
        u = u0.detach().contiguous().clone()
        dt_log = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=u.device)
        seg_dt = _segment_dt(solver, every, u.device)
        checkpoints = []
        s = 0
        while s < nsteps:
            checkpoints.append(u.clone())
            m = min(every, nsteps - s)
            solver.rk_step(u, m, 0.0, seg_dt)
            dt_log[s:s + m].copy_(seg_dt[:m])
            s += m
        solver.check()
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        ctx.checkpoints, ctx.dt_log = checkpoints, dt_log
        return u

    @staticmethod
    def backward(ctx, grad_out):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.every
        lam = grad_out.detach().contiguous().clone()
        if nsteps == 0:
            return lam, None, None, None
        tapes = torch.empty((min(every, nsteps), solver.tape_len), dtype=torch.float64, device=lam.device)
        for seg in reversed(range(len(ctx.checkpoints))):
            s0 = seg * every
            m = min(every, nsteps - s0)
            u = ctx.checkpoints[seg].clone()
            solver.rk_step_tape(u, ctx.dt_log[s0:s0 + m], tapes)
            solver.adjoint_rk_step(tapes, ctx.dt_log[s0:s0 + m], lam)
        solver.check()
        return lam, None, None, None


def evolve(u0: torch.Tensor, solver: sedg.Solver, nsteps: int, every: int = 20) -> torch.Tensor:
    """Differentiable evolution: torch.autograd sees the adjoint of the frozen map."""
    return RK3Evolve.apply(u0, solver, nsteps, every)


def dt_log_of(u_out: torch.Tensor) -> torch.Tensor:
    """The step sizes used by the evolution that produced u_out."""
    return u_out.grad_fn.dt_log


def record_frozen(solver: sedg.Solver, u0: torch.Tensor, dt_log: torch.Tensor) -> torch.Tensor:
    """Replay the evolution from u0 with the logged step sizes and return, per step,
    the factor block of its tape, [alpha x 3 | beta x 3] (nsteps x 6 x alpha_len)."""
    ns, na = solver.state_len, solver.alpha_len
    u = u0.detach().contiguous().clone()
    tape = torch.empty(solver.tape_len, dtype=torch.float64, device=u.device)
    out = torch.empty((dt_log.numel(), 6, na), dtype=torch.float64, device=u.device)
    for j in range(dt_log.numel()):
        solver.rk_step_tape(u, dt_log[j:j + 1], tape)
        out[j].copy_(tape[3 * ns:3 * ns + 6 * na].view(6, na))
    solver.check()
    return out


def frozen_evolve(solver: sedg.Solver, u0: torch.Tensor, frozen: torch.Tensor, dt_log: torch.Tensor) -> torch.Tensor:
    """The frozen forward map (sedg_rk_step_frozen): SSP-RK3 with every stage's factors
    held at `frozen` (from record_frozen) and the logged step sizes; no autograd."""
    u = u0.detach().contiguous().clone()
    solver.rk_step_frozen(u, dt_log.contiguous(), frozen.contiguous())
    return u
