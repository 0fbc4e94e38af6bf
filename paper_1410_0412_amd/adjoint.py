"""Gradient of an outlet momentum flux with respect to per-node
partial-bounce-back solid fractions, through the hand-written adjoint AA
kernels (``lbm_adjoint_*``) with checkpointed recomputation.

J(ns) = sum_n weight[n] * j_axis(n, T) after T AA steps from the rest state.
The forward pass stores the AA grid every ``every`` steps. The backward pass
walks the segments from last to first: it restores a checkpoint, recomputes
the segment with steps that also store the state each of them reads, and runs
the adjoint step over those states in reverse. Device memory:
ceil(T / every) + every grids, and one more grid while a backward pass runs.

The backward pass uses the solid fraction and weight saved by its own forward
pass, whatever the solver ran in between (another forward pass with other
fractions, for instance). It leaves the solver as it found it: grid, time
step and solid fraction are restored when it returns.
"""

from __future__ import annotations

import torch


class OutletFlux(torch.autograd.Function):
    """``OutletFlux.apply(ns, solver, steps, every, weight, axis)`` -> J (0-dim).

    ``solver`` must be an AA / FP64 / BGK :class:`Solver` created with
    ``pbb=True``; ``ns`` and ``weight`` are device float64 tensors of shape
    (N,) in node order.
    """

    @staticmethod
    def forward(ctx, ns, solver, steps, every, weight, axis=0):
        steps, every = int(steps), int(every)
        if steps < 0 or every < 1:
            raise ValueError("steps >= 0 and every >= 1 required")
        solver.set_solid_fraction(ns.detach())
        solver.init()
        ckpts = []
        for t0 in range(0, steps, every):
            ckpts.append((t0, solver.pdf[0].clone()))
            solver.step(min(every, steps - t0))
        J = solver.weighted_momentum(weight, axis)
        ctx.solver, ctx.steps, ctx.every, ctx.axis = solver, steps, every, axis
        ctx.ckpts = ckpts
        # the fractions this pass ran with (a copy: the caller may change ns)
        ctx.save_for_backward(weight, ns.detach().clone())
        return J

    @staticmethod
    def backward(ctx, gJ):
        weight, ns = ctx.saved_tensors
        s, T, every = ctx.solver, ctx.steps, ctx.every
        # the solver's state when backward starts, restored at the end
        keep_pdf, keep_t, keep_ns = s.pdf[0].clone(), s.t, s.solid_frac[: s.n_fluid].clone()
        s.set_solid_fraction(ns)
        lam = torch.empty_like(s.pdf[0])
        grad = torch.zeros(s.n_fluid, dtype=torch.float64, device=s.device)
        s.adjoint_seed(weight, ctx.axis, T, lam)
        # the recomputed states of one segment; each step writes its f(t)
        states = [torch.empty_like(s.pdf[0]) for _ in range(min(every, T))]
        for t0, ck in reversed(ctx.ckpts):
            t1 = min(t0 + every, T)
            s.pdf[0].copy_(ck)
            s.set_time(t0)
            for t in range(t0, t1):
                s.step_save(states[t - t0])
            for t in range(t1 - 1, t0 - 1, -1):
                s.adjoint_step(states[t - t0], t, lam, grad)
        ctx.ckpts = None
        s.pdf[0].copy_(keep_pdf)
        s.set_time(keep_t)
        s.set_solid_fraction(keep_ns)
        return grad * gJ, None, None, None, None, None


def outlet_flux(ns, solver, steps, every, weight, axis=0):
    """J(ns) as a differentiable function of ``ns`` (see :class:`OutletFlux`)."""
    return OutletFlux.apply(ns, solver, steps, every, weight, axis)
