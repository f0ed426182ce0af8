"""torch.autograd front end of the discrete adjoint.

Forward and backward of every Function below are single C-ABI calls
(mfc_rhs / mfc_rhs_vjp, mfc_step / mfc_step_vjp, the conversions and their
adjoints); torch only chains them.  FP64 contexts only.

`rollout_objective` is the adjoint problem of the shock-cylinder physics:
J = sum_{n=1..N} dt * sum_j p(q^n)_{j, nx-1} * dy (time-integrated pressure in
the last interior column, next to the right wall), with a frozen dt and
checkpoints every `every` steps; its backward recomputes each segment from its
checkpoint and runs the step adjoints in reverse, injecting dJ/dq^n.
"""
from __future__ import annotations

import torch

from .solver import Solver


class RHS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, solver: Solver):
        ctx.solver = solver
        ctx.save_for_backward(q)
        return solver.rhs(q.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        return ctx.solver.rhs_vjp(q, g.contiguous()), None


class Step(torch.autograd.Function):
    """One SSP-RK3 step with a fixed dt (out of place)."""

    @staticmethod
    def forward(ctx, q, solver: Solver, dt: float):
        ctx.solver, ctx.dt = solver, float(dt)
        ctx.save_for_backward(q)
        out = q.detach().clone().contiguous()
        solver.step(out, dt_fixed=dt)
        return out

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        return ctx.solver.step_vjp(q, ctx.dt, g.contiguous()), None, None


class PrimToCons(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, solver: Solver):
        ctx.solver = solver
        ctx.save_for_backward(w)
        return solver.prim_to_cons(w.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        (w,) = ctx.saved_tensors
        return ctx.solver.prim_to_cons_vjp(w, g.contiguous()), None


class ConsToPrim(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, solver: Solver):
        ctx.solver = solver
        ctx.save_for_backward(q)
        return solver.cons_to_prim(q.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        return ctx.solver.cons_to_prim_vjp(q, g.contiguous()), None


def _wall_weights(solver: Solver, column: int, scale: float):
    """dJ_n/dw: `scale` on the pressure row of one x-column, zero elsewhere."""
    wb = torch.zeros(solver.shape, dtype=torch.float64, device=solver.device)
    wb[solver.num_fluids + solver.ndim, :, :, column] = scale
    return wb


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q0, solver: Solver, nsteps: int, dt: float, every: int, column: int):
        q = q0.detach().clone().contiguous()
        dy = solver.dx[1] if solver.ndim > 1 else 1.0
        dz = solver.dx[2] if solver.ndim > 2 else 1.0
        prow = solver.num_fluids + solver.ndim
        checkpoints = {0: q.clone()}
        J = torch.zeros((), dtype=torch.float64, device=solver.device)
        for n in range(1, nsteps + 1):
            solver.step(q, dt_fixed=dt)
            w = solver.cons_to_prim(q)
            J = J + dt * dy * dz * w[prow, :, :, column].sum()
            if n % every == 0 and n < nsteps:
                checkpoints[n] = q.clone()
        ctx.solver, ctx.nsteps, ctx.dt, ctx.every, ctx.column = solver, nsteps, float(dt), every, column
        ctx.checkpoints = checkpoints
        ctx.scale = dt * dy * dz
        return J

    @staticmethod
    def backward(ctx, gJ):
        S = ctx.solver
        g = float(gJ)
        wb = _wall_weights(S, ctx.column, ctx.scale * g)
        qbar = torch.zeros(S.shape, dtype=torch.float64, device=S.device)
        starts = sorted(ctx.checkpoints)
        for seg_start in reversed(starts):
            seg_end = min(seg_start + ctx.every, ctx.nsteps)
            # replay the segment once, keeping every step's input and stage states
            states, stages = [ctx.checkpoints[seg_start]], []
            for _ in range(seg_start, seg_end):
                nxt = states[-1].clone()
                q1, q2 = torch.empty_like(nxt), torch.empty_like(nxt)
                S.step_save_stages(nxt, ctx.dt, q1, q2)
                states.append(nxt)
                stages.append((q1, q2))
            for n in range(seg_end, seg_start, -1):
                # inject dJ/dq^n, then pull through step n-1 -> n
                k = n - seg_start
                S.cons_to_prim_vjp(states[k], wb, out=qbar, accumulate=True)
                q1, q2 = stages[k - 1]
                qbar = S.step_vjp_stages(states[k - 1], q1, q2, ctx.dt, qbar)
        return qbar, None, None, None, None, None


def rollout_objective(q0, solver: Solver, nsteps: int, dt: float, every: int = 20, column: int = -1):
    """Time-integrated pressure of one x-column (default: the last, at the right wall)."""
    if column < 0:
        column = solver.n[0] + column
    return _Rollout.apply(q0, solver, nsteps, dt, every, column)
