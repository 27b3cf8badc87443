"""torch.autograd.Function wrappers of the hand-written adjoint kernels.

RKRollout(U0, op, n_steps, dt, ckpt_every) advances U0 by n_steps of the
2N-storage Runge-Kutta scheme; its backward pass stores the state every
ckpt_every steps during the forward pass, recomputes each segment's states from
its checkpoint and applies the per-step adjoint (dgns_rk_step_vjp) in reverse.
KineticEnergy(U, op) is K = int |u|^2/2 with gradient dgns_kinetic_energy_vjp.
Both run entirely in the HIP library; torch supplies memory and streams.
"""

import torch


class RKRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, op, n_steps, dt, ckpt_every=10, t0=0.0):
        U = U0.detach().contiguous().clone()
        work = torch.empty(2 * op.n_dof, dtype=torch.float64, device=U.device)
        ckpts = {}
        t = t0
        for s in range(n_steps):
            if s % ckpt_every == 0:
                ckpts[s] = U.clone()
            op.rk_step(U, work, t, dt)
            t += dt
        ctx.op, ctx.n_steps, ctx.dt, ctx.ckpt_every, ctx.t0 = op, n_steps, dt, ckpt_every, t0
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, Ubar):
        op, dt = ctx.op, ctx.dt
        Ub = Ubar.detach().contiguous().clone()
        work = torch.empty(2 * op.n_dof, dtype=torch.float64, device=Ub.device)
        work9 = torch.empty((len(op.rk_scheme()[0]) + 4) * op.n_dof, dtype=torch.float64, device=Ub.device)
        starts = sorted(ctx.ckpts)
        for i in reversed(range(len(starts))):
            s0 = starts[i]
            s1 = starts[i + 1] if i + 1 < len(starts) else ctx.n_steps
            states = [ctx.ckpts[s0].clone()]
            for s in range(s0, s1 - 1):
                U = states[-1].clone()
                op.rk_step(U, work, ctx.t0 + s * dt, dt)
                states.append(U)
            for s in reversed(range(s0, s1)):
                op.rk_step_vjp(states[s - s0], ctx.t0 + s * dt, dt, Ub, out=Ub, work=work9)
        ctx.ckpts = None
        return Ub, None, None, None, None, None


class KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, op):
        Uc = U.detach().contiguous()
        ctx.save_for_backward(Uc)
        ctx.op = op
        return torch.tensor(op.kinetic_energy(Uc), dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.op.kinetic_energy_vjp(U) * g, None


def rk_rollout(U0, op, n_steps, dt, ckpt_every=10, t0=0.0):
    return RKRollout.apply(U0, op, n_steps, dt, ckpt_every, t0)


def kinetic_energy(U, op):
    return KineticEnergy.apply(U, op)
