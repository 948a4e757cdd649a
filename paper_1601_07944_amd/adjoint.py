"""Reverse-mode differentiation of many SSP-RK3 steps through the library's
hand-written adjoint kernels (dg_rk_step_vjp), with checkpointing.

Forward: N steps with a fixed step length (the step length is held fixed and
not differentiated), keeping the state every `every` steps.  Backward: for
each segment, last to first, recompute its steps from the checkpoint while
keeping their input and stage states (dg_rk_step_stages_to, which writes each
step's result to a new state), then chain the step adjoints backwards.  Memory: N/every checkpoints plus 3*every states for one segment.

every = 0 keeps every step's input and stage states from the forward pass
itself (3N states, e.g. 192 GB for 50 steps of the 4,000,000-triangle mesh
at p = 3): the backward pass then runs the step adjoints alone, with no
recomputation.  Its steps are the out-of-place ones of the recomputation
(dg_rk_step_stages_to), so its C_N equals dg_rk_step's to rounding.
choose_every() picks that when the states fit in the free device memory.
All arithmetic runs in libdgmi's kernels; torch provides memory and streams.
"""
from __future__ import annotations

import torch

from . import binding as B


class RKSteps(torch.autograd.Function):
    """C_N = step^N(C_0) on the internal layout; differentiable in C_0."""

    @staticmethod
    def forward(ctx, C0, dm, dt: float, nsteps: int, every: int = 20):
        if every < 0:
            raise ValueError("every must be >= 0 (0: keep every step's stage states)")
        ctx.dm = dm
        ctx.dt = float(dt)
        ctx.nsteps = nsteps
        ctx.every = every
        if every == 0:
            C, ctx.tape = forward_keep_all(dm, C0.detach().clone(), dt, nsteps)
            ctx.ckpts = None
            return C
        C = C0.detach().clone()
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(C.clone())
            dm.rk_step(C, dt)
        ctx.ckpts = ckpts
        ctx.tape = None
        return C

    @staticmethod
    def backward(ctx, gout):
        if ctx.every == 0:
            tape, ctx.tape = ctx.tape, None
            g = backward_tape(ctx.dm, tape, ctx.dt, gout.contiguous())
        else:
            g = backward_sweep(ctx.dm, ctx.ckpts, ctx.dt, ctx.nsteps, ctx.every, gout.contiguous())
        return g, None, None, None, None


def forward_keep_all(dm, C, dt, nsteps):
    """nsteps SSP-RK3 steps from C (which becomes the first step's input and
    must not be modified afterwards), each step's input and stage states kept:
    returns (C_N, tape), tape[n] = (C_n, u1_n, u2_n)."""
    tape = []
    for _ in range(nsteps):
        u1, u2, Cnext = dm.empty_state(), dm.empty_state(), dm.empty_state()
        dm.rk_step_stages_to(C, Cnext, u1, u2, dt)
        tape.append((C, u1, u2))
        C = Cnext
    return C, tape


def backward_tape(dm, tape, dt, gout):
    """Cotangent of C_0 from that of C_N over the kept states of
    forward_keep_all, last step first; each step's states are released
    once its adjoint has run (the list is emptied)."""
    g = gout.clone()
    while tape:
        Cn, u1, u2 = tape.pop()
        g = dm.rk_step_vjp(Cn, g, dt, u1=u1, u2=u2)
        del Cn, u1, u2
    return g


def choose_every(dm, nsteps, every=20, margin=1.10):
    """0 (keep every step's stage states, no recomputation) if the 3 nsteps
    states, times margin, fit in the device's free memory (the caching
    allocator's unused blocks included), else every."""
    import torch

    free, _ = torch.cuda.mem_get_info(dm.device)
    free += torch.cuda.memory_reserved(dm.device) - torch.cuda.memory_allocated(dm.device)
    need = 3 * nsteps * dm.info.state_len * 8
    return 0 if need * margin <= free else every


def backward_sweep(dm, ckpts, dt, nsteps, every, gout):
    """Cotangent of C_0 from the cotangent of C_N (see module docstring)."""
    g = gout.clone()
    nseg = len(ckpts)
    for seg in range(nseg - 1, -1, -1):
        start = seg * every
        end = min(start + every, nsteps)
        # every step's input state is kept: each recomputed step writes its
        # result into a new state instead of over its input (no copies)
        C = ckpts[seg]
        saved = []
        for _ in range(start, end):
            u1 = dm.empty_state()
            u2 = dm.empty_state()
            Cnext = dm.empty_state()
            dm.rk_step_stages_to(C, Cnext, u1, u2, dt)
            saved.append((C, u1, u2))
            C = Cnext
        del C
        for Cn, u1, u2 in reversed(saved):
            g = dm.rk_step_vjp(Cn, g, dt, u1=u1, u2=u2)
    return g


def run_steps(C0, dm, dt, nsteps, every=20):
    """Differentiable wrapper: returns C_N (every: the checkpoint interval,
    0 to keep every step's stage states, None for choose_every's pick)."""
    if every is None:
        every = choose_every(dm, nsteps)
    return RKSteps.apply(C0, dm, dt, nsteps, every)


def pressure_disk_objective(dm, C, centre=(0.5, 0.5), radius=0.1, gamma=1.4):
    """J = sum_i det J_i sum_k w_k 1[|x_ik - centre| < radius] p(U_h(x_ik))
    over the volume quadrature points (the mask is fixed, so J is smooth in
    C), and dJ/dC in the internal layout.

    dJ/dc_ij = sum_k w_ik mask_ik dp/dU(U_ik) phi_j(r_k), which is
    dg_project applied to det J_i mask_ik dp/dU(U_ik) (dg_project computes
    sum_k w_k phi_j u_k with the reference weights w_k = w_ik / det J_i)."""
    u = dm.eval_points(C)  # [N, nq, 4] user order
    w = dm.quad_weights()  # [N, nq]
    xy = dm.quad_points()
    mask = (((xy[..., 0] - centre[0]) ** 2 + (xy[..., 1] - centre[1]) ** 2) < radius**2).to(u.dtype)
    rho, mx, my, E = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
    g1 = gamma - 1.0
    p = g1 * (E - 0.5 * (mx * mx + my * my) / rho)
    J = torch.sum(w * mask * p)
    dp = torch.stack([g1 * 0.5 * (mx * mx + my * my) / rho**2, -g1 * mx / rho, -g1 * my / rho, g1 * torch.ones_like(rho)],
                     dim=-1)
    det = 2.0 * w.sum(dim=1)  # the reference weights sum to 1/2
    arg = (det[:, None, None] * mask[..., None] * dp).contiguous()
    return J, dm.project(arg)


__all__ = ["RKSteps", "backward_sweep", "run_steps", "pressure_disk_objective", "B"]
