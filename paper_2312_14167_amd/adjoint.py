"""Checkpointed adjoint of an RK4 trajectory with probe sampling, as a torch.autograd.Function.

Forward: K RK4 steps of the FR residual from u_0 with the probe pressure sampled before every
step (p_n = p(u_n), n = 0..K-1), keeping the state every `checkpoint_every` steps.  Backward:
segment by segment in reverse, the segment's states and RK stage states are recomputed from its
checkpoint in one fr_rk_step_stages call, then each step is reversed with fr_rk_step_vjp and the probe
adjoint fr_probe_vjp:  u_bar_n = (du_{n+1}/du_n)^T u_bar_{n+1} + (dp_n/du_n)^T p_bar_n.
All arithmetic runs in the library's kernels; torch provides the tensors and the tape.
"""
from __future__ import annotations

import torch


class FRTrajectory(torch.autograd.Function):
    """p = FRTrajectory.apply(u0, solver, dt, n_steps, checkpoint_every, nodes)
    -> [n_steps, n_probe] FP64.

    ``nodes``: None, or a float64 CUDA tensor [n_node, dim] equal to the solver's mesh node
    coordinates; when it requires grad, backward also returns dJ/dX through every stage residual
    (metrics and normals) and through the probe location (fixed in physical space)."""

    @staticmethod
    def forward(ctx, u0, solver, dt, n_steps: int, checkpoint_every: int, nodes):
        C = max(1, int(checkpoint_every))
        if solver.n_probe < 1 or solver.max_samples < n_steps:
            raise ValueError("the solver needs probes and max_samples >= n_steps (one sample per step)")
        if nodes is not None:
            ref = torch.as_tensor(solver.node_xyz, dtype=torch.float64)
            if tuple(nodes.shape) != tuple(ref.shape) or not torch.equal(nodes.detach().cpu(), ref):
                raise ValueError("nodes must equal the solver's mesh node coordinates")
        u = u0.detach().clone()
        ckpts = {0: u.clone()}
        solver.reset_accumulators()
        for n in range(n_steps):
            solver.rk_step(u, dt, 1, sample_every=1)
            if (n + 1) % C == 0 and n + 1 < n_steps:
                ckpts[n + 1] = u.clone()
        series = solver.probe_series(n_steps)                    # [n_probe, K]
        ctx.solver, ctx.dt, ctx.K, ctx.C, ctx.ckpts = solver, dt, n_steps, C, ckpts
        ctx.with_nodes = nodes is not None
        return torch.tensor(series.T.copy(), dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, p_bar):
        sol, dt, K, C = ctx.solver, ctx.dt, ctx.K, ctx.C
        p_bar = p_bar.detach().to(torch.float64).contiguous()
        dev = p_bar.device
        ub = torch.zeros(sol.shape, dtype=sol.dtype, device=dev)   # dJ/du_K = 0
        xb = None
        if ctx.with_nodes and ctx.needs_input_grad[5]:
            xb = torch.zeros((sol.n_node, sol.dim), dtype=torch.float64, device=dev)
        states = torch.empty((C,) + sol.shape, dtype=sol.dtype, device=dev)      # reused by every segment
        stages = torch.empty((C, 3) + sol.shape, dtype=sol.dtype, device=dev)
        res = torch.empty((C, 4) + sol.shape, dtype=sol.dtype, device=dev) if xb is not None else None
        if xb is not None:
            sol.geo_adjoint_begin()   # metric / normal adjoints of all steps mapped to the nodes once
        for s0 in reversed(range(0, K, C)):
            s1 = min(s0 + C, K)
            u = ctx.ckpts[s0].clone()
            sol.rk_step_stages(u, dt, stages[:s1 - s0], states=states[:s1 - s0],
                               residuals=None if res is None else res[:s1 - s0])
            for n in reversed(range(s0, s1)):
                sol.rk_step_vjp(states[n - s0], dt, ub, stages[n - s0], x_bar=xb,
                                residuals=None if res is None else res[n - s0])
                sol.probe_vjp(states[n - s0], p_bar[n], ub, x_bar=xb)
        if xb is not None:
            sol.geo_adjoint_end(xb)
        return ub, None, None, None, None, xb


def probe_variance_gradient(solver, u0, dt, n_steps: int, checkpoint_every: int = 20, with_nodes: bool = False):
    """J = sum over probes of (1/K) sum_n (p_n - mean p)^2 (the time-mean square of the probe
    pressure fluctuation), dJ/du0 and (with_nodes) dJ/dX for the mesh node coordinates."""
    u = u0.detach().clone().requires_grad_(True)
    X = None
    if with_nodes:
        X = torch.tensor(solver.node_xyz, dtype=torch.float64, device=u0.device, requires_grad=True)
    p = FRTrajectory.apply(u, solver, dt, n_steps, checkpoint_every, X)
    J = ((p - p.mean(dim=0, keepdim=True)) ** 2).mean(dim=0).sum()
    J.backward()
    return (float(J.detach()), u.grad, X.grad) if with_nodes else (float(J.detach()), u.grad)
