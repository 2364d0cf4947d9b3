"""Checkpointed adjoint of an RK4 trajectory with probe sampling, as a torch.autograd.Function.

Forward: K RK4 steps of the FR residual from u_0 with the probe pressure sampled before every
step (p_n = p(u_n), n = 0..K-1), keeping the state every `checkpoint_every` steps.  Backward:
segment by segment in reverse, the segment's states and RK stage states are recomputed from its
checkpoint in one fr_rk_step_stages call (on a second stream, overlapping the reverse sweep of
the segment after it), then each step is reversed with fr_rk_step_vjp and the probe
adjoint fr_probe_vjp:  u_bar_n = (du_{n+1}/du_n)^T u_bar_{n+1} + (dp_n/du_n)^T p_bar_n.
All arithmetic runs in the library's kernels; torch provides the tensors and the tape.
"""
from __future__ import annotations

import torch


_SIDE_STREAMS = {}


def _side_stream(dev):
    """One extra stream per device (default priority) for the recompute of checkpoint segments."""
    key = torch.device(dev).index
    if key not in _SIDE_STREAMS:
        _SIDE_STREAMS[key] = torch.cuda.Stream(device=dev)
    return _SIDE_STREAMS[key]


def _record_slots(sol, C, nslot, with_res, dev):
    """Record buffers of the reverse sweep (base states, stage states, stage residuals of C steps),
    kept on the solver and reused by later backward passes of the same segment length."""
    key = (C, nslot, with_res, str(dev))
    cache = sol.__dict__.setdefault("_adjoint_slots", {})
    if key not in cache:
        cache[key] = [{"u": torch.empty(sol.shape, dtype=sol.dtype, device=dev),
                       "states": torch.empty((C,) + sol.shape, dtype=sol.dtype, device=dev),
                       "stages": torch.empty((C, 3) + sol.shape, dtype=sol.dtype, device=dev),
                       "res": torch.empty((C, 4) + sol.shape, dtype=sol.dtype, device=dev) if with_res else None,
                       "pbar": torch.empty((C, sol.n_probe), dtype=torch.float64, device=dev)}
                      for _ in range(nslot)]
    return cache[key]


def _adjoint_accumulators(sol, with_nodes, dev):
    """u_bar (and x_bar) buffers of the reverse sweep, kept on the solver so that the captured
    reverse-segment graphs see the same addresses on every backward pass."""
    key = (with_nodes, str(dev))
    cache = sol.__dict__.setdefault("_adjoint_acc", {})
    if key not in cache:
        cache[key] = (torch.empty(sol.shape, dtype=sol.dtype, device=dev),
                      torch.empty((sol.n_node, sol.dim), dtype=torch.float64, device=dev) if with_nodes else None)
    return cache[key]


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
        with_nodes = bool(ctx.with_nodes and ctx.needs_input_grad[5])
        ub, xb = _adjoint_accumulators(sol, with_nodes, dev)
        ub.zero_()                                                 # dJ/du_K = 0
        if xb is not None:
            xb.zero_()
        # Segments in reverse order.  The recompute of a segment needs only its checkpoint, so it
        # runs on a second stream while the previous (later-in-time) segment is being reversed;
        # two record slots alternate, and a slot is refilled only after the reverse sweep that
        # read it has finished.  At adjoint-workload sizes single kernels leave most of the chip
        # idle, so the two chains overlap; the reverse kernels touch only their own work arrays.
        segs = [(s0, min(s0 + C, K)) for s0 in range(0, K, C)][::-1]
        nslot = min(2, len(segs))
        slots = _record_slots(sol, C, nslot, xb is not None, dev)
        main = torch.cuda.current_stream(dev)
        side = _side_stream(dev) if nslot > 1 else main
        recorded = [torch.cuda.Event() for _ in segs]
        reversed_ = [torch.cuda.Event() for _ in segs]
        if xb is not None:
            sol.geo_adjoint_begin(stream=main)   # metric / normal adjoints of all steps mapped to the nodes once
        side.wait_stream(main)

        def record(i):
            s0, s1 = segs[i]
            sl = slots[i % nslot]
            if i >= nslot:
                side.wait_event(reversed_[i - nslot])
            with torch.cuda.stream(side):
                sl["u"].copy_(ctx.ckpts[s0])
                sol.rk_step_stages(sl["u"], dt, sl["stages"][:s1 - s0], states=sl["states"][:s1 - s0],
                                   residuals=None if sl["res"] is None else sl["res"][:s1 - s0], stream=side)
            recorded[i].record(side)

        for i in range(nslot):
            record(i)
        for i, (s0, s1) in enumerate(segs):
            sl = slots[i % nslot]
            main.wait_event(recorded[i])
            with torch.cuda.stream(main):
                sl["pbar"][:s1 - s0].copy_(p_bar[s0:s1])
            # the segment's steps in reverse, each followed by its probe sample's adjoint (one
            # graph replay per segment)
            sol.rk_segment_vjp(sl["states"], dt, ub, sl["stages"], sl["pbar"], s1 - s0, x_bar=xb,
                               residuals=sl["res"], stream=main)
            reversed_[i].record(main)
            if i + nslot < len(segs):
                record(i + nslot)
        main.wait_stream(side)
        if xb is not None:
            sol.geo_adjoint_end(xb, stream=main)
        return ub.clone(), None, None, None, None, (xb.clone() if xb is not None else None)


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
