"""Seeded test cases shared by the parity tests: each returns the mesh, degree, flow, equation
set and an initial state evaluated at the ORACLE's solution-point coordinates (inputs never
come from the HIP path)."""
from __future__ import annotations

import numpy as np
import torch

import fr_inputs as fi


def rel_l2(a: torch.Tensor, b: torch.Tensor) -> float:
    """max over variables of ||a_v - b_v||_2 / ||b_v||_2 over all solution points (state layout
    [Ne][nv][Ns])."""
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    num = ((a - b) ** 2).sum(dim=(0, 2)).sqrt()
    den = (b ** 2).sum(dim=(0, 2)).sqrt().clamp_min(1e-300)
    return float((num / den).max())


def make_case(name: str):
    """(mesh, p, flow, equations, init_fn(x) -> conserved [.., nv], dt, probes)"""
    if name == "euler_vortex":
        m = fi.periodic_box(2, 8, q=1)
        return m, 3, fi.vortex_params(), "euler", lambda x: fi.vortex_state(x), np.array([2.12e-3 * 4]), [[0.3, 1.7]]
    if name == "euler_farfield_curved":
        m = fi.periodic_box(2, 5, q=3, curv=0.2, bc="farfield", seed=4)
        fp = fi.freestream_params(2, 0.3, None, aoa_deg=15.0)
        return m, 4, fp, "euler", _noisy(fp, 21, 0.02), np.array([2e-3]), [[0.4, -0.6]]
    if name == "ns_periodic_curved":
        m = fi.periodic_box(2, 5, q=2, curv=0.2, seed=7)
        fp = fi.freestream_params(2, 0.2, 200.0, aoa_deg=10.0)
        return m, 4, fp, "ns", _noisy(fp, 5, 0.02), np.array([1e-3]), [[1.1, -0.2]]
    if name == "ns_ogrid":
        m = fi.o_grid(24, 8, q=4, r1=6.0, stretch=1.2, seed=3)
        fp = fi.freestream_params(2, 0.2, 1000.0)
        return m, 4, fp, "ns", _noisy(fp, 6, 1e-2), np.array([2e-4]), [[0.0, 3.0]]
    if name == "ns_channel_p3":
        m = fi.periodic_box(2, (6, 4), q=2, curv=0.15, bc="channel", seed=8)
        fp = fi.freestream_params(2, 0.3, 100.0)
        return m, 3, fp, "ns", _noisy(fp, 9, 0.03), np.array([1e-3]), [[0.2, 0.3]]
    if name == "ns_box3d_p2":
        m = fi.periodic_box(3, 3, q=2, curv=0.2, seed=2)
        fp = fi.freestream_params(3, 0.2, 100.0, aoa_deg=20.0)
        return m, 2, fp, "ns", _noisy(fp, 10, 0.02), np.array([2e-3]), [[0.3, 0.2, -1.0]]
    if name == "ns_cgrid_p4":
        m = fi.c_grid_naca(n_wake=3, n_foil=8, n_normal=3, n_span=2, q=2, camber=0.02, r_out=4.0, x_out=6.0,
                           h_wall=0.05)
        fp = fi.freestream_params(3, 0.2, 23000.0, aoa_deg=4.0)
        return m, 4, fp, "ns", _noisy(fp, 11, 1e-2), np.array([5e-5]), [[1.0, -2.0, 0.1]]
    if name == "ns_cavity_batch":
        ms = [fi.cavity(1.5, h=0.5, q=2, upstream=2.0, top=3.0, outflow=3.0, top_buffer=1.0, out_buffer=1.0),
              fi.cavity(2.5, h=0.5, q=2, upstream=2.0, top=3.0, outflow=3.0, top_buffer=1.0, out_buffer=1.0)]
        m = fi.concat_meshes(ms)
        fp = fi.freestream_params(2, 0.15, 1500.0, n_mesh=2)
        fp.vel_inf[1] = [0.9, 0.1]
        fp.p_inf[1] *= 1.01
        return m, 3, fp, "ns", _noisy(fp, 12, 1e-2, mesh=m), np.array([1e-3, 7e-4]), [[0.5, 1.2], [0.5, 0.8]]
    raise KeyError(name)


def _noisy(fp, seed, amp, mesh=None):
    def f(x):
        u = fi.freestream_state(x, fp, 0)
        if mesh is not None:  # per-mesh free stream over element ranges (x is [Ne, Ns, d])
            for k in range(mesh.n_mesh):
                lo, hi = mesh.mesh_elem_begin[k], mesh.mesh_elem_begin[k + 1]
                u[lo:hi] = fi.freestream_state(x[lo:hi], fp, k)
        n = fi.noise_like(u.shape, seed, amp)
        u = u.copy()
        u[..., 1:-1] += n[..., 1:-1]
        u[..., 0] *= 1.0 + 0.1 * n[..., 0]
        return u
    return f


def oracle_for(name: str, with_probes=True):
    from oracle import OracleSystem
    m, p, fp, eq, init, dt, probes = make_case(name)
    pm = None
    if m.n_mesh > 1:
        pm = list(range(len(probes)))
    s = OracleSystem(m, p, fp, equations=eq, probes=probes if with_probes else None, probe_mesh=pm)
    x = s.solpt_coords()
    u0 = torch.tensor(init(x)).permute(0, 2, 1).contiguous()
    return s, m, p, fp, eq, u0, dt, probes, pm
