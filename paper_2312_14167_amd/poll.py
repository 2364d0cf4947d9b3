"""Batched evaluation of one MADS poll of the airfoil problem: every candidate design (maximum
camber, its chordwise position, thickness, angle of attack) gets its own extruded C-grid, the
meshes are concatenated into one batched solver (one launch per kernel for all candidates), all
candidates advance together, and each candidate's OASPL at its observer, mean lift and drag
coefficients (Eq. (8), computed by the library) and penalised objective are computed from the
FP64 probe series and wall force.
"""
from __future__ import annotations

import numpy as np
import torch

import fr_inputs as fi

from .mads import naca_objective
from .solver import Solver


def naca_candidate_mesh(x, grid: dict):
    """C-grid around the NACA 4-digit section of design x = (camber %, camber position in tenths,
    thickness %, angle of attack in degrees)."""
    camber, pos, thick, _ = (float(v) for v in x)
    return fi.c_grid_naca(camber=camber / 100.0, camber_pos=pos / 10.0, thickness=thick / 100.0, **grid)


def naca_poll(designs, grid: dict, p: int, steps: int, dt: float, mach: float = 0.2, reynolds: float = 23000.0,
              probe=(1.0, -2.0), p_ref_pa: float = 2e-5, precision: str = "fp32", cl_base=None, cd_base=None,
              span: float | None = None, sample_every: int = 1, device="cuda"):
    """Evaluate all designs together.  Returns per design: OASPL (dB, 20 log10(p_RMS / p_ref)
    with p_ref mapped by p_inf <-> 101325 Pa), mean C_L, C_D (force on the walls over
    1/2 rho U^2 chord span, lift normal to the free stream) and, with baselines, the penalised
    objective."""
    designs = np.atleast_2d(np.asarray(designs, float))
    meshes = [naca_candidate_mesh(x, grid) for x in designs]
    mesh = fi.concat_meshes(meshes)
    nm = len(meshes)
    fp = fi.freestream_params(3, mach, reynolds, n_mesh=nm)
    for k, x in enumerate(designs):
        a = np.deg2rad(x[3])
        fp.vel_inf[k] = [np.cos(a), np.sin(a), 0.0]
    span = grid.get("span", 0.2) if span is None else span
    probes = [[probe[0], probe[1], 0.5 * span] for _ in range(nm)]
    sol = Solver(mesh, p, fp, equations="ns", precision=precision, probes=probes, probe_mesh=list(range(nm)),
                 max_samples=steps, forces=True)
    x = sol.solpt_coords()
    u = np.empty(x.shape[:-1] + (5,))
    for k in range(nm):
        lo, hi = mesh.mesh_elem_begin[k], mesh.mesh_elem_begin[k + 1]
        u[lo:hi] = fi.freestream_state(x[lo:hi], fp, k)
    ut = torch.tensor(u, dtype=sol.dtype).permute(0, 2, 1).contiguous().to(device)
    dtt = torch.full((nm,), dt, dtype=torch.float64, device=device)
    sol.reset_accumulators()
    sol.rk_step(ut, dtt, steps, sample_every=sample_every)
    st = sol.probe_oaspl(p_ref=p_ref_pa * fp.p_inf[0] / 101325.0)
    # Eq. (8) in the library: drag along the free stream, lift normal to it in the x-y plane,
    # reference area chord (1) x span
    ed = np.asarray(fp.vel_inf) / np.linalg.norm(np.asarray(fp.vel_inf), axis=1, keepdims=True)
    el = np.stack([-ed[:, 1], ed[:, 0], np.zeros(nm)], axis=1)
    c = sol.force_coefficients(np.stack([ed, el], axis=1), np.full(nm, span))
    cd, cl = c[:, 0], c[:, 1]
    out = {"oaspl": st["oaspl"], "cl": cl, "cd": cd, "n_samples": st["n_samples"],
           "finite": bool(torch.isfinite(ut).all())}
    if cl_base is not None and cd_base is not None:
        out["objective"] = naca_objective(st["oaspl"], cl, cd, cl_base, cd_base)
    sol.close()
    return out
