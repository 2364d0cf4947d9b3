"""FR residual, RK4 trajectory, probe / force sampling and OASPL statistics (oracle).

TEST INFRASTRUCTURE ONLY.  Plain, dense, slow and written to be read against
the method: every element operator is a full matrix applied with einsum.

Residual (FR with the g_DG correction, conservation law Eq. (1) in transformed form):
    u_f   = M0 u                                  (solution -> flux points)
    NS:   u^ = (1/2 + beta) u_L + (1/2 - beta) u_R  (LDG common solution; BC state on boundaries)
          d_xi_k u = D_k u + sum_{f: k_f = k} s_f g_R'(s_f xi^(k)) (u^_f - u_f)    (corrected gradient)
          grad_x u = J^{-1} S^T grad_xi u ;  grad u_f = M0 grad_x u
    F     = F_inv(u) - F_vis(u, grad u)            (Eqs. (3)-(7))
    F~_k  = sum_j S_kj F_j
    F^_n  = [Rusanov(u_L, u_R, n) - LDG viscous(n)] |N| on the L side, its negation on the R side
    R     = -(1/J) [ sum_k D_k F~_k + Lift (F^_n - s_f (M0 F~_{k_f})) ]
RK4: classical four-stage scheme with an explicit dt per mesh.
Sampling: before every ``sample_every``-th step the probe pressure (interpolate the
conserved state, then Eq. (5)) and the wall force (integral of p n - tau n over the
wall, used for Eq. (8)) of the current state are recorded.
"""
from __future__ import annotations

import numpy as np
import torch

from .basis import TensorOps
from .flow import (farfield_state, inviscid_flux, pressure, rusanov, viscous_flux, wall_ghost_inviscid,
                   wall_state_viscous)
from .geometry import adjugate, element_map, geometry_basis, locate_point, match_faces

FACE_AUTO, BC_WALL, BC_FARFIELD = 0, 1, 2
DT = torch.float64


class OracleSystem:
    def __init__(self, mesh, p: int, flow, equations: str = "ns", probes=None, probe_mesh=None,
                 node_xyz: torch.Tensor | None = None):
        self.dim = d = mesh.dim
        self.p = p
        self.mesh = mesh
        self.flow = flow
        self.equations = equations
        self.viscous = equations == "ns"
        self.ops = ops = TensorOps(d, p)
        self.nv = d + 2
        self.Ne = mesh.n_elem
        t = lambda a: torch.as_tensor(np.asarray(a), dtype=DT)  # noqa: E731
        self.M0, self.Dk, self.Lift, self.LiftG = t(ops.M0), t(ops.Dk), t(ops.Lift), t(ops.LiftG)
        self.fpt_k = torch.as_tensor(ops.fpt_k)
        self.fpt_s = t(ops.fpt_s)
        self.fpt_w = t(ops.fpt_w)
        self.sol_w = t(ops.sol_w)
        # geometry bases at solution and flux points
        self.phi_s, self.dphi_s = geometry_basis(d, mesh.q, ops.ref_solpts())
        self.phi_f, self.dphi_f = geometry_basis(d, mesh.q, ops.ref_fpts())
        elem_mesh = np.zeros(self.Ne, dtype=np.int64)
        for m in range(mesh.n_mesh):
            elem_mesh[mesh.mesh_elem_begin[m]:mesh.mesh_elem_begin[m + 1]] = m
        self.elem_mesh = torch.as_tensor(elem_mesh)
        nodes = torch.as_tensor(mesh.node_xyz, dtype=DT) if node_xyz is None else node_xyz
        self.nodes = nodes
        geo = self.geometry(nodes)
        scale = float(np.ptp(mesh.node_xyz, axis=0).max())
        (eL, fL, eR, fR), (bE, bF, bT) = match_faces(
            d, geo["x_f"].detach().numpy(), ops.fpt_k, ops.fpt_s, ops.Nfp, mesh.face_bc, mesh.periodic_vec, scale,
            elem_mesh)
        self.eL, self.fL, self.eR, self.fR = map(torch.as_tensor, (eL, fL, eR, fR))
        self.bE, self.bF, self.bT = map(torch.as_tensor, (bE, bF, bT))
        self.geo = geo
        # free-stream per boundary point
        self.rho_inf = t(flow.rho_inf)
        self.v_inf = t(flow.vel_inf)
        self.p_inf = t(flow.p_inf)
        self.mu = t(flow.mu)
        # probes
        self.probes = []
        self.probe_xyz = []
        if probes is not None:
            probes = np.atleast_2d(np.asarray(probes, float))
            self.probe_xyz = list(probes)
            pm = np.zeros(len(probes), dtype=np.int64) if probe_mesh is None else np.asarray(probe_mesh)
            for a, xp in enumerate(probes):
                lo, hi = mesh.mesh_elem_begin[pm[a]], mesh.mesh_elem_begin[pm[a] + 1]
                e, xi = locate_point(xp, mesh.node_xyz, mesh.elem_nodes[lo:hi], d, mesh.q)
                self.probes.append((int(lo + e), xi, int(pm[a])))

    # ------------------------------------------------------------------ geometry
    def geometry(self, nodes: torch.Tensor) -> dict:
        """Metrics at solution points and normals at flux points from node coordinates."""
        x_s, A_s = element_map(nodes, self.mesh.elem_nodes, self.phi_s, self.dphi_s)
        x_f, A_f = element_map(nodes, self.mesh.elem_nodes, self.phi_f, self.dphi_f)
        J = torch.linalg.det(A_s)
        if bool((J <= 0).any()):
            raise ValueError("element with non-positive Jacobian")
        S = adjugate(A_s)                                     # [Ne, Ns, k, j]
        Sf = adjugate(A_f)                                    # [Ne, Nf, k, j]
        k = self.fpt_k
        N = self.fpt_s[None, :, None] * Sf[:, torch.arange(Sf.shape[1]), k, :]   # [Ne, Nf, d]
        magN = torch.linalg.norm(N, dim=-1)
        return {"x_s": x_s, "x_f": x_f, "J": J, "S": S, "N": N, "magN": magN, "n": N / magN[..., None]}

    def set_nodes(self, nodes: torch.Tensor):
        """Recompute the metrics from (possibly differentiable) node coordinates; topology and the
        probes' elements are kept."""
        self.nodes = nodes
        self.geo = self.geometry(nodes)

    def _probe_weights(self, a: int) -> torch.Tensor:
        """Tensor Lagrange weights of probe a.  The probe is fixed in physical space, so when the
        node coordinates carry gradients its reference coordinates xi follow them: one Newton
        correction xi = xi0 - A^{-1} (x(xi0) - x_p) from the converged point (residual ~ 0) has
        the implicit-function derivative d xi / d X_n = -A^{-1} phi_n(xi)."""
        e, xi0, _ = self.probes[a]
        if not (isinstance(self.nodes, torch.Tensor) and self.nodes.requires_grad):
            return torch.as_tensor(self.ops.interp_weights(xi0), dtype=DT)
        d = self.dim
        phi, dphi = geometry_basis(d, self.mesh.q, np.asarray(xi0, float)[None, :])
        Xe = self.nodes[torch.as_tensor(self.mesh.elem_nodes[e])]
        x = torch.as_tensor(phi[0]) @ Xe
        A = torch.stack([torch.as_tensor(dphi[k, 0]) @ Xe for k in range(d)], dim=1)      # A[j, k]
        xi = torch.as_tensor(np.asarray(xi0, float)) - torch.linalg.solve(
            A, x - torch.as_tensor(self.probe_xyz[a], dtype=DT))
        nodes1 = torch.as_tensor(self.ops.xi, dtype=DT)
        w = torch.ones(self.ops.Ns, dtype=DT)
        for k in range(d):
            lk = torch.stack([torch.prod(torch.stack([(xi[k] - nodes1[m]) / (nodes1[b] - nodes1[m])
                                                      for m in range(self.ops.P) if m != b]))
                              for b in range(self.ops.P)])
            w = w * lk[torch.as_tensor(self.ops.sol_idx[:, k])]
        return w

    def solpt_coords(self) -> np.ndarray:
        return self.geo["x_s"].detach().numpy()            # [Ne, Ns, d]

    # ------------------------------------------------------------------ residual
    def _bc_data(self, geo, uB):
        m = self.elem_mesh[self.bE]
        nB = geo["n"][self.bE, self.bF]
        far = farfield_state(uB, nB, self.rho_inf[m], self.v_inf[m], self.p_inf[m], self.flow.gamma)
        wall = (self.bT == BC_WALL)[:, None]
        ghost_inv = torch.where(wall, wall_ghost_inviscid(uB), far)
        ghost_vis = torch.where(wall, wall_state_viscous(uB), far)
        return nB, ghost_inv, ghost_vis, m

    def residual(self, u: torch.Tensor, geo: dict | None = None, aux: bool = False):
        geo = self.geo if geo is None else geo
        g, Pr = self.flow.gamma, self.flow.prandtl
        beta, tau_p = self.flow.ldg_beta, self.flow.ldg_tau
        S, J = geo["S"], geo["J"]
        uf = torch.einsum('fs,evs->evf', self.M0, u)
        uL = uf[self.eL, :, self.fL]
        uR = uf[self.eR, :, self.fR]
        uB = uf[self.bE, :, self.bF]
        nP = geo["n"][self.eL, self.fL]
        magP = geo["magN"][self.eL, self.fL]
        magB = geo["magN"][self.bE, self.bF]
        nB, ghost_inv, ghost_vis, mB = self._bc_data(geo, uB)
        out = {}
        if self.viscous:
            uhat = (0.5 + beta) * uL + (0.5 - beta) * uR
            du = torch.zeros_like(uf)
            du[self.eL, :, self.fL] = uhat - uL
            du[self.eR, :, self.fR] = uhat - uR
            du[self.bE, :, self.bF] = ghost_vis - uB
            grad_ref = torch.einsum('kis,evs->evik', self.Dk, u) + torch.einsum('kif,evf->evik', self.LiftG, du)
            grad = torch.einsum('eikj,evik->evij', S / J[..., None, None], grad_ref)    # [Ne, nv, Ns, d]
            grad_f = torch.einsum('fs,evsj->evfj', self.M0, grad)
            mu_e = self.mu[self.elem_mesh]
            F = inviscid_flux(u.transpose(1, 2), g) - viscous_flux(
                u.transpose(1, 2), grad.transpose(1, 2), mu_e[:, None], g, Pr)          # [Ne, Ns, nv, d]
            out.update(du=du, grad=grad, grad_f=grad_f)
        else:
            F = inviscid_flux(u.transpose(1, 2), g)
        F = F.transpose(1, 2)                                                             # [Ne, nv, Ns, d]
        Ft = torch.einsum('eikj,evij->evik', S, F)
        FtM0 = torch.einsum('fs,evsk->evfk', self.M0, Ft)
        Nf = uf.shape[2]
        Fn_int = FtM0[:, :, torch.arange(Nf), self.fpt_k] * self.fpt_s
        # common normal fluxes (physical, unit normal of the L side)
        fP = rusanov(uL, uR, nP, g)
        fB = rusanov(uB, ghost_inv, nB, g)
        if self.viscous:
            gL = grad_f[self.eL, :, self.fL]
            gR = grad_f[self.eR, :, self.fR]
            gB = grad_f[self.bE, :, self.bF]
            muP = self.mu[self.elem_mesh[self.eL]]
            fvL = (viscous_flux(uL, gL, muP, g, Pr) * nP[:, None, :]).sum(-1)
            fvR = (viscous_flux(uR, gR, muP, g, Pr) * nP[:, None, :]).sum(-1)
            fP = fP - ((0.5 - beta) * fvL + (0.5 + beta) * fvR - tau_p * (uL - uR))
            muB = self.mu[mB]
            heat = (self.bT != BC_WALL)
            fvB_heat = (viscous_flux(ghost_vis, gB, muB, g, Pr, heat=True) * nB[:, None, :]).sum(-1)
            fvB_noheat = (viscous_flux(ghost_vis, gB, muB, g, Pr, heat=False) * nB[:, None, :]).sum(-1)
            fB = fB - torch.where(heat[:, None], fvB_heat, fvB_noheat)
        Fhat = torch.zeros_like(uf)
        Fhat[self.eL, :, self.fL] = fP * magP[:, None]
        Fhat[self.eR, :, self.fR] = -fP * magP[:, None]
        Fhat[self.bE, :, self.bF] = fB * magB[:, None]
        div = torch.einsum('kis,evsk->evi', self.Dk, Ft) + torch.einsum('if,evf->evi', self.Lift, Fhat - Fn_int)
        R = -div / J[:, None, :]
        if aux:
            out.update(uf=uf, Fhat=Fhat, Fn_int=Fn_int, Ft=Ft, F=F)
            return R, out
        return R

    # ------------------------------------------------------------------ time stepping
    def rk4_step(self, u, dt, geo=None):
        """Classical RK4 with dt[mesh] (a float, a float64 array or a float64 tensor)."""
        if isinstance(dt, torch.Tensor) and dt.dtype != DT:
            raise TypeError("dt must be float64 (a float32 dt silently perturbs the step size)")
        dte = torch.as_tensor(dt, dtype=DT).reshape(-1)[self.elem_mesh][:, None, None]
        k1 = self.residual(u, geo)
        k2 = self.residual(u + 0.5 * dte * k1, geo)
        k3 = self.residual(u + 0.5 * dte * k2, geo)
        k4 = self.residual(u + dte * k3, geo)
        return u + dte / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def probe_pressure(self, u, geo=None):
        """Pressure at each probe: interpolate the conserved state with the tensor Lagrange
        weights at the probe's reference coordinates, then apply Eq. (5)."""
        if not self.probes:
            return torch.zeros(0, dtype=DT)
        vals = []
        for a, (e, xi, _) in enumerate(self.probes):
            w = self._probe_weights(a)
            up = (u[e] * w[None, :]).sum(-1)
            vals.append(pressure(up, self.flow.gamma))
        return torch.stack(vals)

    def wall_force(self, u, geo=None):
        """Force on the walls of each mesh: sum over wall flux points of w_f |N| (p n - tau n),
        n the fluid element's outward normal, tau from the corrected gradient with v = 0."""
        geo = self.geo if geo is None else geo
        nm = self.mesh.n_mesh
        if not self.viscous:
            R, aux = None, None
        wall = self.bT == BC_WALL
        if not bool(wall.any()):
            return torch.zeros((nm, self.dim), dtype=DT)
        g, Pr = self.flow.gamma, self.flow.prandtl
        _, aux = self.residual(u, geo, aux=True)
        e, f = self.bE[wall], self.bF[wall]
        uB = aux["uf"][e, :, f]
        n = geo["n"][e, f]
        mag = geo["magN"][e, f]
        w = self.fpt_w[f]
        p = pressure(uB, g)
        traction = p[:, None] * n
        if self.viscous:
            gB = aux["grad_f"][e, :, f]
            m = self.elem_mesh[e]
            fv = viscous_flux(wall_state_viscous(uB), gB, self.mu[m], g, Pr, heat=False)
            traction = traction - (fv[:, 1:1 + self.dim, :] * n[:, None, :]).sum(-1)
        contrib = (w * mag)[:, None] * traction
        out = torch.zeros((nm, self.dim), dtype=DT)
        return out.index_add(0, self.elem_mesh[e], contrib)

    def run(self, u, dt, n_steps: int, sample_every: int = 1, step0: int = 0, geo=None, forces: bool = True):
        """Advance n_steps RK4 steps; before each step whose global index is a multiple of
        sample_every, record the probe pressures and wall forces of the current state."""
        ps, fs = [], []
        for n in range(n_steps):
            if sample_every > 0 and (step0 + n) % sample_every == 0:
                ps.append(self.probe_pressure(u, geo))
                if forces:
                    fs.append(self.wall_force(u, geo))
            u = self.rk4_step(u, dt, geo)
        P = torch.stack(ps) if ps else torch.zeros((0, len(self.probes)), dtype=DT)
        Fz = torch.stack(fs) if fs else torch.zeros((0, self.mesh.n_mesh, self.dim), dtype=DT)
        return u, P, Fz

    # ------------------------------------------------------------------ helpers
    def integrate(self, v: torch.Tensor, geo=None) -> torch.Tensor:
        """Quadrature integral over the domain, per variable: sum_e sum_i w_i J_i v_i."""
        geo = self.geo if geo is None else geo
        return torch.einsum('i,ei,evi->v', self.sol_w, geo["J"], v)


def cumulative_prms(p: np.ndarray) -> np.ndarray:
    """Vectors of Eqs. (10)-(12): element k (1-based) is the RMS of the first k samples about
    their own mean (the cumulative time average of Eq. (12))."""
    p = np.asarray(p, float)
    out = np.empty(len(p))
    for k in range(1, len(p) + 1):
        pbar_k = p[:k].sum() / k
        out[k - 1] = np.sqrt(((p[:k] - pbar_k) ** 2).sum() / k)
    return out


def oaspl_from_series(p: np.ndarray, p_ref: float) -> float:
    """OASPL = 20 log10(p_RMS / p_ref), Eq. (9), with p_RMS the last element of the
    cumulative vector (population RMS of all samples about their mean)."""
    prms = cumulative_prms(p)[-1]
    with np.errstate(divide="ignore"):
        return float(20.0 * np.log10(prms / p_ref))


def force_coefficients(force: np.ndarray, rho_inf, vel_inf, directions: np.ndarray, ref_area) -> np.ndarray:
    """Force coefficients of Eq. (8): the time-mean wall force of each mesh projected on each
    given unit direction, over the free-stream dynamic pressure 1/2 rho_inf |U_inf|^2 times the
    reference area (span times length).  force [n_mesh][dim], rho_inf [n_mesh],
    vel_inf [n_mesh][dim], directions [n_mesh][n_dir][dim], ref_area [n_mesh] -> [n_mesh][n_dir]."""
    force = np.asarray(force, float)
    q = 0.5 * np.asarray(rho_inf, float) * np.sum(np.asarray(vel_inf, float) ** 2, axis=-1)
    out = np.empty(np.asarray(directions).shape[:2])
    for m in range(force.shape[0]):
        for j in range(out.shape[1]):
            out[m, j] = float(np.dot(force[m], directions[m][j])) / (q[m] * float(ref_area[m]))
    return out


def airfoil_objective(oaspl, cl, cd, cl_base, cd_base, eps1: float = 8000.0, eps2: float = 400000.0):
    """Penalised objective of the airfoil optimisation: OASPL plus eps1 times the squared departure
    of the mean lift coefficient from the baseline's, plus eps2 times the squared excess of the
    mean drag coefficient when it is above the baseline's (eps1 = 8000, eps2 = 400000)."""
    f = float(oaspl) + eps1 * (float(cl) - cl_base) ** 2
    if float(cd) > cd_base:
        f += eps2 * (float(cd) - cd_base) ** 2
    return f
