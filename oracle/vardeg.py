"""Flux reconstruction with a solution degree per element (oracle; test infrastructure only).

The airfoil case's computational details use a solution degree that falls from P4 (or P3) near
the airfoil to P0 towards the boundaries, to damp acoustic waves before they reach them; the
paper shows the distribution but not how faces between degrees are treated.  Reading taken:
* every element is FR of its own degree p_e (Gauss-Legendre points, g_DG correction; p_e = 0 is
  one point with g_R' = 1/2, i.e. a finite-volume cell);
* faces between equal degrees: as in fr.py;
* a face between degrees p_lo < p_hi is a mortar made of the higher side's flux points: the lower
  side's trace polynomial (through its own flux points) is evaluated there; the common solution
  and the common flux are formed there, with the higher side's unit normal and |N|; the viscous
  normal flux of each side at its own flux points (its own outward normal) is carried to the
  mortar the same way; the higher side takes the mortar values at its own points, the lower side
  takes their L2 projection onto its face polynomials (Gauss quadrature on the mortar points),
  for the transformed common flux (F^ |N|) as well, so each face's integrated flux is the same
  from both sides and the scheme stays conservative across degree jumps.
The state is a list with one tensor [n_elem of the group, nv, P^dim] per degree group (groups in
increasing degree, elements of a group in increasing element number).
"""
from __future__ import annotations

import itertools

import numpy as np
import torch
from scipy.spatial import cKDTree

from .basis import TensorOps, lagrange_eval
from .flow import (farfield_state, inviscid_flux, pressure, rusanov, viscous_flux, wall_ghost_inviscid,
                   wall_state_viscous)
from .geometry import adjugate, element_map, geometry_basis, locate_point

DT = torch.float64
FACE_AUTO, BC_WALL, BC_FARFIELD = 0, 1, 2


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=DT)


class _Group:
    """Operators, metrics and flux-point geometry of the elements of one degree."""

    def __init__(self, mesh, p, elems, nodes):
        d = mesh.dim
        self.p, self.elems = p, elems
        self.ops = ops = TensorOps(d, p)
        self.M0, self.Dk, self.Lift, self.LiftG = _t(ops.M0), _t(ops.Dk), _t(ops.Lift), _t(ops.LiftG)
        self.fpt_k = torch.as_tensor(ops.fpt_k)
        self.fpt_s = _t(ops.fpt_s)
        self.fpt_w = _t(ops.fpt_w)
        self.sol_w = _t(ops.sol_w)
        phi_s, dphi_s = geometry_basis(d, mesh.q, ops.ref_solpts())
        phi_f, dphi_f = geometry_basis(d, mesh.q, ops.ref_fpts())
        en = mesh.elem_nodes[elems]
        x_s, A_s = element_map(nodes, en, phi_s, dphi_s)
        x_f, A_f = element_map(nodes, en, phi_f, dphi_f)
        J = torch.linalg.det(A_s)
        if bool((J <= 0).any()):
            raise ValueError("element with non-positive Jacobian")
        S = adjugate(A_s)
        Sf = adjugate(A_f)
        N = self.fpt_s[None, :, None] * Sf[:, torch.arange(Sf.shape[1]), self.fpt_k, :]
        mag = torch.linalg.norm(N, dim=-1)
        self.x_s, self.x_f, self.J, self.S, self.magN, self.n = x_s, x_f, J, S, mag, N / mag[..., None]


class VarDegreeOracle:
    def __init__(self, mesh, degree, flow, equations: str = "ns", probes=None):
        d = mesh.dim
        self.dim, self.mesh, self.flow = d, mesh, flow
        self.nv = d + 2
        self.viscous = equations == "ns"
        self.degree = degree = np.asarray(degree, dtype=np.int64)
        if degree.shape != (mesh.n_elem,) or degree.min() < 0 or degree.max() > 4:
            raise ValueError("one degree in 0..4 per element")
        nodes = _t(mesh.node_xyz)
        self.degs = sorted(set(degree.tolist()))
        self.groups = [_Group(mesh, p, np.nonzero(degree == p)[0], nodes) for p in self.degs]
        self.gidx = np.zeros(mesh.n_elem, dtype=np.int64)   # group of each element
        self.lidx = np.zeros(mesh.n_elem, dtype=np.int64)   # index inside the group
        for g, G in enumerate(self.groups):
            self.gidx[G.elems] = g
            self.lidx[G.elems] = np.arange(len(G.elems))
        elem_mesh = np.zeros(mesh.n_elem, dtype=np.int64)
        for m in range(mesh.n_mesh):
            elem_mesh[mesh.mesh_elem_begin[m]:mesh.mesh_elem_begin[m + 1]] = m
        self.elem_mesh = elem_mesh
        self.rho_inf, self.v_inf = _t(flow.rho_inf), _t(flow.vel_inf)
        self.p_inf, self.mu = _t(flow.p_inf), _t(flow.mu)
        self._connect(nodes)
        self.probes = []
        if probes is not None:
            for xp in np.atleast_2d(np.asarray(probes, float)):
                e, xi = locate_point(xp, mesh.node_xyz, mesh.elem_nodes, d, mesh.q)
                G = self.groups[self.gidx[e]]
                self.probes.append((int(self.gidx[e]), int(self.lidx[e]), _t(G.ops.interp_weights(xi))))

    # ------------------------------------------------------------------ connectivity
    def _map(self, e, ref):
        """Physical coordinates of reference points ref [n, d] in element e."""
        phi, _ = geometry_basis(self.dim, self.mesh.q, np.atleast_2d(ref))
        return phi @ self.mesh.node_xyz[self.mesh.elem_nodes[e]]

    def _connect(self, nodes):
        mesh, d = self.mesh, self.dim
        nface = 2 * d
        scale = float(np.ptp(mesh.node_xyz, axis=0).max())
        cref = np.zeros((nface, d))
        for f in range(nface):
            cref[f, f // 2] = -1.0 if f % 2 == 0 else 1.0
        phi_c, _ = geometry_basis(d, mesh.q, cref)
        cent = np.einsum('fn,enj->efj', phi_c, mesh.node_xyz[mesh.elem_nodes])       # [Ne, nface, d]
        auto = [(e, f) for e in range(mesh.n_elem) for f in range(nface) if mesh.face_bc[e, f] == FACE_AUTO]
        shifts = [np.zeros(d)] + [s * v for v in np.asarray(mesh.periodic_vec).reshape(-1, d) for s in (1.0, -1.0)]
        tree = cKDTree(np.array([cent[e, f] for e, f in auto])) if auto else None
        partner = {}
        for a, (e, f) in enumerate(auto):
            if (e, f) in partner:
                continue
            found = None
            for sh in shifts:
                for b in tree.query_ball_point(cent[e, f] + sh, 1e-8 * scale):
                    if b != a and self.elem_mesh[auto[b][0]] == self.elem_mesh[e]:
                        found = (auto[b], sh)
                        break
                if found:
                    break
            if found is None:
                raise ValueError(f"unmatched face: element {e} face {f}")
            (e2, f2), sh = found
            partner[(e, f)] = ((e2, f2), sh)
            partner[(e2, f2)] = ((e, f), -sh)
        ng = len(self.groups)
        self.pairs = [[] for _ in range(ng)]       # per group: (eL, fpL, eR, fpR) local indices
        self.mortars = []                          # mixed-degree faces
        for (e, f), ((e2, f2), sh) in partner.items():
            if (e, f) > (e2, f2):
                continue
            ga, gb = self.gidx[e], self.gidx[e2]
            Ga, Gb = self.groups[ga], self.groups[gb]
            if ga == gb:
                Nfp = Ga.ops.Nfp
                xa = Ga.x_f[self.lidx[e], f * Nfp:(f + 1) * Nfp].numpy() + sh
                xb = Gb.x_f[self.lidx[e2], f2 * Nfp:(f2 + 1) * Nfp].numpy()
                dist = np.linalg.norm(xa[:, None] - xb[None], axis=-1)
                j = dist.argmin(axis=1)
                if dist[np.arange(Nfp), j].max() > 1e-7 * scale or len(set(j.tolist())) != Nfp:
                    raise ValueError(f"non-conforming face pair ({e},{f})-({e2},{f2})")
                for t in range(Nfp):
                    self.pairs[ga].append((self.lidx[e], f * Nfp + t, self.lidx[e2], f2 * Nfp + j[t]))
                continue
            # mortar on the higher side's flux points
            hi_is_a = Ga.p > Gb.p
            (eh, fh, gh), (el, fl, gl) = ((e, f, ga), (e2, f2, gb)) if hi_is_a else ((e2, f2, gb), (e, f, ga))
            shl = sh if hi_is_a else -sh            # x on the lower side = x on the higher side + shl
            H, Lo = self.groups[gh], self.groups[gl]
            k = fh // 2
            others = [m for m in range(d) if m != k]
            # canonical lower-degree points: the lower degree's Gauss points along the higher face's
            # tangential coordinates (lowest coordinate fastest), matched to the lower face's points
            can = []
            for t in itertools.product(range(Lo.p + 1), repeat=d - 1):
                t = t[::-1]
                r = np.zeros(d)
                r[k] = -1.0 if fh % 2 == 0 else 1.0
                for m, tm in zip(others, t):
                    r[m] = Lo.ops.xi[tm]
                can.append(r)
            can = np.array(can)
            xc = self._map(eh, can) + shl
            Nlo = Lo.ops.Nfp
            xl = Lo.x_f[self.lidx[el], fl * Nlo:(fl + 1) * Nlo].numpy()
            dist = np.linalg.norm(xc[:, None] - xl[None], axis=-1)
            perm = dist.argmin(axis=1)
            if dist[np.arange(Nlo), perm].max() > 1e-7 * scale or len(set(perm.tolist())) != Nlo:
                raise ValueError(f"non-conforming mixed-degree face ({e},{f})-({e2},{f2})")
            # I[i, j]: lower-degree tensor Lagrange basis j at mortar point i; Pi = W_lo^-1 I^T W_m
            Nm = H.ops.Nfp
            I = np.ones((Nm, Nlo))
            for i in range(Nm):
                tmap = H.ops.fpt_t[fh * Nm + i]
                for jdx in range(Nlo):
                    val = 1.0
                    for a, m in enumerate(others):
                        xm = H.ops.xi[tmap[m]]
                        lj = lagrange_eval(Lo.ops.xi, np.array([xm]))[0]
                        # index of canonical point jdx along coordinate m (lowest coordinate fastest)
                        tj_m = (jdx // (Lo.p + 1) ** a) % (Lo.p + 1)
                        val *= lj[tj_m]
                    I[i, jdx] = val
            wm = np.array([np.prod([H.ops.w[H.ops.fpt_t[fh * Nm + i][m]] for m in others]) for i in range(Nm)])
            wl = np.array([np.prod([Lo.ops.w[(jdx // (Lo.p + 1) ** a) % (Lo.p + 1)] for a in range(d - 1)])
                           for jdx in range(Nlo)])
            Pi = (I * wm[:, None]).T / wl[:, None]
            self.mortars.append(dict(gh=gh, eh=self.lidx[eh], fph=np.arange(fh * Nm, (fh + 1) * Nm),
                                     gl=gl, el=self.lidx[el], fpl=fl * Nlo + perm, I=_t(I), Pi=_t(Pi),
                                     hi_is_L=bool(hi_is_a)))
        # boundary points per group
        self.bnd = []
        for G in self.groups:
            bE, bF, bT = [], [], []
            Nfp = G.ops.Nfp
            for le, e in enumerate(G.elems):
                for f in range(nface):
                    if mesh.face_bc[e, f] != FACE_AUTO:
                        for t in range(Nfp):
                            bE.append(le)
                            bF.append(f * Nfp + t)
                            bT.append(int(mesh.face_bc[e, f]))
            self.bnd.append(tuple(torch.as_tensor(np.array(a, dtype=np.int64)) for a in (bE, bF, bT)))
        self.pairs = [tuple(torch.as_tensor(np.array([q[c] for q in P], dtype=np.int64)) for c in range(4))
                      for P in self.pairs]

    # ------------------------------------------------------------------ helpers
    def solpt_coords(self):
        return [G.x_s.numpy() for G in self.groups]

    def split(self, flat: torch.Tensor):
        """Per-group tensors from a flat state in group order."""
        out, o = [], 0
        for G in self.groups:
            n = len(G.elems) * self.nv * G.ops.Ns
            out.append(flat[o:o + n].reshape(len(G.elems), self.nv, G.ops.Ns))
            o += n
        return out

    @staticmethod
    def join(parts):
        return torch.cat([p.reshape(-1) for p in parts])

    def integrate(self, parts):
        """sum over groups and elements of sum_i w_i J_i v_i, per variable."""
        return sum(torch.einsum('i,ei,evi->v', G.sol_w, G.J, v) for G, v in zip(self.groups, parts))

    # ------------------------------------------------------------------ residual
    def _traces(self, u):
        """Own flux-point states and boundary data (states, normals, inviscid and viscous ghosts)."""
        g_ = self.flow.gamma
        uf = [torch.einsum('fs,evs->evf', G.M0, ug) for G, ug in zip(self.groups, u)]
        bdata = []
        for gi, G in enumerate(self.groups):
            bE, bF, bT = self.bnd[gi]
            uB = uf[gi][bE, :, bF]
            m = torch.as_tensor(self.elem_mesh[G.elems])[bE]
            nB = G.n[bE, bF]
            far = farfield_state(uB, nB, self.rho_inf[m], self.v_inf[m], self.p_inf[m], g_)
            wall = (bT == BC_WALL)[:, None]
            bdata.append((uB, nB, torch.where(wall, wall_ghost_inviscid(uB), far),
                          torch.where(wall, wall_state_viscous(uB), far), m))
        return uf, bdata

    def _gradients(self, u, uf, bdata):
        """LDG common solution (pairs, boundaries, mortars) and the corrected physical gradient at
        solution points and at own flux points, per group."""
        beta = self.flow.ldg_beta
        du = [torch.zeros_like(x) for x in uf]
        for gi in range(len(self.groups)):
            eL, fL, eR, fR = self.pairs[gi]
            uL, uR = uf[gi][eL, :, fL], uf[gi][eR, :, fR]
            uh = (0.5 + beta) * uL + (0.5 - beta) * uR
            du[gi][eL, :, fL] = uh - uL
            du[gi][eR, :, fR] = uh - uR
            bE, bF, _ = self.bnd[gi]
            du[gi][bE, :, bF] = bdata[gi][3] - bdata[gi][0]
        for M in self.mortars:
            uh_ = uf[M["gh"]][M["eh"], :, M["fph"]]                 # [nv, Nm]
            ul_ = uf[M["gl"]][M["el"], :, M["fpl"]] @ M["I"].T      # lower trace at the mortar
            uL, uR = (uh_, ul_) if M["hi_is_L"] else (ul_, uh_)
            uhat = (0.5 + beta) * uL + (0.5 - beta) * uR
            du[M["gh"]][M["eh"], :, M["fph"]] = uhat - uh_
            du[M["gl"]][M["el"], :, M["fpl"]] = uhat @ M["Pi"].T - uf[M["gl"]][M["el"], :, M["fpl"]]
        grad, grad_f = [], []
        for gi, G in enumerate(self.groups):
            gr = torch.einsum('kis,evs->evik', G.Dk, u[gi]) + torch.einsum('kif,evf->evik', G.LiftG, du[gi])
            gr = torch.einsum('eikj,evik->evij', G.S / G.J[..., None, None], gr)
            grad.append(gr)
            grad_f.append(torch.einsum('fs,evsj->evfj', G.M0, gr))
        return grad, grad_f

    def residual(self, u):
        g_, Pr, beta, tau = self.flow.gamma, self.flow.prandtl, self.flow.ldg_beta, self.flow.ldg_tau
        groups = self.groups
        uf, bdata = self._traces(u)
        Fhat = [torch.zeros_like(x) for x in uf]
        mu_e = [self.mu[torch.as_tensor(self.elem_mesh[G.elems])] for G in groups]
        if self.viscous:
            grad, grad_f = self._gradients(u, uf, bdata)
        fvn, F_all = [], []
        for gi, G in enumerate(groups):
            F = inviscid_flux_t(u[gi], g_)
            if self.viscous:
                F = F - viscous_flux(u[gi].transpose(1, 2), grad[gi].transpose(1, 2), mu_e[gi][:, None], g_,
                                     Pr).transpose(1, 2)
                # viscous normal flux at own flux points along the own outward normal
                fvn.append((viscous_flux(uf[gi].transpose(1, 2), grad_f[gi].transpose(1, 2), mu_e[gi][:, None],
                                         g_, Pr) * G.n[:, :, None, :]).sum(-1).transpose(1, 2))    # [Ne, nv, Nf]
            F_all.append(F)
        # common fluxes inside groups and on boundaries (as in fr.py)
        for gi, G in enumerate(groups):
            eL, fL, eR, fR = self.pairs[gi]
            uL, uR = uf[gi][eL, :, fL], uf[gi][eR, :, fR]
            nP, magP = G.n[eL, fL], G.magN[eL, fL]
            fP = rusanov(uL, uR, nP, g_)
            uB, nB, ghost_inv, ghost_vis, mB = bdata[gi]
            bE, bF, bT = self.bnd[gi]
            fB = rusanov(uB, ghost_inv, nB, g_)
            if self.viscous:
                muP = mu_e[gi][eL]
                fvL = (viscous_flux(uL, grad_f[gi][eL, :, fL], muP, g_, Pr) * nP[:, None, :]).sum(-1)
                fvR = (viscous_flux(uR, grad_f[gi][eR, :, fR], muP, g_, Pr) * nP[:, None, :]).sum(-1)
                fP = fP - ((0.5 - beta) * fvL + (0.5 + beta) * fvR - tau * (uL - uR))
                heat = (bT != BC_WALL)
                gB = grad_f[gi][bE, :, bF]
                muB = self.mu[mB]
                fvh = (viscous_flux(ghost_vis, gB, muB, g_, Pr, heat=True) * nB[:, None, :]).sum(-1)
                fvq = (viscous_flux(ghost_vis, gB, muB, g_, Pr, heat=False) * nB[:, None, :]).sum(-1)
                fB = fB - torch.where(heat[:, None], fvh, fvq)
            Fhat[gi][eL, :, fL] = fP * magP[:, None]
            Fhat[gi][eR, :, fR] = -fP * magP[:, None]
            Fhat[gi][bE, :, bF] = fB * G.magN[bE, bF][:, None]
        # mortar faces
        for M in self.mortars:
            H = groups[M["gh"]]
            uh_ = uf[M["gh"]][M["eh"], :, M["fph"]].T                       # [Nm, nv]
            ul_ = (uf[M["gl"]][M["el"], :, M["fpl"]] @ M["I"].T).T
            nh = H.n[M["eh"], M["fph"]]
            mag = H.magN[M["eh"], M["fph"]]
            if M["hi_is_L"]:
                uL, uR, nL = uh_, ul_, nh
            else:
                uL, uR, nL = ul_, uh_, -nh
            F = rusanov(uL, uR, nL, g_)
            if self.viscous:
                fvh = fvn[M["gh"]][M["eh"], :, M["fph"]].T                  # along the higher side's normal
                fvl = (fvn[M["gl"]][M["el"], :, M["fpl"]] @ M["I"].T).T     # along the lower side's normal
                fvL, fvR = (fvh, fvl) if M["hi_is_L"] else (fvl, fvh)
                # along n_L: the L side's own normal flux, minus the R side's (whose normal is -n_L)
                F = F - ((0.5 - beta) * fvL - (0.5 + beta) * fvR - tau * (uL - uR))
            Fm = (F * mag[:, None]).T                                         # [nv, Nm], along n_L, x |N|
            sh = 1.0 if M["hi_is_L"] else -1.0
            Fhat[M["gh"]][M["eh"], :, M["fph"]] = sh * Fm
            Fhat[M["gl"]][M["el"], :, M["fpl"]] = -sh * (Fm @ M["Pi"].T)
        R = []
        for gi, G in enumerate(groups):
            Ft = torch.einsum('eikj,evij->evik', G.S, F_all[gi])
            FtM0 = torch.einsum('fs,evsk->evfk', G.M0, Ft)
            Nf = uf[gi].shape[2]
            Fn_int = FtM0[:, :, torch.arange(Nf), G.fpt_k] * G.fpt_s
            div = torch.einsum('kis,evsk->evi', G.Dk, Ft) + torch.einsum('if,evf->evi', G.Lift, Fhat[gi] - Fn_int)
            R.append(-div / G.J[:, None, :])
        return R

    # ------------------------------------------------------------------ time stepping, sampling
    def rk4_step(self, u, dt):
        dt = torch.as_tensor(dt, dtype=DT).reshape(-1)
        dte = [dt[torch.as_tensor(self.elem_mesh[G.elems])][:, None, None] for G in self.groups]

        def axpy(a, k):
            return [ui + a * d * ki for ui, d, ki in zip(u, dte, k)]
        k1 = self.residual(u)
        k2 = self.residual(axpy(0.5, k1))
        k3 = self.residual(axpy(0.5, k2))
        k4 = self.residual(axpy(1.0, k3))
        return [ui + d / 6.0 * (a + 2.0 * b + 2.0 * c + e) for ui, d, a, b, c, e in zip(u, dte, k1, k2, k3, k4)]

    def probe_pressure(self, u):
        return torch.stack([pressure((u[g][e] * w[None, :]).sum(-1), self.flow.gamma) for g, e, w in self.probes]) \
            if self.probes else torch.zeros(0, dtype=DT)

    def wall_force(self, u):
        """Force on the walls of each mesh, summed over the degree groups: sum over wall flux points
        of w_f |N| (p n - tau n) (see fr.py)."""
        nm, d = self.mesh.n_mesh, self.dim
        out = torch.zeros((nm, d), dtype=DT)
        if not self.viscous:
            return out
        g_, Pr = self.flow.gamma, self.flow.prandtl
        uf, bdata = self._traces(u)
        _, grad_f = self._gradients(u, uf, bdata)
        for gi, G in enumerate(self.groups):
            bE, bF, bT = self.bnd[gi]
            wall = bT == BC_WALL
            if not bool(wall.any()):
                continue
            e, f = bE[wall], bF[wall]
            uB = uf[gi][e, :, f]
            n = G.n[e, f]
            p = pressure(uB, g_)
            m = torch.as_tensor(self.elem_mesh[G.elems])[e]
            fv = viscous_flux(wall_state_viscous(uB), grad_f[gi][e, :, f], self.mu[m], g_, Pr, heat=False)
            traction = p[:, None] * n - (fv[:, 1:1 + d, :] * n[:, None, :]).sum(-1)
            out = out.index_add(0, m, (G.fpt_w[f] * G.magN[e, f])[:, None] * traction)
        return out

    def run(self, u, dt, n_steps: int, sample_every: int = 1, forces: bool = True):
        ps, fs = [], []
        for n in range(n_steps):
            if sample_every > 0 and n % sample_every == 0:
                ps.append(self.probe_pressure(u))
                if forces:
                    fs.append(self.wall_force(u))
            u = self.rk4_step(u, dt)
        P = torch.stack(ps) if ps else torch.zeros((0, len(self.probes)), dtype=DT)
        F = torch.stack(fs) if fs else torch.zeros((0, self.mesh.n_mesh, self.dim), dtype=DT)
        return u, P, F


def inviscid_flux_t(u, gamma):
    """Inviscid flux [Ne, nv, Ns, d] of a state [Ne, nv, Ns]."""
    return inviscid_flux(u.transpose(1, 2), gamma).transpose(1, 2)
