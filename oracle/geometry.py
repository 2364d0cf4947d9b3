"""Curved-element geometry, metrics, face matching and probe location (oracle; test infrastructure only).

Elements are mapped from the reference cube by x(xi) = sum_n x_n phi_n(xi) with
phi_n the tensor Lagrange basis on Gauss-Lobatto-Legendre nodes of degree q.
The metric terms follow the standard transformed form of the conservation law
(Eq. (1)): A = dx/dxi, J = det A, S = J A^{-1} (the adjugate of A), so that the
reference flux is F~_k = sum_j S_kj F_j and the physical gradient is
grad_x u = J^{-1} S^T grad_xi u.  At a flux point of face f (coordinate k_f,
side s_f) the scaled outward normal is N = s_f S[k_f, :]; |N| is the surface
Jacobian and n = N / |N| the unit normal.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch
from scipy.spatial import cKDTree

from .basis import gll_nodes, lagrange_eval, lagrange_deriv


def geometry_basis(dim: int, q: int, pts: np.ndarray):
    """phi[a, n] and dphi[k, a, n] of the degree-q GLL tensor basis at reference points pts[a]."""
    nodes = gll_nodes(q)
    nidx = np.array(list(itertools.product(range(q + 1), repeat=dim)))[:, ::-1]  # node multi-index, first fastest
    Lv = [lagrange_eval(nodes, pts[:, k]) for k in range(dim)]
    Ld = [lagrange_deriv(nodes, pts[:, k]) for k in range(dim)]
    phi = np.ones((pts.shape[0], nidx.shape[0]))
    for k in range(dim):
        phi *= Lv[k][:, nidx[:, k]]
    dphi = np.ones((dim, pts.shape[0], nidx.shape[0]))
    for kd in range(dim):
        for k in range(dim):
            dphi[kd] *= (Ld[k] if k == kd else Lv[k])[:, nidx[:, k]]
    return phi, dphi


def adjugate(A: torch.Tensor) -> torch.Tensor:
    """adj(A) with A[..., j, k] = dx_j/dxi_k; row k of adj(A) is S[k, :]."""
    d = A.shape[-1]
    if d == 2:
        return torch.stack([torch.stack([A[..., 1, 1], -A[..., 0, 1]], -1),
                            torch.stack([-A[..., 1, 0], A[..., 0, 0]], -1)], -2)
    a0, a1, a2 = A[..., :, 0], A[..., :, 1], A[..., :, 2]
    return torch.stack([torch.linalg.cross(a1, a2, dim=-1), torch.linalg.cross(a2, a0, dim=-1),
                        torch.linalg.cross(a0, a1, dim=-1)], -2)


def element_map(node_xyz: torch.Tensor, elem_nodes: np.ndarray, phi: np.ndarray, dphi: np.ndarray):
    """Physical points x[e, a, j] and Jacobian A[e, a, j, k] at reference points of every element."""
    Xe = node_xyz[torch.as_tensor(elem_nodes)]                      # [Ne, Nn, d]
    x = torch.einsum('an,enj->eaj', torch.as_tensor(phi), Xe)
    A = torch.einsum('kan,enj->eajk', torch.as_tensor(dphi), Xe)
    return x, A


def match_faces(dim, fpt_x: np.ndarray, fpt_k, fpt_s, Nfp: int, face_bc: np.ndarray, periodic_vec: np.ndarray,
                scale: float, elem_mesh: np.ndarray | None = None):
    """Pair FACE_AUTO faces geometrically (directly or under +-periodic translations); faces of
    different meshes of a batch (``elem_mesh``) are never paired, even where they coincide.

    fpt_x[e, f*Nfp + t, :] are the flux-point coordinates.  Returns per flux-point pair
    (eL, fptL, eR, fptR) with L the lexicographically smaller (element, face), and the
    boundary flux points (e, fpt, tag).  Raises ValueError on an unmatched face.
    """
    Ne = fpt_x.shape[0]
    nface = 2 * dim
    cent = fpt_x.reshape(Ne, nface, Nfp, dim).mean(axis=2)        # [Ne, nface, d]
    auto = [(e, f) for e in range(Ne) for f in range(nface) if face_bc[e, f] == 0]
    tol = 1e-8 * scale
    shifts = [np.zeros(dim)] + [s * v for v in periodic_vec for s in (1.0, -1.0)]
    pts = np.array([cent[e, f] for e, f in auto]) if auto else np.zeros((0, dim))
    tree = cKDTree(pts) if len(pts) else None
    partner = {}
    for a, (e, f) in enumerate(auto):
        if (e, f) in partner:
            continue
        found = None
        for sh in shifts:
            for b in tree.query_ball_point(cent[e, f] + sh, tol):
                if b != a and (elem_mesh is None or elem_mesh[auto[b][0]] == elem_mesh[e]):
                    found = (auto[b], sh)
                    break
            if found:
                break
        if found is None:
            raise ValueError(f"unmatched face: element {e} face {f}")
        (e2, f2), sh = found
        partner[(e, f)] = ((e2, f2), sh)
        partner[(e2, f2)] = ((e, f), -sh)
    eL, fL, eR, fR = [], [], [], []
    for (e, f), ((e2, f2), sh) in partner.items():
        if (e, f) > (e2, f2):
            continue
        xa = fpt_x[e, f * Nfp:(f + 1) * Nfp] + sh
        xb = fpt_x[e2, f2 * Nfp:(f2 + 1) * Nfp]
        dist = np.linalg.norm(xa[:, None, :] - xb[None, :, :], axis=-1)
        j = dist.argmin(axis=1)
        if dist[np.arange(Nfp), j].max() > 1e-7 * scale or len(set(j.tolist())) != Nfp:
            raise ValueError(f"non-conforming face pair ({e},{f})-({e2},{f2})")
        for t in range(Nfp):
            eL.append(e)
            fL.append(f * Nfp + t)
            eR.append(e2)
            fR.append(f2 * Nfp + j[t])
    bE, bF, bT = [], [], []
    for e in range(Ne):
        for f in range(nface):
            if face_bc[e, f] != 0:
                for t in range(Nfp):
                    bE.append(e)
                    bF.append(f * Nfp + t)
                    bT.append(int(face_bc[e, f]))
    a = lambda v: np.array(v, dtype=np.int64)  # noqa: E731
    return (a(eL), a(fL), a(eR), a(fR)), (a(bE), a(bF), a(bT))


def locate_point(xp: np.ndarray, node_xyz: np.ndarray, elem_nodes: np.ndarray, dim: int, q: int,
                 candidates=None, tol_in: float = 1e-12):
    """Lowest-index element containing xp and its reference coordinates (Newton on x(xi) = xp)."""
    Xe_all = node_xyz[elem_nodes]
    lo = Xe_all.min(axis=1)
    hi = Xe_all.max(axis=1)
    span = (hi - lo).max(axis=1)
    near = np.where(np.all((xp >= lo - 0.25 * span[:, None]) & (xp <= hi + 0.25 * span[:, None]), axis=1))[0]
    for e in near:
        xi = np.zeros(dim)
        Xe = Xe_all[e]
        ok = False
        polish = 0
        for _ in range(60):
            phi, dphi = geometry_basis(dim, q, xi[None, :])
            x = phi[0] @ Xe
            A = np.stack([dphi[k, 0] @ Xe for k in range(dim)], axis=1)  # A[j, k]
            try:
                dxi = np.linalg.solve(A, x - xp)
            except np.linalg.LinAlgError:
                break
            xi = xi - dxi
            if np.max(np.abs(xi)) > 3.0:
                break
            # converged to 1e-12 in reference coordinates, then two polishing iterations (round-off
            # in x limits |dxi| to ~eps |x| / h, above 1e-14 for small elements far from the origin)
            if ok:
                polish += 1
                if polish == 2:
                    break
            elif np.max(np.abs(dxi)) < 1e-12:
                ok = True
        if ok and np.max(np.abs(xi)) <= 1.0 + tol_in:
            return int(e), xi
    raise ValueError(f"point {xp} is outside every element")
