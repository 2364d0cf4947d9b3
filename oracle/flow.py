"""Pointwise compressible Navier-Stokes physics (oracle; test infrastructure only).

Conserved variables u = (rho, rho u_i, rho E) (Eq. (2)); inviscid flux Eq. (3);
viscous flux Eq. (4) with stress tensor Eq. (6) and heat flux Eq. (7); ideal
gas Eq. (5).  Readings taken where the paper is inconsistent or silent:
* the energy entry of Eq. (4) carries signs that cannot both be physical; the
  residual uses F = F_inv - F_vis with F_vis = (0, tau_ij, u_i tau_ij - q_j);
* the argument of the heat flux in Eq. (7) is the specific enthalpy
  gamma/(gamma-1) p/rho, so q_j = -mu gamma / (Pr (gamma-1)) d_j(p/rho);
* constant viscosity per mesh.
Common fluxes: Rusanov (local Lax-Friedrichs) for the inviscid part, LDG for
the viscous part; far field from the Riemann invariants named in the
computational-details paragraphs (subsonic textbook form).
All functions act on the trailing variable axis; normals are unit vectors.
"""
from __future__ import annotations

import torch


def primitives(u, gamma):
    d = u.shape[-1] - 2
    rho = u[..., 0]
    v = u[..., 1:1 + d] / rho[..., None]
    p = (gamma - 1.0) * (u[..., -1] - 0.5 * rho * (v * v).sum(-1))
    return rho, v, p


def pressure(u, gamma):
    return primitives(u, gamma)[2]


def inviscid_flux(u, gamma):
    """F_inv[..., var, j] (Eq. (3))."""
    d = u.shape[-1] - 2
    rho, v, p = primitives(u, gamma)
    E = u[..., -1]
    rows = [rho[..., None] * v]
    eye = torch.eye(d, dtype=u.dtype)
    for i in range(d):
        rows.append(rho[..., None] * v[..., i:i + 1] * v + p[..., None] * eye[i])
    rows.append(v * (E + p)[..., None])
    return torch.stack(rows, dim=-2)


def viscous_flux(u, gu, mu, gamma, prandtl, heat: bool = True):
    """F_vis[..., var, j] = (0, tau_ij, u_i tau_ij - q_j) from the state u and the conserved
    gradient gu[..., var, j] (Eqs. (4), (6), (7); primitive gradients by the quotient rule)."""
    d = u.shape[-1] - 2
    rho, v, p = primitives(u, gamma)
    E = u[..., -1]
    grho = gu[..., 0, :]
    dv = (gu[..., 1:1 + d, :] - v[..., :, None] * grho[..., None, :]) / rho[..., None, None]  # dv[i, j] = d_j v_i
    de = (gu[..., -1, :] - (E / rho)[..., None] * grho) / rho[..., None]                       # d_j (E/rho)
    dtheta = (gamma - 1.0) * (de - (v[..., :, None] * dv).sum(-2))                            # d_j (p/rho)
    div = sum(dv[..., i, i] for i in range(d))
    eye = torch.eye(d, dtype=u.dtype)
    mu = torch.as_tensor(mu, dtype=u.dtype)
    while mu.dim() < dv.dim() - 2:
        mu = mu[..., None]
    tau = mu[..., None, None] * (dv + dv.transpose(-1, -2) - (2.0 / 3.0) * div[..., None, None] * eye)
    q = -(mu * gamma / (prandtl * (gamma - 1.0)))[..., None] * dtheta
    energy = (v[..., :, None] * tau).sum(-2)
    if heat:
        energy = energy - q
    zero = torch.zeros_like(grho)
    return torch.cat([zero[..., None, :], tau, energy[..., None, :]], dim=-2)


TIE_RTOL = 1e-12


class _TieAveragedMax(torch.autograd.Function):
    """max(a, b) whose derivative is the average of both one-sided derivatives when a and b agree
    to a relative 1e-12 (a kink: any convex combination is a valid derivative; averaging makes
    the choice insensitive to round-off), and that of the larger argument otherwise."""

    @staticmethod
    def forward(ctx, a, b):
        ctx.save_for_backward(a, b)
        return torch.maximum(a, b)

    @staticmethod
    def backward(ctx, g):
        a, b = ctx.saved_tensors
        tie = (a - b).abs() <= TIE_RTOL * torch.maximum(a.abs(), b.abs())
        wa = torch.where(tie, torch.full_like(a, 0.5), (a > b).to(a.dtype))
        return g * wa, g * (1.0 - wa)


def rusanov(uL, uR, n, gamma):
    """Rusanov common normal flux 1/2 (F(uL) + F(uR)).n - 1/2 lambda (uR - uL),
    lambda = max(|v_L.n| + c_L, |v_R.n| + c_R)."""
    fL = (inviscid_flux(uL, gamma) * n[..., None, :]).sum(-1)
    fR = (inviscid_flux(uR, gamma) * n[..., None, :]).sum(-1)
    rL, vL, pL = primitives(uL, gamma)
    rR, vR, pR = primitives(uR, gamma)
    aL = (vL * n).sum(-1).abs() + torch.sqrt(gamma * pL / rL)
    aR = (vR * n).sum(-1).abs() + torch.sqrt(gamma * pR / rR)
    lam = _TieAveragedMax.apply(aL, aR)
    return 0.5 * (fL + fR) - 0.5 * lam[..., None] * (uR - uL)


def farfield_state(uL, n, rho_inf, v_inf, p_inf, gamma):
    """Riemann-invariant far-field state.  R+ = v_n,L + 2 c_L/(gamma-1) leaves the domain,
    R- = v_n,inf - 2 c_inf/(gamma-1) enters it; tangential velocity and entropy p/rho^gamma
    come from inside on outflow (v_n > 0) and from the free stream on inflow."""
    rL, vL, pL = primitives(uL, gamma)
    cL = torch.sqrt(gamma * pL / rL)
    c_inf = torch.sqrt(gamma * p_inf / rho_inf)
    vnL = (vL * n).sum(-1)
    vn_inf = (v_inf * n).sum(-1)
    Rp = vnL + 2.0 * cL / (gamma - 1.0)
    Rm = vn_inf - 2.0 * c_inf / (gamma - 1.0)
    vn = 0.5 * (Rp + Rm)
    c = 0.25 * (gamma - 1.0) * (Rp - Rm)
    out = vn > 0
    s = torch.where(out, pL / rL ** gamma, p_inf / rho_inf ** gamma)
    vt = torch.where(out[..., None], vL - vnL[..., None] * n, v_inf - vn_inf[..., None] * n)
    rho = (c * c / (gamma * s)) ** (1.0 / (gamma - 1.0))
    p = rho * c * c / gamma
    v = vt + vn[..., None] * n
    E = p / (gamma - 1.0) + 0.5 * rho * (v * v).sum(-1)
    return torch.cat([rho[..., None], rho[..., None] * v, E[..., None]], dim=-1)


def wall_ghost_inviscid(uB):
    """No-slip reflection ghost (rho, -rho v, rho E)."""
    return torch.cat([uB[..., :1], -uB[..., 1:-1], uB[..., -1:]], dim=-1)


def wall_state_viscous(uB):
    """No-slip wall state: velocity zero, same density and internal energy."""
    rho = uB[..., 0]
    ke = 0.5 * (uB[..., 1:-1] ** 2).sum(-1) / rho
    return torch.cat([uB[..., :1], torch.zeros_like(uB[..., 1:-1]), (uB[..., -1] - ke)[..., None]], dim=-1)
