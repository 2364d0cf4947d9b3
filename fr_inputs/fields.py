"""Flow parameters and analytic initial fields (evaluated at caller-given points).

Every field function takes physical coordinates ``x`` of shape ``[..., dim]`` and
returns conserved variables ``[..., dim + 2]`` ordered (rho, rho*u_i, rho*E),
the variable set of the conservation law in the governing-equations section.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FlowParams:
    """Per-mesh free stream and fluid constants (nondimensional).

    Arrays are per mesh: ``rho_inf[n_mesh]``, ``vel_inf[n_mesh, dim]``, ``p_inf[n_mesh]``,
    ``mu[n_mesh]`` (constant dynamic viscosity).  ``gamma`` = 1.4 and ``prandtl`` = 0.71
    as stated under the governing equations.
    """
    dim: int
    rho_inf: np.ndarray
    vel_inf: np.ndarray
    p_inf: np.ndarray
    mu: np.ndarray
    gamma: float = 1.4
    prandtl: float = 0.71
    ldg_beta: float = 0.5
    ldg_tau: float = 0.1

    @property
    def n_mesh(self) -> int:
        return int(len(self.rho_inf))


def freestream_params(dim: int, mach: float, reynolds: float | None, aoa_deg: float = 0.0,
                      n_mesh: int = 1, length: float = 1.0, gamma: float = 1.4) -> FlowParams:
    """rho_inf = |U_inf| = 1, p_inf = 1/(gamma M^2), mu = |U_inf| L / Re (0 if Re is None).
    The angle of attack rotates the free-stream vector in the x-y plane."""
    a = np.deg2rad(aoa_deg)
    v = np.zeros(dim)
    v[0], v[1] = np.cos(a), np.sin(a)
    mu = 0.0 if reynolds is None else length / reynolds
    return FlowParams(dim=dim, rho_inf=np.ones(n_mesh), vel_inf=np.tile(v, (n_mesh, 1)),
                      p_inf=np.full(n_mesh, 1.0 / (gamma * mach * mach)), mu=np.full(n_mesh, mu), gamma=gamma)


def vortex_params(mach: float = 0.15, gamma: float = 1.4) -> FlowParams:
    """Isentropic-vortex convention: rho_inf = p_inf = 1, u_inf = M sqrt(gamma) along x, inviscid."""
    return FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.array([[mach * np.sqrt(gamma), 0.0]]),
                      p_inf=np.ones(1), mu=np.zeros(1), gamma=gamma)


def _cons(rho, vel, p, gamma):
    vel = np.asarray(vel)
    ke = 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, (p / (gamma - 1.0) + ke)[..., None]], axis=-1)


def freestream_state(x: np.ndarray, fp: FlowParams, mesh: int = 0) -> np.ndarray:
    shp = x.shape[:-1]
    rho = np.full(shp, fp.rho_inf[mesh])
    vel = np.broadcast_to(fp.vel_inf[mesh], shp + (fp.dim,))
    p = np.full(shp, fp.p_inf[mesh])
    return _cons(rho, vel, p, fp.gamma)


def vortex_state(x: np.ndarray, t: float = 0.0, beta: float = 5.0, mach: float = 0.15, gamma: float = 1.4,
                 center=(0.0, 0.0), period: float | None = 10.0) -> np.ndarray:
    """Shu's isentropic vortex advected by the free stream: the exact Euler solution
    (on a periodic domain, the nearest periodic image of the centre is used)."""
    uinf = mach * np.sqrt(gamma)
    xc = center[0] + uinf * t
    yc = center[1]
    dx = x[..., 0] - xc
    dy = x[..., 1] - yc
    if period is not None:
        dx = dx - period * np.round(dx / period)
        dy = dy - period * np.round(dy / period)
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    u = uinf - beta / (2 * np.pi) * dy * e
    v = beta / (2 * np.pi) * dx * e
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return _cons(rho, np.stack([u, v], axis=-1), p, gamma)


def entropy_wave_state(x: np.ndarray, t: float = 0.0, vel=(1.0, 1.0), p0: float = 1.0, amp: float = 0.2,
                       period: float = 10.0, gamma: float = 1.4) -> np.ndarray:
    """rho = 1 + amp sin(2 pi (s - |v|-advected)/period) with uniform velocity and pressure:
    an exact Euler solution (density advected by the flow)."""
    d = x.shape[-1]
    vel = np.asarray(vel[:d], float)
    arg = np.zeros(x.shape[:-1])
    for k in range(min(d, 2)):
        arg = arg + (x[..., k] - vel[k] * t)
    rho = 1.0 + amp * np.sin(2 * np.pi * arg / period)
    return _cons(rho, np.broadcast_to(vel, x.shape[:-1] + (d,)), np.full(x.shape[:-1], p0), gamma)


def shear_wave_state(x: np.ndarray, amp: float = 0.1, k: float = 2 * np.pi / 10.0, p0: float = 10.0,
                     gamma: float = 1.4) -> np.ndarray:
    """rho = 1, u_x = amp sin(k y), other velocity components 0, uniform p."""
    d = x.shape[-1]
    vel = np.zeros(x.shape[:-1] + (d,))
    vel[..., 0] = amp * np.sin(k * x[..., 1])
    return _cons(np.ones(x.shape[:-1]), vel, np.full(x.shape[:-1], p0), gamma)


def thermal_wave_state(x: np.ndarray, theta0: float = 1.0, amp: float = 0.1, k: float = 2 * np.pi / 10.0,
                       p0: float = 1.0, gamma: float = 1.4) -> np.ndarray:
    """Fluid at rest with uniform p and p/rho = theta0 + amp sin(k x)."""
    d = x.shape[-1]
    th = theta0 + amp * np.sin(k * x[..., 0])
    return _cons(p0 / th, np.zeros(x.shape[:-1] + (d,)), np.full(x.shape[:-1], p0), gamma)


def noise_like(shape, seed: int, amp: float) -> np.ndarray:
    """Seeded uniform noise in [-amp, amp]."""
    return np.random.default_rng(seed).uniform(-amp, amp, size=shape)


def developed_state(x: np.ndarray, fp: FlowParams, seed: int, amp: float = 0.1, n_modes: int = 4,
                    length: float = 1.0, periods=None, noise: float = 1e-3, mesh=None) -> np.ndarray:
    """Free stream plus a smooth seeded disturbance with the magnitudes of a developed flow: every
    velocity component carries a sum of ``n_modes`` Fourier modes of amplitude ``amp`` |U_inf|
    (wavelengths of order ``length``, integer harmonics along the directions given in ``periods``
    so that periodic meshes see a periodic field), density and pressure carry modes of relative
    size ``amp``/2 and ``amp`` gamma M^2, and every point gets seeded uniform noise of ``noise``
    on the momentum.  Evaluated per mesh (element ranges of ``mesh``) with that mesh's free
    stream.  Points x [..., Ns, dim] with the element axis first when ``mesh`` is given."""
    d = fp.dim
    rng = np.random.default_rng(seed)
    periods = [None] * d if periods is None else list(periods)

    def modes():
        ks, phs = [], []
        for _ in range(n_modes):
            k = np.empty(d)
            for j in range(d):
                if periods[j] is not None:
                    k[j] = 2 * np.pi * rng.integers(-2, 3) / periods[j]
                else:
                    k[j] = 2 * np.pi * rng.uniform(-1.0, 1.0) / length
            ks.append(k)
            phs.append(rng.uniform(0, 2 * np.pi))
        return np.array(ks), np.array(phs)

    def field(xx, ks, phs, a):
        return sum(a[m] * np.sin(xx @ ks[m] + phs[m]) for m in range(len(phs)))

    vel_modes = [modes() for _ in range(d)]
    rho_modes, p_modes = modes(), modes()
    amps = [rng.uniform(0.5, 1.0, n_modes) / np.sqrt(n_modes) for _ in range(d + 2)]
    ranges = [(0, x.shape[0], 0)] if mesh is None else [
        (mesh.mesh_elem_begin[k], mesh.mesh_elem_begin[k + 1], k) for k in range(mesh.n_mesh)]
    out = np.empty(x.shape[:-1] + (d + 2,))
    for lo, hi, k in ranges:
        xx = x[lo:hi]
        U = float(np.linalg.norm(fp.vel_inf[k]))
        M2 = fp.rho_inf[k] * U * U / (fp.gamma * fp.p_inf[k])
        vel = np.empty(xx.shape[:-1] + (d,))
        for j in range(d):
            vel[..., j] = fp.vel_inf[k][j] + amp * U * field(xx, *vel_modes[j], amps[j])
        rho = fp.rho_inf[k] * (1.0 + 0.5 * amp * field(xx, *rho_modes, amps[d]))
        p = fp.p_inf[k] * (1.0 + fp.gamma * M2 * amp * field(xx, *p_modes, amps[d + 1]))
        out[lo:hi] = _cons(rho, vel, p, fp.gamma)
    if noise:
        out[..., 1:-1] += np.random.default_rng(seed + 1000).uniform(-noise, noise, size=out[..., 1:-1].shape)
    return out
