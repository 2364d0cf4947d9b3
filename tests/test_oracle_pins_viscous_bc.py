"""Further pins of the FP64 oracle (CPU only): the terms a closed form with a divergence-free or
resting flow does not reach.

* the dilatation term -(2/3) div v delta_ij of the stress tensor (Eq. (6)): a longitudinal
  velocity wave, whose viscous residual is (4/3) mu times the Laplacian of the velocity
  (Stokes' hypothesis), also along a diagonal so that every stress entry enters;
* the whole Navier-Stokes residual (Eqs. (1)-(7)) against a symbolic derivation of the textbook
  equations written in temperature form, on a general smooth field;
* the Rusanov wave speed max(|v_L.n| + c_L, |v_R.n| + c_R) from hand-computed two-state numbers;
* the Riemann-invariant far-field state away from the free stream, inflow and outflow: R+ from
  inside, R- from the free stream, tangential velocity and entropy from the upwind side;
* the LDG penalty: an exact energy identity (it removes tau_p |N| w |u_L - u_R|^2 per flux
  point), so its sign and size are fixed; the discrete kinetic-energy decay rate of a shear
  layer against its closed form;
* the viscous part of the wall force: a channel flow with a parabolic streamwise profile, a
  wall-normal velocity vanishing on the walls and a linear pressure, whose wall force is known
  in closed form (shear stress, normal viscous stress with the dilatation term, pressure).
"""
import math

import numpy as np
import pytest
import sympy as sp
import torch

import fr_inputs as fi
from oracle import OracleSystem
from oracle.flow import farfield_state, inviscid_flux, rusanov

GAMMA, PR = 1.4, 0.71


def cons(rho, vel, p, gamma=GAMMA):
    """Conserved variables from primitive arrays (Eqs. (2), (5))."""
    ke = 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, (p / (gamma - 1.0) + ke)[..., None]], axis=-1)


def prim(u, gamma=GAMMA):
    """Primitive variables (rho, v, p) of conserved arrays, written out here (Eq. (5))."""
    u = np.asarray(u, float)
    rho = u[..., 0]
    v = u[..., 1:-1] / rho[..., None]
    p = (gamma - 1.0) * (u[..., -1] - 0.5 * rho * np.sum(v * v, axis=-1))
    return rho, v, p


def to_state(x, fn):
    return torch.tensor(fn(x)).permute(0, 2, 1).contiguous()


def flow(dim, mu, tau=0.1, beta=0.5):
    return fi.FlowParams(dim=dim, rho_inf=np.ones(1), vel_inf=np.zeros((1, dim)), p_inf=np.ones(1),
                         mu=np.full(1, float(mu)), ldg_beta=beta, ldg_tau=tau)


# ----------------------------------------------------------------------------- dilatation term
def _longitudinal(khat, A, k):
    khat = np.asarray(khat, float) / np.linalg.norm(khat)

    def field(x):
        phase = k * (x @ khat)
        vel = A * np.sin(phase)[..., None] * khat
        return cons(np.ones(x.shape[:-1]), vel, np.full(x.shape[:-1], 10.0))

    def exact(x, mu):
        """Viscous residual div F_vis: momentum (4/3) mu lap(v) = -(4/3) mu A k^2 khat sin(phase),
        energy div(v.tau) = (4/3) mu A^2 k^2 cos(2 phase); mass 0; heat flux 0 (p/rho uniform)."""
        phase = k * (x @ khat)
        d = x.shape[-1]
        out = np.zeros(x.shape[:-1] + (d + 2,))
        out[..., 1:1 + d] = -(4.0 / 3.0) * mu * A * k * k * np.sin(phase)[..., None] * khat
        out[..., -1] = (4.0 / 3.0) * mu * A * A * k * k * np.cos(2.0 * phase)
        return out
    return field, exact


def _viscous_part_error(dim, n, p, field, exact, mu=0.05):
    """max |(R_NS - R_{mu=0}) - exact| / max |exact| on a curved periodic box: the difference
    removes the inviscid part and the LDG penalty (both independent of mu) and leaves div F_vis."""
    m = fi.periodic_box(dim, n, q=2, curv=0.15, seed=11)
    s_mu = OracleSystem(m, p, flow(dim, mu), equations="ns")
    s_0 = OracleSystem(m, p, flow(dim, 0.0), equations="ns")
    x = s_mu.solpt_coords()
    u = to_state(x, field)
    Rv = s_mu.residual(u) - s_0.residual(u)
    Rex = torch.tensor(exact(x, mu)).permute(0, 2, 1)
    return (Rv - Rex).abs().max().item() / Rex.abs().max().item()


@pytest.mark.parametrize("khat", [(1.0, 0.0), (1.0, 1.0)])
def test_dilatation_term_longitudinal_wave_2d(khat):
    """v = A sin(k.x) khat (div v != 0), rho = 1, uniform p: the viscous residual is
    (4/3) mu lap(v).  A wrong 2/3 (coefficient or sign), a dilatation term missing from one
    normal stress, or a transposed stress entry changes the 4/3 and fails.  The diagonal wave
    brings tau_xy and tau_yy into the momentum balance."""
    k = 2 * np.pi / 10 * np.linalg.norm(khat)
    field, exact = _longitudinal(khat, 0.1, k)
    e1 = _viscous_part_error(2, 8, 4, field, exact)
    e2 = _viscous_part_error(2, 16, 4, field, exact)
    assert e2 < 5e-3 and e1 / e2 > 6.0, (e1, e2)


def test_dilatation_term_longitudinal_wave_3d():
    """The same along the cube diagonal (1, 1, 1): all three normal stresses carry -(2/3) div v."""
    khat = (1.0, 1.0, 1.0)
    k = 2 * np.pi / 10 * np.sqrt(3.0)
    field, exact = _longitudinal(khat, 0.1, k)
    e1 = _viscous_part_error(3, 4, 4, field, exact)
    e2 = _viscous_part_error(3, 8, 4, field, exact)
    assert e2 < 3e-2 and e1 / e2 > 8.0, (e1, e2)


# ----------------------------------------------------------------------------- general residual
def _symbolic_ns_residual(mu, gamma, prandtl):
    """-div(F_inv - F_vis) of the textbook compressible Navier-Stokes equations in temperature
    form (gas constant 1: T = p/rho, c_p = gamma/(gamma-1), Fourier conduction with
    kappa = mu c_p / Pr, Stokes' hypothesis lambda = -2/3 mu), derived by sympy for a smooth
    periodic field on [-5, 5]^2.  Returns numpy functions of (x, y) for the primitive field and
    the exact residual of the four conserved variables."""
    x, y = sp.symbols("x y", real=True)
    w = 2 * sp.pi / 10
    rho = 1 + sp.Rational(1, 10) * sp.sin(w * x) * sp.cos(w * y)
    vx = sp.Rational(3, 10) + sp.Rational(1, 10) * sp.cos(w * (x + y))
    vy = -sp.Rational(1, 5) + sp.Rational(1, 10) * sp.sin(w * (x - 2 * y))
    p = 5 + sp.Rational(1, 5) * sp.cos(w * (2 * x - y))
    V = [vx, vy]
    X = [x, y]
    T = p / rho
    E = p / (gamma - 1) / rho + (vx ** 2 + vy ** 2) / 2
    div = sp.diff(vx, x) + sp.diff(vy, y)
    tau = [[mu * (sp.diff(V[i], X[j]) + sp.diff(V[j], X[i])) - sp.Rational(2, 3) * mu * div * (1 if i == j else 0)
            for j in range(2)] for i in range(2)]
    kappa = mu * gamma / (gamma - 1) / prandtl
    heat = [-kappa * sp.diff(T, X[j]) for j in range(2)]
    # total flux G_j = F_inv,j - F_vis,j for each conserved variable (textbook form)
    G = [[rho * V[j] for j in range(2)]]
    for i in range(2):
        G.append([rho * V[i] * V[j] + (p if i == j else 0) - tau[i][j] for j in range(2)])
    G.append([(rho * E + p) * V[j] - sum(V[i] * tau[i][j] for i in range(2)) + heat[j] for j in range(2)])
    res = [-(sp.diff(Gv[0], x) + sp.diff(Gv[1], y)) for Gv in G]
    prim_f = sp.lambdify((x, y), [rho, vx, vy, p], "numpy")
    res_f = sp.lambdify((x, y), res, "numpy")
    return prim_f, res_f


def _general_residual_error(n, p, prim_f, res_f, mu):
    m = fi.periodic_box(2, n, q=2, curv=0.15, seed=13)
    s = OracleSystem(m, p, flow(2, mu), equations="ns")
    xs = s.solpt_coords()

    def field(x):
        r, a, b, pr = (np.broadcast_to(np.asarray(t, float), x.shape[:-1]) for t in prim_f(x[..., 0], x[..., 1]))
        return cons(r, np.stack([a, b], axis=-1), pr)
    R = s.residual(to_state(xs, field))
    ex = np.stack([np.broadcast_to(np.asarray(t, float), xs.shape[:-1]) for t in res_f(xs[..., 0], xs[..., 1])],
                  axis=-1)
    Rex = torch.tensor(ex).permute(0, 2, 1)
    per_var = ((R - Rex).abs().amax(dim=(0, 2)) / Rex.abs().amax(dim=(0, 2))).numpy()
    return per_var


def test_general_analytic_residual_converges():
    """All of Eqs. (1)-(7) at once (every variable varying, div v != 0, conduction with varying
    density): the FR residual at the solution points converges to the symbolic one at a rate
    above p - 1 in every variable.  A sign or coefficient error anywhere in the fluxes leaves an
    O(1) discrepancy."""
    mu = 0.05
    prim_f, res_f = _symbolic_ns_residual(mu, GAMMA, PR)
    e1 = _general_residual_error(8, 4, prim_f, res_f, mu)
    e2 = _general_residual_error(16, 4, prim_f, res_f, mu)
    rates = np.log2(e1 / e2)
    assert e2.max() < 1e-2 and rates.min() > 3.0, (e1, e2, rates)


# ----------------------------------------------------------------------------- Rusanov wave speed
@pytest.mark.parametrize("case", range(3))
def test_rusanov_wave_speed_hand_computed(case):
    """Rusanov dissipation -1/2 lambda (u_R - u_L) with lambda hand-computed from the two states:
    lambda = max(|v_L.n| + c_L, |v_R.n| + c_R), c = sqrt(gamma p / rho).  Extracted from the mass
    component (whose central flux is written out here) and checked on every component."""
    if case == 0:      # left speed larger, normal along x
        n = [1.0, 0.0]
        L, R = (1.0, [0.5, 0.3], 1.0), (0.8, [-0.2, 0.1], 0.9)
        lam = 0.5 + math.sqrt(1.4 * 1.0 / 1.0)
    elif case == 1:    # right speed larger, negative normal velocities (|.| matters), oblique normal
        n = [0.6, 0.8]
        L, R = (1.2, [0.1, -0.2], 1.0), (0.5, [-0.9, -0.4], 1.1)
        lam = 0.86 + math.sqrt(1.4 * 1.1 / 0.5)           # v_R.n = -0.54 - 0.32
    else:              # 3-D, left side moving against the normal
        n = [0.0, 0.6, -0.8]
        L, R = (0.9, [0.3, -1.0, 0.5], 2.0), (1.1, [0.2, 0.1, 0.1], 1.5)
        lam = 1.0 + math.sqrt(1.4 * 2.0 / 0.9)            # v_L.n = -0.6 - 0.4
    uL = cons(np.array(L[0]), np.array(L[1]), np.array(L[2]))
    uR = cons(np.array(R[0]), np.array(R[1]), np.array(R[2]))
    nn = torch.tensor(n, dtype=torch.float64)
    f = rusanov(torch.tensor(uL)[None], torch.tensor(uR)[None], nn[None], GAMMA)[0].numpy()
    mass_central = 0.5 * (L[0] * np.dot(L[1], n) + R[0] * np.dot(R[1], n))
    lam_oracle = (mass_central - f[0]) / (0.5 * (R[0] - L[0]))
    assert abs(lam_oracle - lam) <= 1e-14 * lam, (lam_oracle, lam)
    fL = (inviscid_flux(torch.tensor(uL), GAMMA) * nn).sum(-1).numpy()
    fR = (inviscid_flux(torch.tensor(uR), GAMMA) * nn).sum(-1).numpy()
    np.testing.assert_allclose(f, 0.5 * (fL + fR) - 0.5 * lam * (uR - uL), rtol=1e-14, atol=1e-14)


# ----------------------------------------------------------------------------- far field
@pytest.mark.parametrize("dim", [2, 3])
def test_far_field_state_off_free_stream(dim):
    """Subsonic characteristic far field with an interior state different from the free stream:
    the returned state carries R+ = v_n + 2c/(gamma-1) of the interior, R- = v_n - 2c/(gamma-1) of
    the free stream, and the tangential velocity and entropy p/rho^gamma of the interior on
    outflow (v_n > 0) and of the free stream on inflow.  Swapped sides, a sign error in R- or the
    wrong entropy fails."""
    rng = np.random.default_rng(17)
    npts = 400
    fp = fi.freestream_params(dim, 0.3, None, aoa_deg=25.0)
    rho_inf, v_inf, p_inf = 1.0, fp.vel_inf[0], fp.p_inf[0]
    nrm = rng.normal(size=(npts, dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    rho = rng.uniform(0.8, 1.25, npts)
    vel = v_inf + rng.normal(size=(npts, dim)) * 0.3
    p = p_inf * rng.uniform(0.85, 1.2, npts)
    uL = cons(rho, vel, p)
    ub = farfield_state(torch.tensor(uL), torch.tensor(nrm), torch.tensor(rho_inf), torch.tensor(v_inf),
                        torch.tensor(p_inf), GAMMA).numpy()
    rb, vb, pb = prim(ub)
    cb, cL, c_inf = np.sqrt(GAMMA * pb / rb), np.sqrt(GAMMA * p / rho), math.sqrt(GAMMA * p_inf / rho_inf)
    vnb, vnL, vn_inf = (vb * nrm).sum(1), (vel * nrm).sum(1), nrm @ v_inf
    g1 = GAMMA - 1.0
    assert np.all(np.abs(vnb) < cb)                                     # subsonic cases only
    np.testing.assert_allclose(vnb + 2 * cb / g1, vnL + 2 * cL / g1, rtol=1e-13)
    np.testing.assert_allclose(vnb - 2 * cb / g1, vn_inf - 2 * c_inf / g1, rtol=1e-13)
    out = vnb > 0
    assert 50 < out.sum() < npts - 50                                   # both directions occur
    vt = lambda v, vn: v - vn[:, None] * nrm                            # noqa: E731
    np.testing.assert_allclose(vt(vb, vnb)[out], vt(vel, vnL)[out], atol=1e-13)
    np.testing.assert_allclose(vt(vb, vnb)[~out], vt(np.tile(v_inf, (npts, 1)), np.full(npts, 0.0) + vn_inf)[~out],
                               atol=1e-13)
    np.testing.assert_allclose((pb / rb ** GAMMA)[out], (p / rho ** GAMMA)[out], rtol=1e-13)
    np.testing.assert_allclose((pb / rb ** GAMMA)[~out], p_inf / rho_inf ** GAMMA, rtol=1e-13)


# ----------------------------------------------------------------------------- LDG penalty
@pytest.mark.parametrize("dim,tau", [(2, 0.1), (2, 0.37), (3, 0.1)])
def test_ldg_penalty_energy_identity(dim, tau):
    """With mu = 0 the viscous flux vanishes and R_NS - R_Euler is the penalty term alone.  With
    Gauss points and g_DG (FR = nodal DG), its contribution to d/dt of the discrete L2 energy
    sum_e sum_i w_i J_i |u_i|^2 / 2 is exactly -tau_p sum_pairs w_f |N_f| |u_L - u_R|^2 <= 0:
    the penalty is dissipative, of size tau_p, and acts on the jump of the traces."""
    m = fi.periodic_box(dim, 4 if dim == 2 else 2, q=2, curv=0.2, seed=6)
    fp_ns = fi.freestream_params(dim, 0.3, None)
    fp_ns.ldg_tau = tau
    s_ns = OracleSystem(m, 3 if dim == 2 else 2, fp_ns, equations="ns")
    s_eu = OracleSystem(m, 3 if dim == 2 else 2, fp_ns, equations="euler")
    u = to_state(s_ns.solpt_coords(), lambda x: fi.freestream_state(x, fp_ns))
    u = u * (1.0 + torch.tensor(fi.noise_like(u.shape, 3, 0.05)))
    Rp = s_ns.residual(u) - s_eu.residual(u)
    lhs = float(torch.einsum('i,ei,evi->', s_ns.sol_w, s_ns.geo["J"], u * Rp))
    uf = torch.einsum('fs,evs->evf', s_ns.M0, u)
    jump = uf[s_ns.eL, :, s_ns.fL] - uf[s_ns.eR, :, s_ns.fR]
    wN = s_ns.fpt_w[s_ns.fL] * s_ns.geo["magN"][s_ns.eL, s_ns.fL]
    rhs = -tau * float((wN[:, None] * jump * jump).sum())
    assert rhs < 0 and abs(lhs - rhs) <= 1e-11 * abs(rhs), (lhs, rhs)


def test_kinetic_energy_decay_rate_of_shear_layer():
    """Shear layer u_x = A sin(k y), rho = 1, uniform p (div v = 0, no pressure work): the kinetic
    energy decays at d/dt int rho |v|^2 / 2 = -mu int |du_x/dy|^2 = -mu A^2 k^2 |Omega| / 2.  The
    discrete rate sum w J (v . R_mom - |v|^2 R_rho / 2) converges to it; over a few RK4 steps (at an
    acoustic CFL number below one) the discrete kinetic energy falls monotonically."""
    A, k, mu = 0.1, 2 * np.pi / 10, 0.05
    exact = -mu * A * A * k * k * 100.0 / 2.0
    rates = []
    for n in (4, 8):
        m = fi.periodic_box(2, n, q=2, curv=0.1, seed=4)
        s = OracleSystem(m, 4, flow(2, mu), equations="ns")
        u = to_state(s.solpt_coords(), lambda x: fi.shear_wave_state(x, amp=A, k=k))
        R = s.residual(u)
        v = u[:, 1:3] / u[:, :1]
        dke = (v * R[:, 1:3]).sum(1) - 0.5 * (v * v).sum(1) * R[:, 0]
        rates.append(float(torch.einsum('i,ei,ei->', s.sol_w, s.geo["J"], dke)))
    errs = [abs(r - exact) / abs(exact) for r in rates]
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 8.0, (rates, exact)
    ke = []
    for _ in range(4):
        ke.append(float(torch.einsum('i,ei,ei->', s.sol_w, s.geo["J"],
                                     0.5 * (u[:, 1:3] ** 2).sum(1) / u[:, 0])))
        u = s.rk4_step(u, torch.tensor([0.01], dtype=torch.float64))
    assert all(b < a for a, b in zip(ke, ke[1:])), ke


# ----------------------------------------------------------------------------- viscous wall force
@pytest.mark.parametrize("dim", [2, 3])
def test_wall_force_channel_closed_form(dim):
    """Channel between adiabatic no-slip walls at y = -h and y = +h (periodic in x, and z in 3-D),
    rho = 1, v_x = U (1 - y^2/h^2), v_y = c (y^2 - h^2), p = p0 + b y: no slip holds exactly and
    every field is a polynomial of degree <= 4 in y, so at p = 4 the wall gradient is exact.  The
    force on the walls (fluid element's outward normal n, which points into the wall) is
        F_x = 2 * (2 mu U / h) * area,            shear stress on both walls, downstream,
        F_y = 2 b h area - 2 * (8/3) mu c h area, pressure difference and normal viscous stress
                                                  tau_yy = mu (2 - 2/3) dv_y/dy on each wall,
    with area = L_x (L_z) the area of one wall."""
    U, c, p0, b, mu = 0.2, 0.03, 7.0, 0.01, 0.02
    h, Lx = 5.0, 10.0
    area = Lx if dim == 2 else Lx * Lx
    m = fi.periodic_box(dim, 3 if dim == 2 else 2, q=1, bc="channel")
    s = OracleSystem(m, 4, flow(dim, mu), equations="ns")

    def field(x):
        y = x[..., 1]
        vel = np.zeros(x.shape[:-1] + (dim,))
        vel[..., 0] = U * (1.0 - y * y / (h * h))
        vel[..., 1] = c * (y * y - h * h)
        return cons(np.ones(x.shape[:-1]), vel, p0 + b * y)
    F = s.wall_force(to_state(s.solpt_coords(), field))[0].numpy()
    Fx = 2.0 * (2.0 * mu * U / h) * area
    Fy = 2.0 * b * h * area - 2.0 * (8.0 / 3.0) * mu * c * h * area
    expect = np.zeros(dim)
    expect[0], expect[1] = Fx, Fy
    np.testing.assert_allclose(F, expect, rtol=1e-11, atol=1e-12 * p0 * area)
