"""Pins of the FP64 oracle against facts fixed outside it (closed forms, invariants,
textbook routines).  CPU only.

Each test names what pins it.  A plausible mistake in the oracle (wrong sign of a
viscous term, a transposed metric, a dropped correction term, a wrong face pairing)
fails at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.interpolate
import torch

import fr_inputs as fi
from oracle import OracleSystem, TensorOps, correction_deriv, cumulative_prms, oaspl_from_series
from oracle.flow import farfield_state, inviscid_flux, rusanov

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def state_at(sys_, fn, **kw):
    x = sys_.solpt_coords()
    return torch.tensor(fn(x, **kw)).permute(0, 2, 1).contiguous()


# ----------------------------------------------------------------------------- operators
@pytest.mark.parametrize("p", [1, 2])
def test_gauss_points_closed_form(p):
    """Gauss-Legendre nodes/weights for 2 and 3 points are known in closed form."""
    ops = TensorOps(1, p)
    if p == 1:
        np.testing.assert_allclose(ops.xi, [-1 / np.sqrt(3), 1 / np.sqrt(3)], atol=1e-15)
        np.testing.assert_allclose(ops.w, [1, 1], atol=1e-15)
    else:
        np.testing.assert_allclose(ops.xi, [-np.sqrt(0.6), 0, np.sqrt(0.6)], atol=1e-15)
        np.testing.assert_allclose(ops.w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gdg_equals_dg_lifting(p):
    """Huynh's g_DG makes FR identical to nodal DG: g_R'(xi_i) = l_i(1) / w_i (collocated
    Gauss points, diagonal mass matrix).  l_i(1) from scipy's Lagrange interpolation."""
    xi, w = np.polynomial.legendre.leggauss(p + 1)
    li1 = np.array([scipy.interpolate.lagrange(xi, np.eye(p + 1)[i])(1.0) for i in range(p + 1)])
    np.testing.assert_allclose(correction_deriv(p, xi), li1 / w, rtol=1e-10, atol=1e-11)
    # boundary values of g_R: 1 at +1, 0 at -1
    leg = np.polynomial.legendre.Legendre
    g = 0.5 * (leg.basis(p + 1) + leg.basis(p))
    assert abs(g(1.0) - 1) < 1e-14 and abs(g(-1.0)) < 1e-14


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2), (2, 4)])
def test_tensor_operators_exact_on_polynomials(dim, p):
    """D_k differentiates and M0 interpolates any tensor polynomial of degree <= p exactly;
    rows of D_k sum to zero."""
    ops = TensorOps(dim, p)
    rng = np.random.default_rng(0)
    C = rng.normal(size=(p + 1,) * dim)

    def poly(x, deriv=None):
        out = np.zeros(len(x))
        for idx in np.ndindex(C.shape):
            term = np.full(len(x), C[idx])
            for k in range(dim):
                e = idx[k]
                if deriv == k:
                    term *= e * x[:, k] ** max(e - 1, 0) if e > 0 else 0.0
                else:
                    term *= x[:, k] ** e
            out += term
        return out
    xs = ops.ref_solpts()
    xf = ops.ref_fpts()
    u = poly(xs)
    for k in range(dim):
        np.testing.assert_allclose(ops.Dk[k] @ u, poly(xs, deriv=k), atol=1e-10 * np.abs(C).sum() * p * p)
        np.testing.assert_allclose(ops.Dk[k].sum(axis=1), 0.0, atol=1e-12)
    np.testing.assert_allclose(ops.M0 @ u, poly(xf), atol=1e-11 * np.abs(C).sum())


# ----------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("dim,eq", [(2, "euler"), (2, "ns"), (3, "ns")])
def test_freestream_preservation_curved_periodic(dim, eq):
    """A uniform flow is an exact solution: the residual vanishes on curved elements when
    the metric identities hold discretely."""
    m = fi.periodic_box(dim, 4 if dim == 2 else 3, q=2, curv=0.25, seed=3)
    fp = fi.freestream_params(dim, 0.2, 100.0 if eq == "ns" else None, aoa_deg=20.0)
    s = OracleSystem(m, 3 if dim == 2 else 2, fp, equations=eq)
    R = s.residual(state_at(s, fi.freestream_state, fp=fp))
    assert R.abs().max().item() < 1e-11 * fp.p_inf[0]


def test_freestream_preservation_ogrid_farfield():
    """Perturbed curved O-grid with characteristic far field on both rings: R(u_inf) = 0."""
    m = fi.o_grid(12, 6, q=4, r1=8.0, wall="farfield", seed=5)
    fp = fi.freestream_params(2, 0.2, 1000.0)
    s = OracleSystem(m, 4, fp, equations="ns")
    R = s.residual(state_at(s, fi.freestream_state, fp=fp))
    assert R.abs().max().item() < 1e-11 * fp.p_inf[0]


@pytest.mark.parametrize("dim,eq", [(2, "euler"), (2, "ns"), (3, "ns")])
def test_discrete_conservation_periodic(dim, eq):
    """On a periodic mesh the common fluxes cancel pairwise: sum_e sum_i w_i J_i R_i = 0 for
    mass, momentum and energy, to round-off."""
    m = fi.periodic_box(dim, 4 if dim == 2 else 3, q=2, curv=0.2, seed=1)
    fp = fi.freestream_params(dim, 0.3, 50.0 if eq == "ns" else None)
    s = OracleSystem(m, 3 if dim == 2 else 2, fp, equations=eq)
    u = state_at(s, fi.freestream_state, fp=fp)
    u = u * (1.0 + torch.tensor(fi.noise_like(u.shape, 7, 0.05)))
    R = s.residual(u)
    tot = s.integrate(R)
    scale = s.integrate(R.abs())
    assert (tot.abs() / scale).max().item() < 1e-12


def test_closed_adiabatic_channel_conserves_mass_and_energy():
    """Periodic channel with adiabatic no-slip walls: wall mass and energy fluxes are exactly
    zero (reflection ghost; zero wall velocity; zero normal heat flux), so total mass and
    energy are conserved to round-off while momentum is not."""
    m = fi.periodic_box(2, 4, q=2, curv=0.15, bc="channel", seed=2)
    fp = fi.freestream_params(2, 0.3, 30.0)
    s = OracleSystem(m, 3, fp, equations="ns")
    u = state_at(s, fi.freestream_state, fp=fp)
    u = u * (1.0 + torch.tensor(fi.noise_like(u.shape, 9, 0.05)))
    R, aux = s.residual(u, aux=True)
    tot = s.integrate(R)
    scale = s.integrate(R.abs())
    assert abs(tot[0] / scale[0]) < 1e-12 and abs(tot[-1] / scale[-1]) < 1e-12
    assert abs(tot[1] / scale[1]) > 1e-6  # walls exert a force
    Fh = aux["Fhat"][s.bE, :, s.bF]
    assert Fh[:, 0].abs().max() < 1e-13 and Fh[:, -1].abs().max() < 1e-12


def test_rusanov_consistency_and_far_field_identity():
    """Rusanov(u, u, n) = F(u).n; Rusanov(uL, uR, n) = -Rusanov(uR, uL, -n); the
    Riemann-invariant far-field state of u_inf is u_inf."""
    rng = np.random.default_rng(4)
    for d in (2, 3):
        u = torch.tensor(np.concatenate([rng.uniform(0.5, 2, (50, 1)), rng.normal(size=(50, d)),
                                         rng.uniform(20, 30, (50, 1))], axis=1))
        u2 = u.flip(0)
        n = torch.tensor(rng.normal(size=(50, d)))
        n = n / n.norm(dim=1, keepdim=True)
        f = (inviscid_flux(u, 1.4) * n[:, None, :]).sum(-1)
        assert torch.allclose(rusanov(u, u, n, 1.4), f, rtol=1e-14, atol=1e-12)
        assert torch.allclose(rusanov(u, u2, n, 1.4), -rusanov(u2, u, -n, 1.4), rtol=1e-14, atol=1e-12)
        fp = fi.freestream_params(d, 0.2, None, aoa_deg=30.0)
        uinf = torch.tensor(fi.freestream_state(np.zeros((50, d)), fp))
        ub = farfield_state(uinf, n, torch.tensor(1.0), torch.tensor(fp.vel_inf[0]), torch.tensor(fp.p_inf[0]), 1.4)
        assert torch.allclose(ub, uinf, rtol=1e-13, atol=1e-13)


# ----------------------------------------------------------------------------- closed forms
def _l2(sys_, v):
    return torch.sqrt(sys_.integrate(v * v)).max().item()


def test_entropy_wave_order():
    """Density wave advected by a uniform flow is an exact Euler solution; the FR error
    after a fixed time converges at order ~ p+1 under mesh refinement."""
    p, T = 2, 0.5
    errs = []
    for n in (4, 8, 16):
        m = fi.periodic_box(2, n, q=2, curv=0.1, seed=1)
        fp = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.ones((1, 2)), p_inf=np.ones(1), mu=np.zeros(1))
        s = OracleSystem(m, p, fp, equations="euler")
        u = state_at(s, fi.entropy_wave_state)
        nst = 25
        u, _, _ = s.run(u, torch.tensor([T / nst], dtype=torch.float64), nst, sample_every=0)
        ue = state_at(s, fi.entropy_wave_state, t=T)
        errs.append(_l2(s, u - ue))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 0.5 and rates.min() > p, (errs, rates)


def test_isentropic_vortex_closed_form():
    """The cfg-0 problem: Shu vortex (beta 5, M 0.15) on a 32x32 periodic [-5,5]^2 mesh at
    p = 3, 20 RK4 steps of dt = 2.12e-3; the solution stays within the periodic-truncation
    floor of the translated closed form."""
    m = fi.periodic_box(2, 32, q=1)
    fp = fi.vortex_params()
    s = OracleSystem(m, 3, fp, equations="euler")
    u = state_at(s, fi.vortex_state)
    dt = 2.120e-3
    u, _, _ = s.run(u, torch.tensor([dt], dtype=torch.float64), 20, sample_every=0)
    ue = state_at(s, fi.vortex_state, t=20 * dt)
    err = (u - ue).abs().max().item()
    assert err < 1e-4, err


def _ns_residual_error(n, p, field, exact, curv=0.15):
    m = fi.periodic_box(2, n, q=2, curv=curv, seed=11)
    mu = 0.05
    fp = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.zeros((1, 2)), p_inf=np.ones(1), mu=np.full(1, mu))
    s = OracleSystem(m, p, fp, equations="ns")
    R = s.residual(state_at(s, field))
    x = s.solpt_coords()
    Rex = torch.tensor(exact(x, mu, fp.gamma, fp.prandtl)).permute(0, 2, 1)
    return (R - Rex).abs().max().item() / Rex.abs().max().item()


def test_viscous_shear_wave_closed_form():
    """u_x = A sin(k y), rho = 1, uniform p: exact residual R_mom_x = -mu k^2 A sin(k y),
    R_E = mu A^2 k^2 cos(2 k y), others 0 (pins the sign of tau and of u_i tau_ij)."""
    A, k = 0.1, 2 * np.pi / 10

    def exact(x, mu, g, Pr):
        y = x[..., 1]
        out = np.zeros(x.shape[:-1] + (4,))
        out[..., 1] = -mu * k * k * A * np.sin(k * y)
        out[..., 3] = mu * A * A * k * k * np.cos(2 * k * y)
        return out
    e1 = _ns_residual_error(8, 4, lambda x: fi.shear_wave_state(x, amp=A, k=k), exact)
    e2 = _ns_residual_error(16, 4, lambda x: fi.shear_wave_state(x, amp=A, k=k), exact)
    assert e2 < 5e-3 and e1 / e2 > 6.0, (e1, e2)


def test_heat_conduction_closed_form():
    """Fluid at rest, uniform p, p/rho = th0 + a sin(k x): R_E = -mu g/(Pr (g-1)) a k^2 sin(k x)
    (pins the heat-flux reading of Eq. (7)); mass and momentum residuals vanish."""
    a, k = 0.1, 2 * np.pi / 10

    def exact(x, mu, g, Pr):
        out = np.zeros(x.shape[:-1] + (4,))
        out[..., 3] = -mu * g / (Pr * (g - 1)) * a * k * k * np.sin(k * x[..., 0])
        return out
    e1 = _ns_residual_error(8, 4, lambda x: fi.thermal_wave_state(x, amp=a, k=k), exact)
    e2 = _ns_residual_error(16, 4, lambda x: fi.thermal_wave_state(x, amp=a, k=k), exact)
    assert e2 < 5e-3 and e1 / e2 > 6.0, (e1, e2)


def test_rk4_temporal_order():
    """Classical RK4: error against a dt/8 reference falls by ~16 when dt halves."""
    m = fi.periodic_box(2, 4, q=1)
    fp = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.ones((1, 2)), p_inf=np.ones(1), mu=np.zeros(1))
    s = OracleSystem(m, 2, fp, equations="euler")
    u0 = state_at(s, fi.entropy_wave_state, amp=0.3)
    T, n = 1.0, 16
    ref, _, _ = s.run(u0, torch.tensor([T / (8 * n)], dtype=torch.float64), 8 * n, sample_every=0)
    e = []
    for mult in (1, 2):
        u, _, _ = s.run(u0, torch.tensor([T / (mult * n)], dtype=torch.float64), mult * n, sample_every=0)
        e.append((u - ref).abs().max().item())
    assert 12.0 < e[0] / e[1] < 20.0, e


# ----------------------------------------------------------------------------- probes, forces, OASPL
def test_probe_interpolation_exact_for_linear_field():
    """On affine elements the tensor Lagrange interpolant reproduces a linear field exactly at
    the probe, and Eq. (5) then gives the pressure of that state."""
    m = fi.periodic_box(2, 5, q=1)
    fp = fi.vortex_params()
    xp = np.array([[0.37, -1.91], [2.0, 2.0]])
    s = OracleSystem(m, 3, fp, equations="euler", probes=xp)

    def lin(x):
        out = np.zeros(x.shape[:-1] + (4,))
        out[..., 0] = 1 + 0.01 * x[..., 0] + 0.02 * x[..., 1]
        out[..., 1] = 0.1 - 0.03 * x[..., 1]
        out[..., 2] = 0.05 * x[..., 0]
        out[..., 3] = 3.0 + 0.1 * x[..., 0]
        return out
    u = state_at(s, lin)
    ue = lin(xp)
    pex = 0.4 * (ue[:, 3] - 0.5 * (ue[:, 1] ** 2 + ue[:, 2] ** 2) / ue[:, 0])
    np.testing.assert_allclose(s.probe_pressure(u).numpy(), pex, rtol=1e-13)


def test_uniform_pressure_gives_zero_force_on_closed_body():
    """Fluid at rest with uniform p around the cylinder: the closed-surface integral of p n
    vanishes and the viscous stress is zero, so the wall force is zero."""
    m = fi.o_grid(16, 4, q=4, r1=5.0, seed=2)
    fp = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.zeros((1, 2)), p_inf=np.full(1, 17.857), mu=np.full(1, 1e-3))
    s = OracleSystem(m, 4, fp, equations="ns")
    u = state_at(s, fi.freestream_state, fp=fp)
    F = s.wall_force(u)
    assert F.abs().max().item() < 1e-12 * 17.857
    # while a uniform flow past it is not force free through the pressure term alone
    # (sanity that the integral is not identically zero): half-body pressure integral
    geo = s.geo
    wall = s.bT == 1
    n = geo["n"][s.bE[wall], s.bF[wall]]
    assert n[:, 0].abs().max() > 0.9


def test_oaspl_closed_forms_golden():
    """Eqs. (9)-(12): pure tones over whole periods (tests/golden/oaspl_closed_forms.txt)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "oaspl_closed_forms.txt"))
    for p0, A, pref, spp, per, prms, db in rows:
        t = np.arange(int(spp * per)) / spp
        sig = p0 + A * np.sin(2 * np.pi * t)
        assert abs(cumulative_prms(sig)[-1] - prms) < 1e-12 * max(1.0, p0)
        assert abs(oaspl_from_series(sig, pref) - db) < 1e-9


def test_cumulative_vector_matches_numpy_std_and_constant_is_minus_inf():
    """Element k of the cumulative p_RMS vector is the population std of the first k samples."""
    rng = np.random.default_rng(0)
    sig = 17.0 + rng.normal(size=200) * 1e-3
    c = cumulative_prms(sig)
    for k in (1, 2, 17, 200):
        assert abs(c[k - 1] - np.std(sig[:k], ddof=0)) < 1e-13
    assert oaspl_from_series(np.full(10, 3.0), 2e-5) == -np.inf


# ----------------------------------------------------------------------------- error paths
def test_unmatched_face_and_inverted_element_raise():
    m = fi.periodic_box(2, 3, q=1)
    m.periodic_vec = m.periodic_vec[:1]            # y-sides no longer identified
    with pytest.raises(ValueError, match="unmatched"):
        OracleSystem(m, 2, fi.vortex_params(), equations="euler")
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    m.elem_nodes[0] = m.elem_nodes[0][[1, 0, 3, 2]]  # mirror one element
    with pytest.raises(ValueError, match="Jacobian"):
        OracleSystem(m, 2, fi.vortex_params(), equations="euler")
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    with pytest.raises(ValueError, match="outside"):
        OracleSystem(m, 2, fi.vortex_params(), equations="euler", probes=[[50.0, 0.0]])


@pytest.mark.parametrize("kind", ["cavities", "periodic_cgrids"])
def test_batched_meshes_equal_separate_solves(kind):
    """Concatenated independent meshes (a poll's designs) evolve exactly as separate solves, even
    when their geometries overlap in space (faces never pair across meshes), also for spanwise
    periodic meshes sharing their period."""
    if kind == "cavities":
        ms = [fi.cavity(a, h=0.5, q=2, upstream=2.0, top=3.0, outflow=3.0, top_buffer=1.0, out_buffer=1.0)
              for a in (1.5, 2.5)]
        fps = [fi.freestream_params(2, 0.15, 1500.0), fi.freestream_params(2, 0.2, 1000.0, aoa_deg=5.0)]
    else:
        g = dict(n_wake=2, n_foil=6, n_normal=2, n_span=2, q=2, r_out=4.0, x_out=6.0, h_wall=0.05)
        ms = [fi.c_grid_naca(camber=c, thickness=t, **g) for c, t in ((0.0, 0.12), (0.03, 0.09))]
        fps = [fi.freestream_params(3, 0.2, 23000.0, aoa_deg=a) for a in (2.0, 5.0)]
    batch = fi.concat_meshes(ms)
    fpb = fi.FlowParams(dim=2, rho_inf=np.concatenate([f.rho_inf for f in fps]),
                        vel_inf=np.concatenate([f.vel_inf for f in fps]),
                        p_inf=np.concatenate([f.p_inf for f in fps]), mu=np.concatenate([f.mu for f in fps]))
    pdeg = 3 if kind == "cavities" else 2
    sb = OracleSystem(batch, pdeg, fpb, equations="ns")
    parts = []
    for m, f in zip(ms, fps):
        s = OracleSystem(m, pdeg, f, equations="ns")
        u = state_at(s, fi.freestream_state, fp=f)
        u = u * (1.0 + torch.tensor(fi.noise_like(u.shape, 4, 0.01)))
        parts.append((s, u))
    ub = torch.cat([u for _, u in parts])
    Rb = sb.residual(ub)
    Rs = torch.cat([s.residual(u) for s, u in parts])
    assert torch.allclose(Rb, Rs, rtol=1e-13, atol=1e-12 * Rs.abs().max().item())


@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_oracle_gradient_matches_central_differences(eq):
    """The oracle gradient (reverse-mode autograd through the FP64 residual) agrees with central
    finite differences along seeded directions: <J^T r, v> = <r, (R(u + e v) - R(u - e v)) / 2e>."""
    m = fi.o_grid(8, 3, q=2, r1=4.0, stretch=1.3, seed=4, wall="wall" if eq == "ns" else "farfield")
    fp = fi.freestream_params(2, 0.3, 100.0 if eq == "ns" else None, aoa_deg=10.0)
    s = OracleSystem(m, 2, fp, equations=eq)
    u0 = state_at(s, fi.freestream_state, fp=fp)
    rng = np.random.default_rng(8)
    u0 = u0 * (1.0 + torch.tensor(rng.uniform(-0.02, 0.02, u0.shape)))
    r = torch.tensor(rng.normal(size=u0.shape))
    u = u0.clone().requires_grad_(True)
    (s.residual(u) * r).sum().backward()
    for _ in range(3):
        v = torch.tensor(rng.normal(size=u0.shape)) * u0.abs().mean()
        eps = 1e-6
        fd = ((s.residual(u0 + eps * v) - s.residual(u0 - eps * v)) * r).sum() / (2 * eps)
        ad = (u.grad * v).sum()
        assert abs(float(fd - ad)) <= 1e-6 * abs(float(ad)), (float(fd), float(ad))


# ----------------------------------------------------------------------------- mesh-node gradient
def _node_case(kind):
    if kind == "euler_periodic":
        m = fi.periodic_box(2, 3, q=2, curv=0.2, seed=3)
        fp = fi.freestream_params(2, 0.3, None, aoa_deg=20.0)
        return m, 2, fp, "euler"
    if kind == "ns_ogrid":
        m = fi.o_grid(8, 3, q=2, r1=4.0, stretch=1.3, seed=4)
        fp = fi.freestream_params(2, 0.3, 100.0, aoa_deg=10.0)
        return m, 2, fp, "ns"
    m = fi.periodic_box(3, 2, q=2, curv=0.15, seed=5, bc="farfield")
    fp = fi.freestream_params(3, 0.3, 100.0, aoa_deg=15.0)
    return m, 2, fp, "ns"


def _node_grad(m, p, fp, eq, u0, r, probes=None):
    X = torch.tensor(m.node_xyz, dtype=torch.float64, requires_grad=True)
    s = OracleSystem(m, p, fp, equations=eq, node_xyz=X, probes=probes)
    val = (s.residual(u0) * r).sum()
    val.backward()
    return s, X.grad.clone(), float(val.detach())


def _noisy_state(s, fp, seed):
    u0 = state_at(s, fi.freestream_state, fp=fp)
    rng = np.random.default_rng(seed)
    return u0 * (1.0 + torch.tensor(rng.uniform(-0.02, 0.02, u0.shape))), rng


@pytest.mark.parametrize("kind", ["euler_periodic", "ns_ogrid", "ns_box3d_farfield"])
def test_node_gradient_translation_and_scaling_invariants(kind):
    """The residual does not depend on where the mesh sits (sum of node adjoints = 0), and it is
    homogeneous in the node coordinates: the inviscid and penalty parts scale as 1/lambda and the
    mu-proportional viscous part as 1/lambda^2 under X -> lambda X, so by Euler's theorem
    sum_n X_n . X_bar_n = -r.R(mu = 0) - 2 r.(R(mu) - R(mu = 0))."""
    m, p, fp, eq = _node_case(kind)
    s0 = OracleSystem(m, p, fp, equations=eq)
    u0, rng = _noisy_state(s0, fp, 12)
    r = torch.tensor(rng.normal(size=u0.shape))
    s, g, _ = _node_grad(m, p, fp, eq, u0, r)
    scale = float(g.abs().max())
    assert float(g.sum(dim=0).abs().max()) <= 1e-11 * scale * g.shape[0] ** 0.5
    lhs = float((torch.tensor(m.node_xyz) * g).sum())
    R = s0.residual(u0)
    if eq == "euler":
        rhs = -float((r * R).sum())
    else:
        fp0 = fi.freestream_params(fp.dim, 0.3, None, aoa_deg=0.0)
        fp0.rho_inf, fp0.vel_inf, fp0.p_inf = fp.rho_inf, fp.vel_inf, fp.p_inf
        fp0.mu = np.zeros_like(np.asarray(fp.mu, float))
        R0 = OracleSystem(m, p, fp0, equations="ns").residual(u0)
        rhs = -float((r * R0).sum()) - 2.0 * float((r * (R - R0)).sum())
    assert abs(lhs - rhs) <= 1e-9 * max(abs(rhs), float((r * R).abs().sum())), (lhs, rhs)


def test_node_gradient_zero_at_free_stream_on_curved_farfield_mesh():
    """A uniform state is preserved on every conforming curved mesh of degree q <= p with far-field
    boundaries, R(X) = 0 for all such X, so its node gradient vanishes.  (On a periodic box a
    single boundary node moved without its periodic image breaks conformity, so that mesh does
    not qualify.)"""
    m = fi.o_grid(8, 3, q=2, r1=4.0, stretch=1.3, seed=4, wall="farfield")
    fp = fi.freestream_params(2, 0.3, 100.0, aoa_deg=10.0)
    p = 2
    s0 = OracleSystem(m, p, fp, equations="ns")
    u0 = state_at(s0, fi.freestream_state, fp=fp)
    r = torch.tensor(np.random.default_rng(3).normal(size=u0.shape))
    _, g, _ = _node_grad(m, p, fp, "ns", u0, r)
    assert float(g.abs().max()) <= 1e-10 * float(u0.abs().max())


@pytest.mark.parametrize("kind", ["euler_periodic", "ns_ogrid", "ns_box3d_farfield"])
def test_node_gradient_matches_central_differences(kind):
    """<X_bar, V> against central differences of r . R(X + e V) along seeded node directions
    (metrics recomputed from the perturbed nodes, face pairing kept)."""
    m, p, fp, eq = _node_case(kind)
    s0 = OracleSystem(m, p, fp, equations=eq)
    u0, rng = _noisy_state(s0, fp, 13)
    r = torch.tensor(rng.normal(size=u0.shape))
    _, g, _ = _node_grad(m, p, fp, eq, u0, r)
    h = float(np.ptp(m.node_xyz, axis=0).max()) / 50.0
    for _ in range(2):
        V = rng.normal(size=m.node_xyz.shape) * h
        eps = 1e-6
        vals = []
        for sg in (1.0, -1.0):
            s0.set_nodes(torch.tensor(m.node_xyz + sg * eps * V))
            vals.append(float((s0.residual(u0) * r).sum()))
        fd = (vals[0] - vals[1]) / (2 * eps)
        ad = float((g * torch.tensor(V)).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8), (fd, ad)


def test_probe_node_gradient_matches_relocated_probe():
    """The probe pressure's node gradient (one differentiable Newton correction) against central
    differences in which the probe is located afresh (Newton from scratch) on each perturbed mesh."""
    m = fi.o_grid(8, 3, q=2, r1=4.0, stretch=1.3, seed=4)
    fp = fi.freestream_params(2, 0.3, 100.0, aoa_deg=10.0)
    probe = np.array([[0.3, 1.1]])
    s0 = OracleSystem(m, 2, fp, equations="ns", probes=probe)
    x = s0.solpt_coords()
    rng = np.random.default_rng(21)
    u0 = state_at(s0, fi.freestream_state, fp=fp)
    u0 = u0 + 0.05 * torch.tensor(np.sin(3 * x[..., 0] + 2 * x[..., 1]))[:, None, :] * u0.abs().mean(dim=(0, 2))[None, :, None]
    X = torch.tensor(m.node_xyz, dtype=torch.float64, requires_grad=True)
    s = OracleSystem(m, 2, fp, equations="ns", node_xyz=X, probes=probe)
    s.probe_pressure(u0).sum().backward()
    g = X.grad
    assert float(g.abs().max()) > 0
    h = 0.02
    for _ in range(3):
        V = rng.normal(size=m.node_xyz.shape) * h
        eps = 1e-6
        vals = []
        for sg in (1.0, -1.0):
            mm = fi.MeshDesc(dim=2, q=m.q, node_xyz=m.node_xyz + sg * eps * V, elem_nodes=m.elem_nodes,
                             face_bc=m.face_bc, periodic_vec=m.periodic_vec, mesh_elem_begin=m.mesh_elem_begin)
            vals.append(float(OracleSystem(mm, 2, fp, equations="ns", probes=probe).probe_pressure(u0).sum()))
        fd = (vals[0] - vals[1]) / (2 * eps)
        ad = float((g * torch.tensor(V)).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-6), (fd, ad)


# ----------------------------------------------------------------------------- observer statistics
def test_welch_psd_matches_scipy_and_tone_closed_form():
    """The oracle's Welch PSD equals scipy.signal.welch with the same segmentation (a textbook
    routine); a tone at an exact bin integrates to A^2/2 (periodic Hann window, density scaling)
    and peaks at its frequency; white noise integrates to its variance."""
    import scipy.signal
    from oracle import welch_psd
    rng = np.random.default_rng(4)
    n, nw, dt = 3001, 6, 0.05
    x = 17.0 + rng.normal(size=n) * 0.3
    f, P = welch_psd(x, nw, dt)
    L = 2 * (n // (nw + 1))
    fr, Pr = scipy.signal.welch(x[:L * (nw + 1) // 2], fs=1 / dt, window="hann", nperseg=L, noverlap=L // 2,
                                detrend="constant", scaling="density")
    np.testing.assert_allclose(f, fr, rtol=1e-14)
    np.testing.assert_allclose(P, Pr, rtol=1e-11, atol=0)
    df = f[1] - f[0]
    assert abs(P.sum() * df - x.var()) <= 0.1 * x.var()
    A, b = 0.7, 23
    t = np.arange(L * (nw + 1) // 2)
    tone = A * np.sin(2 * np.pi * b * t / L)
    f2, P2 = welch_psd(tone, nw, dt)
    assert int(np.argmax(P2)) == b
    assert abs(P2.sum() * (f2[1] - f2[0]) - A * A / 2) <= 1e-12


def test_observer_average_of_rms():
    """Spanwise observer: the averaged p_RMS of identical probes is that probe's p_RMS; probes of
    an observer are averaged in RMS (not in mean square)."""
    from oracle import cumulative_prms, observer_oaspl
    rng = np.random.default_rng(9)
    s1 = rng.normal(size=200)
    s2 = 3.0 * rng.normal(size=200)
    avg, db = observer_oaspl(np.stack([s1, s1, s2, s1]), np.array([0, 0, 1, 1]), 2, 1e-3)
    r1, r2 = cumulative_prms(s1)[-1], cumulative_prms(s2)[-1]
    assert abs(avg[0] - r1) <= 1e-15 * r1
    assert abs(avg[1] - 0.5 * (r1 + r2)) <= 1e-14 * r2
    assert abs(db[0] - 20 * np.log10(r1 / 1e-3)) <= 1e-12
