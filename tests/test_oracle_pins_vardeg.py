"""Pins of the variable-degree oracle (CPU only): it reduces to the single-degree oracle, the
mortar projection returns lower-degree polynomials unchanged, degree jumps keep discrete
conservation and free-stream preservation, an all-P0 mesh is the first-order finite-volume
Rusanov scheme written out here, and a smooth solution converges across a degree jump."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import OracleSystem
from oracle.flow import rusanov
from oracle.vardeg import VarDegreeOracle


def _state(v, fn):
    return [torch.tensor(fn(x)).permute(0, 2, 1).contiguous() for x in v.solpt_coords()]


@pytest.mark.parametrize("dim,p,bc,eq", [(2, 3, "channel", "ns"), (3, 2, "farfield", "ns"), (2, 2, "periodic", "euler"),
                                         (2, 4, "farfield", "ns")])
def test_uniform_degree_equals_single_degree_oracle(dim, p, bc, eq):
    m = fi.periodic_box(dim, 3 if dim == 3 else (4, 3), q=2, curv=0.15, bc=bc, seed=3)
    fp = fi.freestream_params(dim, 0.3, 100.0 if eq == "ns" else None, aoa_deg=20.0)
    s = OracleSystem(m, p, fp, equations=eq)
    v = VarDegreeOracle(m, np.full(m.n_elem, p), fp, equations=eq)
    u = torch.tensor(fi.developed_state(s.solpt_coords(), fp, 3)).permute(0, 2, 1).contiguous()
    assert torch.equal(v.residual([u])[0], s.residual(u))


def test_mortar_projection_reproduces_lower_degree_polynomials():
    """Pi I = identity for every degree pair met on a mesh with all degrees 0..4 (2-D and 3-D):
    the L2 projection (mortar Gauss quadrature) of a lower-degree trace is that trace; Pi
    preserves the face integral (its columns' weighted sums are the mortar weights)."""
    for dim in (2, 3):
        m = fi.periodic_box(dim, 4 if dim == 2 else 3, q=1, seed=2)
        deg = np.random.default_rng(8).integers(0, 5, m.n_elem)
        v = VarDegreeOracle(m, deg, fi.freestream_params(dim, 0.3, 50.0))
        assert len(v.mortars) > 10
        pairs = set()
        for M in v.mortars:
            n_lo = M["I"].shape[1]
            np.testing.assert_allclose(M["Pi"] @ M["I"], np.eye(n_lo), atol=1e-13)
            pairs.add((v.groups[M["gh"]].p, v.groups[M["gl"]].p))
        assert len(pairs) >= 6, pairs


@pytest.mark.parametrize("dim,eq", [(2, "ns"), (3, "ns"), (2, "euler")])
def test_conservation_across_degree_jumps(dim, eq):
    """Periodic curved mesh with random degrees 0..4 and a perturbed state: the integral of the
    residual of mass, momentum and energy vanishes to round-off (every face's transformed common
    flux has the same integral from both sides, mortar faces included)."""
    m = fi.periodic_box(dim, 4 if dim == 2 else 3, q=2, curv=0.15, seed=5)
    fp = fi.freestream_params(dim, 0.3, 50.0 if eq == "ns" else None)
    deg = np.random.default_rng(1).integers(0, 5, m.n_elem)
    v = VarDegreeOracle(m, deg, fp, equations=eq)
    R = v.residual(_state(v, lambda x: fi.developed_state(x, fp, 4)))
    tot = v.integrate(R)
    scale = v.integrate([r.abs() for r in R])
    assert float((tot.abs() / scale).max()) < 1e-13


def test_free_stream_preserved_on_graded_ogrid_and_extruded_box():
    """A uniform flow is preserved across degree jumps where the face normal is a polynomial of
    degree <= the lower degree along the face (then the projection is exact): the curved O-grid
    (quadratic geometry: normals linear along a face) with the degree falling from 4 at the wall
    ring to 0 at the far-field rings (far field on both rings), and the curved extruded 3-D box
    with random degrees that vary in the x-y plane only (as the airfoil's sponge does), so every
    degree jump lies on a face along z, whose normal is linear in-plane and constant along z.
    (A jump on a face normal to z, whose normal is cubic there, is not free-stream exact below
    degree 3.)"""
    m = fi.o_grid(12, 10, q=2, r1=8.0, wall="farfield", seed=5)
    ir = m.info["grid_index"][:, 0]
    deg = np.clip(4 - ir // 2, 0, 4)
    fp = fi.freestream_params(2, 0.2, 1000.0, aoa_deg=10.0)
    v = VarDegreeOracle(m, deg, fp, equations="ns")
    assert {0, 4} <= set(deg.tolist()) and len(v.mortars) > 0
    R = v.residual(_state(v, lambda x: fi.freestream_state(x, fp)))
    assert max(float(r.abs().max()) for r in R) < 1e-11 * fp.p_inf[0]
    m3 = fi.periodic_box(3, 3, q=2, curv=0.2, seed=6)
    fp3 = fi.freestream_params(3, 0.2, 100.0, aoa_deg=25.0)
    gi = m3.info["grid_index"]
    plane = np.random.default_rng(3).integers(0, 5, (3, 3))
    v3 = VarDegreeOracle(m3, plane[gi[:, 0], gi[:, 1]], fp3, equations="ns")
    assert len(v3.mortars) > 0
    R3 = v3.residual(_state(v3, lambda x: fi.freestream_state(x, fp3)))
    assert max(float(r.abs().max()) for r in R3) < 1e-11 * fp3.p_inf[0]


def test_all_p0_is_first_order_finite_volume():
    """P0 everywhere on a uniform Cartesian periodic mesh (Euler): one point per cell, the
    correction derivative 1/2 at both faces, so R_e = -(1/|cell|) sum_faces F^(u_e, u_nb, n) h,
    the Rusanov finite-volume scheme written out here cell by cell."""
    n, L = 5, 10.0
    m = fi.periodic_box(2, n, q=1)
    fp = fi.freestream_params(2, 0.3, None, aoa_deg=15.0)
    v = VarDegreeOracle(m, np.zeros(m.n_elem, dtype=int), fp, equations="euler")
    u = _state(v, lambda x: fi.developed_state(x, fp, 9, amp=0.2, noise=0.0))
    R = v.residual(u)[0][:, :, 0]
    uc = u[0][:, :, 0]
    xc = v.solpt_coords()[0][:, 0, :]
    h = L / n
    for e in range(m.n_elem):
        acc = torch.zeros(4, dtype=torch.float64)
        for nrm in ((1.0, 0.0), (-1.0, 0.0), (0.0, 1.0), (0.0, -1.0)):
            target = xc[e] + h * np.array(nrm)
            target = (target + L / 2) % L - L / 2
            nb = int(np.argmin(np.linalg.norm(xc - target, axis=1)))
            nn = torch.tensor([nrm], dtype=torch.float64)
            acc += rusanov(uc[e][None], uc[nb][None], nn, fp.gamma)[0] * h
        np.testing.assert_allclose(R[e].numpy(), (-acc / (h * h)).numpy(), rtol=1e-12, atol=1e-12)


def test_convergence_across_a_degree_jump():
    """Entropy wave (an exact Euler solution) on periodic meshes whose left half is degree 3 and
    right half degree 2: the error after a fixed time falls at a rate above the lower degree + 1/2
    under refinement, so the mortar faces are consistent."""
    p_lo, T = 2, 0.5
    errs = []
    for n in (4, 8, 16):
        m = fi.periodic_box(2, n, q=1)
        xc = m.node_xyz[m.elem_nodes].mean(axis=1)
        deg = np.where(xc[:, 0] < 0.0, 3, 2)
        fp = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.ones((1, 2)), p_inf=np.ones(1), mu=np.zeros(1))
        v = VarDegreeOracle(m, deg, fp, equations="euler")
        u = _state(v, fi.entropy_wave_state)
        nst = 25
        for _ in range(nst):
            u = v.rk4_step(u, torch.tensor([T / nst], dtype=torch.float64))
        ue = _state(v, lambda x: fi.entropy_wave_state(x, t=T))
        err2 = v.integrate([(a - b) ** 2 for a, b in zip(u, ue)])
        errs.append(float(err2.sqrt().max()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p_lo + 0.5, (errs, rates)


def _viscous_jump_error(n, field, exact, degs=(3, 4)):
    """max |(R_NS - R_{mu=0}) - exact| / max |exact| on a periodic mesh whose degrees alternate in
    a checkerboard, so that degree jumps lie on faces of both orientations."""
    m = fi.periodic_box(2, n, q=1)
    gi = m.info["grid_index"]
    deg = np.where((gi[:, 0] + gi[:, 1]) % 2 == 0, degs[0], degs[1])
    mu = 0.05
    fpm = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.zeros((1, 2)), p_inf=np.ones(1), mu=np.full(1, mu))
    fp0 = fi.FlowParams(dim=2, rho_inf=np.ones(1), vel_inf=np.zeros((1, 2)), p_inf=np.ones(1), mu=np.zeros(1))
    vm = VarDegreeOracle(m, deg, fpm, equations="ns")
    v0 = VarDegreeOracle(m, deg, fp0, equations="ns")
    u = _state(vm, field)
    err, scale = 0.0, 0.0
    for xs, a, b in zip(vm.solpt_coords(), vm.residual(u), v0.residual(u)):
        ex = torch.tensor(exact(xs, mu)).permute(0, 2, 1)
        err = max(err, float((a - b - ex).abs().max()))
        scale = max(scale, float(ex.abs().max()))
    return err / scale


def test_viscous_closed_forms_across_degree_jumps():
    """Shear wave u_x = A sin(k y) (viscous residual mu u_yy, energy mu A^2 k^2 cos 2ky) and a
    diagonal longitudinal wave ((4/3) mu lap v) on checkerboards of degrees 3 and 4: the viscous
    part of the residual converges to the closed form, so the common solution projected to the
    lower side and both sides' viscous shares at mortar faces are consistent (at the rate of the
    lower degree's uniform mesh: the maximum pointwise error of this second-derivative quantity
    falls by ~4 per refinement at degree 3)."""
    A, k = 0.1, 2 * np.pi / 10

    def shear(x):
        vel = np.zeros(x.shape[:-1] + (2,))
        vel[..., 0] = A * np.sin(k * x[..., 1])
        return fi.fields._cons(np.ones(x.shape[:-1]), vel, np.full(x.shape[:-1], 10.0), 1.4)

    def shear_ex(x, mu):
        out = np.zeros(x.shape[:-1] + (4,))
        out[..., 1] = -mu * k * k * A * np.sin(k * x[..., 1])
        out[..., 3] = mu * A * A * k * k * np.cos(2 * k * x[..., 1])
        return out
    kh = np.array([1.0, 1.0]) / np.sqrt(2.0)
    kk = k * np.sqrt(2.0)

    def longi(x):
        ph = kk * (x @ kh)
        vel = A * np.sin(ph)[..., None] * kh
        return fi.fields._cons(np.ones(x.shape[:-1]), vel, np.full(x.shape[:-1], 10.0), 1.4)

    def longi_ex(x, mu):
        ph = kk * (x @ kh)
        out = np.zeros(x.shape[:-1] + (4,))
        out[..., 1:3] = -(4.0 / 3.0) * mu * A * kk * kk * np.sin(ph)[..., None] * kh
        out[..., 3] = (4.0 / 3.0) * mu * A * A * kk * kk * np.cos(2.0 * ph)
        return out
    for field, exact in ((shear, shear_ex), (longi, longi_ex)):
        e1 = _viscous_jump_error(8, field, exact)
        e2 = _viscous_jump_error(16, field, exact)
        assert e2 < 0.04 and e1 / e2 > 3.0, (e1, e2)


@pytest.mark.parametrize("dim", [2, 3])
def test_corrected_gradient_gauss_identity(dim):
    """On an affine periodic mesh the corrected gradient of FR with g_DG integrates exactly to the
    face integrals of the common solution (Gauss): sum_i w_i J_i grad u_i = sum_f w_f N_f u^_f per
    element, and the faces cancel in the sum over the mesh where u^ is single-valued.  With random
    degrees 0..4 and a random state the total is zero to round-off only if the lower side of
    every mortar face receives the projection of the mortar's common solution."""
    m = fi.periodic_box(dim, 4 if dim == 2 else 3, q=1, seed=4)
    fp = fi.freestream_params(dim, 0.3, 50.0)
    deg = np.random.default_rng(11).integers(0, 5, m.n_elem)
    v = VarDegreeOracle(m, deg, fp, equations="ns")
    u = _state(v, lambda x: fi.developed_state(x, fp, 12, amp=0.3, noise=0.05))
    grad, _ = v._gradients(u, *v._traces(u))
    tot = sum(torch.einsum('i,ei,evij->vj', G.sol_w, G.J, g) for G, g in zip(v.groups, grad))
    scale = sum(torch.einsum('i,ei,evij->vj', G.sol_w, G.J, g.abs()) for G, g in zip(v.groups, grad))
    assert float((tot.abs() / scale).max()) < 1e-13
