"""Checkpointed RK4-trajectory adjoint (fr_rk_step_stages / fr_rk_step_vjp / fr_probe_vjp behind a
torch.autograd.Function) against reverse-mode autograd of the FP64 oracle trajectory and against
central differences of the GPU objective.  Objective: time-mean square of the probe pressure
fluctuation, J = (1/K) sum_n (p_n - mean p)^2, gradient with respect to the initial state."""
import numpy as np
import pytest
import torch

import fr_inputs as fi

pytestmark = pytest.mark.gpu


def _case():
    m = fi.o_grid(16, 6, q=3, r1=6.0, stretch=1.2, seed=7)
    fp = fi.freestream_params(2, 0.2, 1000.0)
    return m, 3, fp, [[0.0, 3.0]]


def _objective(p):
    return ((p - p.mean(dim=0, keepdim=True)) ** 2).mean(dim=0).sum()


def test_trajectory_gradient_matches_oracle_and_fd(gpu):
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m, p, fp, probes = _case()
    s = OracleSystem(m, p, fp, equations="ns", probes=probes)
    x = s.solpt_coords()
    u0 = fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (4,), 3, 2e-2)
    u0 = torch.tensor(u0).permute(0, 2, 1).contiguous()
    K, C, dt = 12, 5, 2e-4
    # oracle: autograd through the whole trajectory
    uo = u0.clone().requires_grad_(True)
    u, ps = uo, []
    for n in range(K):
        ps.append(s.probe_pressure(u))
        u = s.rk4_step(u, torch.tensor([dt], dtype=torch.float64))
    Jref = _objective(torch.stack(ps))
    Jref.backward()
    gref = uo.grad
    # GPU adjoint
    sol = Solver(m, p, fp, equations="ns", probes=probes, max_samples=K)
    dtt = torch.tensor([dt], dtype=torch.float64, device=gpu)
    ug = u0.to(gpu).clone().requires_grad_(True)
    P = FRTrajectory.apply(ug, sol, dtt, K, C, None)
    J = _objective(P)
    J.backward()
    g = ug.grad
    # J is the variance of a signal p ~ p_inf = 17.9 with fluctuations sigma ~ 5e-3: its relative
    # round-off is ~ eps (p_inf / sigma)^2 ~ 3e-9 per operation, hence the 1e-6 bound
    assert abs(float(J.detach()) - float(Jref.detach())) <= 1e-6 * abs(float(Jref.detach())), (float(J.detach()), float(Jref.detach()))
    pref = torch.stack(ps).detach()
    dp = float((P.detach().cpu() - pref).abs().max())
    sig = float(pref.std())
    err = float((g.cpu() - gref).norm() / gref.norm())
    print(f"probe series max diff {dp:.3e} (sigma {sig:.3e}); trajectory gradient rel L2 vs oracle {err:.3e}")
    # the gradient (2/K) sum (p_n - mean p) dp_n/du inherits the relative accuracy of the
    # fluctuation p - mean p, i.e. ~ dp / sigma
    assert dp <= 1e-12 * float(pref.abs().max()), dp
    assert err <= max(1e-9, 20 * dp / sig), err
    # central differences of the GPU objective along seeded directions
    rng = np.random.default_rng(11)
    for _ in range(2):
        v = torch.tensor(rng.normal(size=u0.shape), device=gpu) * 1e-2
        eps = 1e-4
        with torch.no_grad():
            Jp = _objective(FRTrajectory.apply(u0.to(gpu) + eps * v, sol, dtt, K, C, None))
            Jm = _objective(FRTrajectory.apply(u0.to(gpu) - eps * v, sol, dtt, K, C, None))
        fd = float((Jp - Jm) / (2 * eps))
        ad = float((g * v).sum())
        print(f"directional derivative: central difference {fd:.10e} adjoint {ad:.10e}")
        assert abs(fd - ad) <= 1e-5 * abs(ad), (fd, ad)


def test_rk_step_vjp_recompute_equals_recorded_stages(gpu):
    from paper_2312_14167_amd import Solver
    m, p, fp, probes = _case()
    sol = Solver(m, p, fp, equations="ns", probes=probes, max_samples=4)
    x = sol.solpt_coords()
    u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (4,), 4, 1e-2)).permute(0, 2, 1)
    u0 = u0.contiguous().to(gpu)
    dtt = torch.tensor([2e-4], dtype=torch.float64, device=gpu)
    st = torch.empty((3,) + sol.shape, dtype=torch.float64, device=gpu)
    u = u0.clone()
    sol.rk_step_stages(u, dtt, st)
    u2 = u0.clone()
    sol.rk_step(u2, dtt, 1)
    assert torch.equal(u, u2)   # the recording step is the same step
    a = torch.tensor(np.random.default_rng(2).normal(size=u0.shape), device=gpu)
    b1 = a.clone()
    sol.rk_step_vjp(u0, dtt, b1, st)
    b2 = a.clone()
    sol.rk_step_vjp(u0, dtt, b2, None)
    assert torch.equal(b1, b2)
    # node adjoint: recorded stage residuals, recomputed ones, and residuals evaluated afresh
    res = torch.empty((4,) + sol.shape, dtype=torch.float64, device=gpu)
    st2 = torch.empty_like(st)
    sol.rk_step_stages(u0.clone(), dtt, st2, residuals=res)
    assert torch.equal(st2, st)
    # u_bar in the node-adjoint mode: the same value to rounding (the mode's extra normal and |N|
    # terms share subexpressions with the state adjoint, so the compiler contracts a few products
    # into FMAs differently), and bit-identical among the mode's three ways of getting the stages
    xbs, bs = [], []
    for stages, residuals in [(st2, res), (None, None), (st2, None)]:
        b = a.clone()
        xb = torch.zeros((sol.n_node, 2), dtype=torch.float64, device=gpu)
        sol.rk_step_vjp(u0, dtt, b, stages, x_bar=xb, residuals=residuals)
        assert float((b - b1).norm() / b1.norm()) <= 1e-14
        bs.append(b)
        xbs.append(xb)
    assert torch.equal(bs[0], bs[1]) and torch.equal(bs[0], bs[2])
    assert torch.equal(xbs[0], xbs[1])
    assert float((xbs[2] - xbs[0]).norm() / xbs[0].norm()) <= 1e-13


def test_multi_step_recording_equals_single_steps(gpu):
    """fr_rk_step_stages over n steps in one call (flux-point values carried between steps, base
    states copied by the first stage kernel) equals n single recording steps, bit for bit."""
    from paper_2312_14167_amd import Solver
    m, p, fp, probes = _case()
    sol = Solver(m, p, fp, equations="ns")
    x = sol.solpt_coords()
    u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (4,), 6, 1e-2)).permute(0, 2, 1)
    u0 = u0.contiguous().to(gpu)
    dtt = torch.tensor([2e-4], dtype=torch.float64, device=gpu)
    n = 3
    states = torch.empty((n,) + sol.shape, dtype=torch.float64, device=gpu)
    stages = torch.empty((n, 3) + sol.shape, dtype=torch.float64, device=gpu)
    u = u0.clone()
    sol.rk_step_stages(u, dtt, stages, states=states)
    v = u0.clone()
    for k in range(n):
        assert torch.equal(states[k], v)
        st1 = torch.empty((3,) + sol.shape, dtype=torch.float64, device=gpu)
        sol.rk_step_stages(v, dtt, st1)
        assert torch.equal(stages[k], st1)
    assert torch.equal(u, v)


def test_adjoint_full_size_cylinder_80x64(gpu):
    """The adjoint workload at full size: cylinder O-grid 80 x 64, p = 3, FP64.
    (a) 200 RK4 steps with checkpoints every 20: the adjoint directional derivative against central
        differences of the GPU objective along 50 seeded random directions in u0;
    (b) 20 steps: the gradient against reverse-mode autograd of the oracle trajectory."""
    import bench
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m, fp = bench.cylinder_workload(80, 64, p=3, q=3)
    probes = [[0.0, 3.0]]
    sol = Solver(m, 3, fp, equations="ns", probes=probes, max_samples=200)
    u0 = bench.initial_state(sol, fp, m, 9).to(gpu)
    dtt = torch.tensor([1e-4], dtype=torch.float64, device=gpu)
    K, C = 200, 20
    ug = u0.clone().requires_grad_(True)
    J = _objective(FRTrajectory.apply(ug, sol, dtt, K, C, None))
    J.backward()
    g = ug.grad
    rng = np.random.default_rng(50)
    worst = 0.0
    for _ in range(50):
        v = torch.tensor(rng.normal(size=u0.shape), device=gpu)
        v = v / v.norm() * u0.norm() * 1e-3
        eps = 1e-3
        with torch.no_grad():
            Jp = _objective(FRTrajectory.apply(u0 + eps * v, sol, dtt, K, C, None))
            Jm = _objective(FRTrajectory.apply(u0 - eps * v, sol, dtt, K, C, None))
        fd = float((Jp - Jm) / (2 * eps))
        ad = float((g * v).sum())
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    print(f"80x64 adjoint: worst relative FD mismatch over 50 directions {worst:.3e}")
    assert worst <= 1e-4, worst
    # oracle gradient over 20 steps at the same size
    s = OracleSystem(m, 3, fp, equations="ns", probes=probes)
    K2 = 20
    uo = u0.cpu().clone().requires_grad_(True)
    u, ps = uo, []
    for n in range(K2):
        ps.append(s.probe_pressure(u))
        u = s.rk4_step(u, torch.tensor([1e-4], dtype=torch.float64))
    _objective(torch.stack(ps)).backward()
    ug2 = u0.clone().requires_grad_(True)
    _objective(FRTrajectory.apply(ug2, sol, dtt, K2, C, None)).backward()
    err = float((ug2.grad.cpu() - uo.grad).norm() / uo.grad.norm())
    print(f"80x64 adjoint, 20 steps: gradient rel L2 vs oracle {err:.3e}")
    assert err <= 1e-9, err


def test_trajectory_node_gradient_matches_oracle(gpu):
    """dJ/dX (mesh nodes) of the checkpointed trajectory adjoint against reverse-mode autograd of the
    oracle trajectory through its geometry and probe location."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m, p, fp, probes = _case()
    s0 = OracleSystem(m, p, fp, equations="ns", probes=probes)
    x = s0.solpt_coords()
    u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (4,), 3, 2e-2))
    u0 = u0.permute(0, 2, 1).contiguous()
    K, C, dt = 8, 3, 2e-4
    X = torch.tensor(m.node_xyz, dtype=torch.float64, requires_grad=True)
    s = OracleSystem(m, p, fp, equations="ns", probes=probes, node_xyz=X)
    u, ps = u0, []
    for n in range(K):
        ps.append(s.probe_pressure(u))
        u = s.rk4_step(u, torch.tensor([dt], dtype=torch.float64))
    _objective(torch.stack(ps)).backward()
    gref = X.grad.detach()
    sol = Solver(m, p, fp, equations="ns", probes=probes, max_samples=K)
    dtt = torch.tensor([dt], dtype=torch.float64, device=gpu)
    Xg = torch.tensor(m.node_xyz, dtype=torch.float64, device=gpu, requires_grad=True)
    ug = u0.to(gpu).clone().requires_grad_(True)
    _objective(FRTrajectory.apply(ug, sol, dtt, K, C, Xg)).backward()
    err = float((Xg.grad.cpu() - gref).norm() / gref.norm())
    print(f"trajectory node gradient rel L2 vs oracle {err:.3e}")
    assert err <= 1e-8, err


def test_adjoint_full_size_node_gradient_fd_80x64(gpu):
    """The adjoint workload's mesh-node gradient (cylinder O-grid 80 x 64, p = 3, 200 steps,
    checkpoints every 20) against central differences of the GPU objective on rebuilt solvers
    along 50 seeded node directions (scaled with the local radius, so every element deforms by a
    similar fraction)."""
    import bench
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    import fr_inputs as fi2
    m, fp = bench.cylinder_workload(80, 64, p=3, q=3)
    probes = [[0.0, 3.0]]
    sol = Solver(m, 3, fp, equations="ns", probes=probes, max_samples=200)
    u0 = bench.initial_state(sol, fp, m, 9).to(gpu)
    dtt = torch.tensor([1e-4], dtype=torch.float64, device=gpu)
    K, C = 200, 20
    Xg = torch.tensor(m.node_xyz, dtype=torch.float64, device=gpu, requires_grad=True)
    _objective(FRTrajectory.apply(u0.clone(), sol, dtt, K, C, Xg)).backward()
    g = Xg.grad.cpu().numpy()
    sol.close()
    rng = np.random.default_rng(51)
    r = np.linalg.norm(m.node_xyz, axis=1, keepdims=True)
    worst = 0.0
    for t in range(50):
        V = rng.normal(size=m.node_xyz.shape) * r * 1e-2
        eps = 1e-4
        vals = []
        for sg in (1.0, -1.0):
            mm = fi2.MeshDesc(dim=2, q=m.q, node_xyz=m.node_xyz + sg * eps * V, elem_nodes=m.elem_nodes,
                              face_bc=m.face_bc, periodic_vec=m.periodic_vec, mesh_elem_begin=m.mesh_elem_begin)
            sp = Solver(mm, 3, fp, equations="ns", probes=probes, max_samples=200)
            with torch.no_grad():
                vals.append(float(_objective(FRTrajectory.apply(u0.clone(), sp, dtt, K, C, None))))
            sp.close()
        fd = (vals[0] - vals[1]) / (2 * eps)
        ad = float((g * V).sum())
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    print(f"80x64 node gradient: worst relative FD mismatch over 50 directions {worst:.3e}")
    assert worst <= 1e-4, worst


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_trajectory_gradient_3d_cgrid_matches_oracle(precision, gpu):
    """3-D p = 4 (the headline element type, whose flux-point values use the face-blocked layout)
    on a small extruded C-grid with a wall, far field and spanwise periodicity: dJ/du0 of the
    checkpointed trajectory adjoint against reverse-mode autograd of the oracle trajectory, in
    FP64 and in FP32.  FP32 bound: the probe pressures carry the FP32 rounding of the state,
    ~ eps_32 rho E ~ 3e-6 absolute, against fluctuations sigma of the series, and the gradient
    (2/K) sum (p_n - mean p) dp_n/du inherits that relative error, so the bound is
    2 eps_32 p_inf / sigma."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m = fi.c_grid_naca(n_wake=3, n_foil=8, n_normal=3, n_span=2, q=2, camber=0.02, r_out=4.0, x_out=6.0,
                       h_wall=0.05)
    fp = fi.freestream_params(3, 0.2, 23000.0, aoa_deg=4.0)
    probes = [[0.6, 0.4, 0.05]]
    s = OracleSystem(m, 4, fp, equations="ns", probes=probes)
    u0 = torch.tensor(fi.developed_state(s.solpt_coords(), fp, 13, periods=[None, None, m.info["span"]]))
    u0 = u0.permute(0, 2, 1).contiguous()
    K, C, dt = 6, 4, 5e-4
    uo = u0.clone().requires_grad_(True)
    u, ps = uo, []
    for n in range(K):
        ps.append(s.probe_pressure(u))
        u = s.rk4_step(u, torch.tensor([dt], dtype=torch.float64))
    Jref = _objective(torch.stack(ps))
    Jref.backward()
    gref = uo.grad
    pref = torch.stack(ps).detach()
    sig = float(pref.std())
    sol = Solver(m, 4, fp, equations="ns", precision=precision, probes=probes, max_samples=K)
    dtt = torch.tensor([dt], dtype=torch.float64, device=gpu)
    ug = u0.to(device=gpu, dtype=sol.dtype).clone().requires_grad_(True)
    P = FRTrajectory.apply(ug, sol, dtt, K, C, None)
    J = _objective(P)
    J.backward()
    err = float((ug.grad.double().cpu() - gref).norm() / gref.norm())
    dp = float((P.detach().cpu() - pref).abs().max())
    print(f"3-D C-grid trajectory adjoint {precision}: probe series max diff {dp:.3e} (sigma {sig:.3e}), "
          f"J {float(J.detach()):.6e} vs {float(Jref.detach()):.6e}, gradient rel L2 vs oracle {err:.3e}")
    if precision == "fp64":
        assert dp <= 1e-12 * float(pref.abs().max()), dp
        assert err <= max(1e-9, 20 * dp / sig), err
    else:
        bound = 2 * 6e-8 * float(fp.p_inf[0]) / sig
        assert err <= bound, (err, bound)
    sol.close()


def test_trajectory_gradient_fp32_2d_matches_oracle(gpu):
    """The FP32 trajectory adjoint (FP32 state, stage records and reverse sweep; FP64 probe
    series) on the 2-D cylinder case against the FP64 oracle's autograd, within the bound derived
    in the 3-D test."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m, p, fp, probes = _case()
    s = OracleSystem(m, p, fp, equations="ns", probes=probes)
    u0 = torch.tensor(fi.developed_state(s.solpt_coords(), fp, 17)).permute(0, 2, 1).contiguous()
    K, C, dt = 12, 5, 2e-4
    uo = u0.clone().requires_grad_(True)
    u, ps = uo, []
    for n in range(K):
        ps.append(s.probe_pressure(u))
        u = s.rk4_step(u, torch.tensor([dt], dtype=torch.float64))
    _objective(torch.stack(ps)).backward()
    gref = uo.grad
    sig = float(torch.stack(ps).detach().std())
    sol = Solver(m, p, fp, equations="ns", precision="fp32", probes=probes, max_samples=K)
    ug = u0.float().to(gpu).clone().requires_grad_(True)
    _objective(FRTrajectory.apply(ug, sol, torch.tensor([dt], dtype=torch.float64, device=gpu), K, C, None)).backward()
    err = float((ug.grad.double().cpu() - gref).norm() / gref.norm())
    bound = 2 * 6e-8 * float(fp.p_inf[0]) / sig
    print(f"2-D trajectory adjoint fp32: gradient rel L2 vs oracle {err:.3e} (sigma {sig:.3e}, bound {bound:.2e})")
    assert err <= bound, (err, bound)
    sol.close()
