"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances: FP64 relative L2 (max over variables) <= 1e-12 on the state after RK4 steps
(the stated per-step target) and <= 1e-11 on the residual itself (the residual is a difference
of fluxes ~ p_inf / h, so its round-off is amplified relative to its size; the bound is the
FP64 unit round-off 1.1e-16 times a conservative 1e5 amplification).  FP32: relative L2 <= 1e-5
on the state after one step (measured <= 1.4e-6); the residual within 5e-4 relative (measured
<= 4.9e-5).  p_RMS from the stored FP64 series (two passes about the mean): 1e-9 relative; from
the running sums once the series capacity is exceeded, where S2/n - (S1/n)^2 cancels
(p_inf / sigma)^2 ~ 1e8 of its digits: 1e-6.
"""
import numpy as np
import pytest
import torch

from cases import make_case, oracle_for, rel_l2

pytestmark = pytest.mark.gpu

CASES = ["euler_vortex", "euler_farfield_curved", "ns_periodic_curved", "ns_ogrid", "ns_channel_p3",
         "ns_box3d_p2", "ns_cgrid_p4", "ns_cavity_batch"]


def _solver(name, precision="fp64", forces=True):
    from paper_2312_14167_amd import Solver
    s, m, p, fp, eq, u0, dt, probes, pm = oracle_for(name)
    sol = Solver(m, p, fp, equations=eq, precision=precision, probes=probes, probe_mesh=pm, max_samples=64,
                 forces=forces)
    return s, sol, u0, dt


@pytest.mark.parametrize("name", CASES)
def test_solpt_coords_match_oracle(name, gpu):
    s, sol, u0, dt = _solver(name)
    np.testing.assert_allclose(sol.solpt_coords(), s.solpt_coords(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", CASES)
def test_rhs_fp64(name, gpu):
    s, sol, u0, dt = _solver(name)
    Rref = s.residual(u0)
    R = sol.rhs(u0.to(gpu))
    torch.cuda.synchronize()
    err = rel_l2(R, Rref)
    print(f"{name}: rhs fp64 rel L2 {err:.3e}")
    assert err <= 1e-11, err


@pytest.mark.parametrize("beta", [-0.5, 0.0, 0.3])
@pytest.mark.parametrize("name", ["ns_ogrid", "ns_box3d_p2", "ns_cgrid_p4"])
def test_rhs_and_step_fp64_other_ldg_beta(name, beta, gpu):
    """The LDG switch beta: -1/2 (the other one-sided form) and two-sided values, where both sides'
    viscous normal fluxes enter every interior common flux."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    m, p, fp, eq, init, dt, probes = make_case(name)
    fp.ldg_beta = beta
    s = OracleSystem(m, p, fp, equations=eq)
    u0 = torch.tensor(init(s.solpt_coords())).permute(0, 2, 1).contiguous()
    sol = Solver(m, p, fp, equations=eq)
    eR = rel_l2(sol.rhs(u0.to(gpu)), s.residual(u0))
    u = u0.to(gpu).clone()
    sol.rk_step(u, torch.tensor(dt, dtype=torch.float64, device=gpu), 2)
    uref, _, _ = s.run(u0, torch.tensor(dt), 2, sample_every=0)
    e2 = rel_l2(u, uref)
    print(f"{name} beta {beta}: rhs rel L2 {eR:.3e}, 2 steps {e2:.3e}")
    assert eR <= 1e-11 and e2 <= 1e-12, (eR, e2)


@pytest.mark.parametrize("name", CASES)
def test_rk4_fp64_1_and_20_steps_with_probe(name, gpu):
    s, sol, u0, dt = _solver(name)
    dtt = torch.tensor(dt, dtype=torch.float64, device=gpu)
    u = u0.to(gpu).clone()
    sol.reset_accumulators()
    sol.rk_step(u, dtt, 1, sample_every=1)
    uref1, P1, F1 = s.run(u0, torch.tensor(dt), 1, sample_every=1)
    torch.cuda.synchronize()
    e1 = rel_l2(u, uref1)
    sol.rk_step(u, dtt, 19, sample_every=1)
    uref, P, F = s.run(uref1, torch.tensor(dt), 19, sample_every=1, step0=1)
    P = torch.cat([P1, P])
    F = torch.cat([F1, F])
    e20 = rel_l2(u, uref)
    ser = sol.probe_series(64)
    st = sol.probe_oaspl(p_ref=2e-5)
    print(f"{name}: rk4 fp64 rel L2 1 step {e1:.3e}, 20 steps {e20:.3e}")
    assert e1 <= 1e-12 and e20 <= 1e-12, (e1, e20)
    assert st["n_samples"] == 20
    np.testing.assert_allclose(ser.T, P.numpy(), rtol=1e-12, atol=0)
    pr = P.numpy()
    np.testing.assert_allclose(st["prms"], pr.std(axis=0), rtol=1e-9, atol=1e-15)
    if s.viscous and (s.bT == 1).any():
        Fm = F.mean(dim=0).numpy()
        scale = np.abs(Fm).max()
        np.testing.assert_allclose(st["mean_force"], Fm, rtol=0, atol=1e-10 * max(scale, 1e-3))


@pytest.mark.parametrize("name", ["euler_vortex", "ns_periodic_curved", "ns_ogrid", "ns_box3d_p2", "ns_cgrid_p4",
                                  "ns_cavity_batch"])
def test_fp32_vs_fp64_oracle(name, gpu):
    s, sol, u0, dt = _solver(name, precision="fp32")
    Rref = s.residual(u0)
    R = sol.rhs(u0.float().to(gpu))
    eR = rel_l2(R, Rref)
    u = u0.float().to(gpu).clone()
    dtt = torch.tensor(dt, dtype=torch.float64, device=gpu)
    sol.rk_step(u, dtt, 1)
    uref, _, _ = s.run(u0, torch.tensor(dt), 1, sample_every=0)
    torch.cuda.synchronize()
    e1 = rel_l2(u, uref)
    print(f"{name}: fp32 rhs rel L2 {eR:.3e}, 1 step {e1:.3e}")
    assert e1 <= 1e-5, e1
    assert eR <= 5e-4, eR


@pytest.mark.parametrize("name", ["ns_ogrid", "ns_cgrid_p4"])
def test_fp32_two_sided_ldg(name, gpu):
    """FP32 with the two-sided LDG flux (beta = 0): every flux point's viscous normal flux is stored
    (3-D p = 4: in the face-blocked layout) and the face kernel forms each pair's common flux."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    m, p, fp, eq, init, dt, probes = make_case(name)
    fp.ldg_beta = 0.0
    s = OracleSystem(m, p, fp, equations=eq)
    u0 = torch.tensor(init(s.solpt_coords())).permute(0, 2, 1).contiguous()
    sol = Solver(m, p, fp, equations=eq, precision="fp32")
    eR = rel_l2(sol.rhs(u0.float().to(gpu)), s.residual(u0))
    u = u0.float().to(gpu).clone()
    sol.rk_step(u, torch.tensor(dt, dtype=torch.float64, device=gpu), 1)
    uref, _, _ = s.run(u0, torch.tensor(dt), 1, sample_every=0)
    torch.cuda.synchronize()
    e1 = rel_l2(u, uref)
    print(f"{name} beta 0 fp32: rhs rel L2 {eR:.3e}, 1 step {e1:.3e}")
    assert e1 <= 1e-5, e1
    assert eR <= 5e-4, eR


def test_graph_replay_matches_direct_launches(gpu, monkeypatch):
    """Steps replayed from the captured graph equal the same steps launched directly, bit for bit,
    and two identical runs are bitwise identical (no atomics in the reductions)."""
    name = "ns_ogrid"
    s, sol, u0, dt = _solver(name)
    dtt = torch.tensor(dt, dtype=torch.float64, device=gpu)
    outs = []
    for _ in range(2):
        u = u0.to(gpu).clone()
        sol.reset_accumulators()
        sol.rk_step(u, dtt, 5, sample_every=2)
        outs.append((u.clone(), sol.probe_series(8)))
    assert torch.equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    monkeypatch.setenv("FRMI_NO_GRAPH", "1")
    _, sol2, _, _ = _solver(name)
    u = u0.to(gpu).clone()
    sol2.rk_step(u, dtt, 5, sample_every=2)
    assert torch.equal(u, outs[0][0])
    np.testing.assert_array_equal(sol2.probe_series(8), outs[0][1])


def test_ragged_tiles_and_single_element(gpu):
    """Element counts that leave partial workgroup tiles, and a one-element periodic mesh (an
    element that is its own neighbour through opposite faces)."""
    import fr_inputs as fi
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    for n, p in [((1, 1), 2), ((7, 3), 4), ((5, 9), 3)]:
        m = fi.periodic_box(2, n, q=2, curv=0.1 if min(n) > 1 else 0.0, seed=1)
        fp = fi.freestream_params(2, 0.3, 100.0, aoa_deg=30.0)
        s = OracleSystem(m, p, fp, equations="ns")
        x = s.solpt_coords()
        u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (4,), 3, 0.01)).permute(0, 2, 1)
        u0 = u0.contiguous()
        sol = Solver(m, p, fp, equations="ns")
        R = sol.rhs(u0.to(gpu))
        assert rel_l2(R, s.residual(u0)) <= 1e-11


@pytest.mark.parametrize("shape,probes", [((3, 1, 1), True), ((1, 3, 1), True), ((3, 3, 1), True),
                                          ((3, 3, 1), False)])
def test_ragged_tiles_3d_p4_channel(shape, probes, gpu):
    """3-D p = 4 (the headline element type) with odd element counts, so the last workgroup of the
    NS volume kernel (2 elements per tile in FP64) and of the lifting + RK kernel is partial; walls
    at the y bounds exercise the boundary flux points and the chunked wall-force sum.  Residual and
    one RK4 step with force sampling against the oracle; without probes the sample count (which
    divides the force sum) still advances."""
    import fr_inputs as fi
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    m = fi.periodic_box(3, shape, q=2, curv=0.1, bc="channel", seed=5)
    fp = fi.freestream_params(3, 0.3, 100.0, aoa_deg=20.0)
    s = OracleSystem(m, 4, fp, equations="ns")
    x = s.solpt_coords()
    u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (5,), 7, 0.01)).permute(0, 2, 1)
    u0 = u0.contiguous()
    sol = Solver(m, 4, fp, equations="ns", forces=True, probes=[[0.1, 0.2, 0.3]] if probes else None,
                 max_samples=4)
    R = sol.rhs(u0.to(gpu))
    assert rel_l2(R, s.residual(u0)) <= 1e-11
    dt = np.array([1e-3])
    u = u0.to(gpu).clone()
    sol.reset_accumulators()
    sol.rk_step(u, torch.tensor(dt, dtype=torch.float64, device=gpu), 1, sample_every=1)
    uref, P, F = s.run(u0, torch.tensor(dt), 1, sample_every=1)
    torch.cuda.synchronize()
    assert rel_l2(u, uref) <= 1e-12
    st = sol.probe_oaspl(p_ref=2e-5)
    assert st["n_samples"] == 1
    Fm = F.numpy().mean(axis=0)
    np.testing.assert_allclose(st["mean_force"], Fm, rtol=0, atol=1e-10 * max(float(np.abs(Fm).max()), 1e-3))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["ns_ogrid", "euler_vortex", "ns_cgrid_p4"])
def test_every_tuner_candidate_gives_the_same_step(name, precision, gpu):
    """Every vector-ALU candidate of the autotuner (tile size x waves-per-SIMD bound) computes a
    bit-identical RK4 step (the tile only regroups elements into workgroups, the bound only the
    register allocation); the matrix-core divergence (FP32 3-D p = 4) rounds differently and is
    held to the FP32 bar against the oracle.  The tuner leaves u untouched, re-captures graphs,
    and a second solver of the same shape takes the remembered choice."""
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd._lib import lib
    s, m, p, fp, eq, u0, dt, probes, pm = oracle_for(name, with_probes=False)
    sol = Solver(m, p, fp, equations=eq, precision=precision)
    dtt = torch.tensor(dt, dtype=torch.float64, device=gpu)
    ug = u0.to(device=gpu, dtype=sol.dtype)
    ref = ug.clone()
    sol.rk_step(ref, dtt, 2)
    uref, _, _ = s.run(u0, torch.tensor(dt), 2, sample_every=0)
    kinds = [0, 1] if eq == "ns" else [2]
    n_mfma = 0
    if eq == "ns":
        # the volume adjoint's candidates give a bit-identical residual adjoint
        rbar = torch.sin(torch.arange(ug.numel(), device=gpu, dtype=sol.dtype)).reshape(ug.shape)
        cands = sol.tune_candidates(3)
        assert len(cands) == 3
        zref = torch.zeros_like(ug)
        sol.rhs_vjp(ug, rbar, zref)
        for c, (E, W, engine) in enumerate(cands):
            sol.tune_select(3, c)
            z = torch.zeros_like(ug)
            sol.rhs_vjp(ug, rbar, z)
            assert torch.equal(z, zref), (c, E, W)
        sol.tune_select(3, 0)
    for k in kinds:
        cands = sol.tune_candidates(k)
        assert len(cands) >= 6
        for c, (E, W, engine) in enumerate(cands):
            sol.tune_select(k, c)
            u = ug.clone()
            sol.rk_step(u, dtt, 2)
            if engine == 0:
                assert torch.equal(u, ref), (k, c, E, W)
            else:
                n_mfma += 1
                e = rel_l2(u, uref)
                print(f"{name} {precision}: matrix-core divergence, 2 steps rel L2 vs oracle {e:.3e}")
                assert e <= 1e-5
        sol.tune_select(k, 0)
    assert n_mfma == (2 if (precision == "fp32" and m.dim == 3 and p == 4) else 0)
    lib().fr_tune_cache_clear()
    keep = ug.clone()
    choice = sol.autotune(ug, dtt, reps=1)
    assert torch.equal(ug, keep)
    print(f"{name} {precision}: autotuned { {k: (v['elements_per_workgroup'], v['waves_per_simd_bound'], v['engine']) for k, v in choice.items()} }")
    assert not any(v["from_cache"] for v in choice.values())
    u = ug.clone()
    sol.rk_step(u, dtt, 2)
    assert rel_l2(u, uref) <= (1e-12 if precision == "fp64" else 1e-5)
    again = Solver(m, p, fp, equations=eq, precision=precision)
    choice2 = again.autotune(ug, dtt, reps=1)
    assert all(v["from_cache"] for v in choice2.values())
    assert {k: v["elements_per_workgroup"] for k, v in choice2.items()} == \
        {k: v["elements_per_workgroup"] for k, v in choice.items()}


@pytest.mark.parametrize("p,dim,eq,bc", [(1, 2, "ns", "channel"), (1, 3, "ns", "channel"), (1, 2, "euler", "periodic"),
                                         (3, 3, "ns", "channel"), (3, 3, "euler", "periodic")])
def test_small_degree_and_3d_p3(p, dim, eq, bc, gpu):
    """p = 1 (2 points per direction: the smallest tiles and the NS tile whose LDS region is sized
    for the neighbour codes rather than the gradient) and 3-D p = 3 (the degree no other 3-D case
    uses): residual and one RK4 step in FP64 against the oracle; in FP32 one RK4 step within the
    FP32 bar (the residual, a small difference of large flux terms, gets the looser bar of the other
    FP32 parity cases)."""
    import fr_inputs as fi
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    shape = (7, 5) if dim == 2 else (3, 3, 2)
    m = fi.periodic_box(dim, shape, q=1, bc=bc, seed=6)
    fp = fi.freestream_params(dim, 0.3, 100.0 if eq == "ns" else None, aoa_deg=25.0)
    s = OracleSystem(m, p, fp, equations=eq)
    x = s.solpt_coords()
    nv = dim + 2
    u0 = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (nv,), 4, 0.01)).permute(0, 2, 1)
    u0 = u0.contiguous()
    sol = Solver(m, p, fp, equations=eq, forces=(eq == "ns"), max_samples=4)
    R = sol.rhs(u0.to(gpu))
    assert rel_l2(R, s.residual(u0)) <= 1e-11
    dt = np.array([2e-3])
    u = u0.to(gpu).clone()
    sol.rk_step(u, torch.tensor(dt, dtype=torch.float64, device=gpu), 1, sample_every=1)
    uref, _, _ = s.run(u0, torch.tensor(dt), 1, sample_every=1)
    torch.cuda.synchronize()
    assert rel_l2(u, uref) <= 1e-12
    s32 = Solver(m, p, fp, equations=eq, precision="fp32")
    R32 = s32.rhs(u0.float().to(gpu))
    assert rel_l2(R32, s.residual(u0)) <= 5e-4
    u32 = u0.float().to(gpu).clone()
    s32.rk_step(u32, torch.tensor(dt, dtype=torch.float64, device=gpu), 1)
    torch.cuda.synchronize()
    assert rel_l2(u32, uref) <= 1e-5


def test_many_probes_sampling_interval_and_series_cap(gpu):
    """Six probes (two in one element): every probe workgroup of a sample stores at the same
    sample index and the last one to finish advances it, so across two rk_step calls with a
    sampling interval of 2 the samples land where the oracle takes them; the series keeps the
    first max_samples of them while the sums (p_RMS) cover all; a reset starts again at index 0."""
    import fr_inputs as fi
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    m = fi.periodic_box(2, (6, 5), q=2, curv=0.15, seed=9)
    fp = fi.freestream_params(2, 0.3, 100.0, aoa_deg=10.0)
    probes = [[0.3, 0.4], [1.2, -0.5], [2.1, 0.6], [0.5, -1.2], [-1.0, 0.2], [3.9, 3.9]]
    s = OracleSystem(m, 3, fp, equations="ns", probes=probes)
    u0 = torch.tensor(fi.freestream_state(s.solpt_coords(), fp)
                      + fi.noise_like(s.solpt_coords().shape[:-1] + (4,), 8, 0.02)).permute(0, 2, 1).contiguous()
    dt = np.array([1e-3])
    dtt = torch.tensor(dt, dtype=torch.float64, device=gpu)
    sol = Solver(m, 3, fp, equations="ns", probes=probes, max_samples=3, forces=False)
    u = u0.to(gpu).clone()
    sol.reset_accumulators()
    sol.rk_step(u, dtt, 5, sample_every=2)
    sol.rk_step(u, dtt, 4, sample_every=2)
    uref, P, _ = s.run(u0, torch.tensor(dt), 9, sample_every=2, forces=False)
    torch.cuda.synchronize()
    assert rel_l2(u, uref) <= 1e-12
    assert P.shape == (5, 6)
    st = sol.probe_oaspl(p_ref=2e-5)
    assert st["n_samples"] == 5
    np.testing.assert_allclose(sol.probe_series(8).T, P.numpy()[:3], rtol=1e-12, atol=0)
    np.testing.assert_allclose(st["prms"], P.numpy().std(axis=0), rtol=1e-6, atol=1e-13)
    # a reset clears the index and the sums; sampling every step from the current state
    sol.reset_accumulators()
    sol.rk_step(u, dtt, 2, sample_every=1)
    _, P2, _ = s.run(uref, torch.tensor(dt), 2, sample_every=1, forces=False)
    st2 = sol.probe_oaspl(p_ref=2e-5)
    assert st2["n_samples"] == 2
    np.testing.assert_allclose(sol.probe_series(8).T, P2.numpy(), rtol=1e-12, atol=0)
    np.testing.assert_allclose(st2["prms"], P2.numpy().std(axis=0), rtol=1e-9, atol=1e-15)
