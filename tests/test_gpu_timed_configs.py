"""Parity at the configurations the bench times, against the FP64 oracle, per variable (the
relative L2 of each conserved variable over all solution points, maximum over variables).

* The headline C-grid (seeded NACA section and angle of attack of the bench) reduced to
  50 x 20 x 4 hexes at p = 4: 1 and 20 RK4 steps with probe and wall-force sampling, FP64
  (<= 1e-12) and FP32 (<= 1e-5), autotuned tiles as the bench runs them.
* A batched poll of three cavities of uneven size at p = 4 (the batched form's degree), in one
  solver, FP64 and FP32, with a probe and wall forces per mesh.
* Per-point checks on the elements next to walls and to the far field, where a localised error
  in a boundary flux would hide in a whole-mesh norm.
* A non-finite state: a NaN written into the state from the host makes the probe statistics call
  report FR_ERR_NONFINITE; a reset clears it.

Initial states have the magnitudes of a developed flow (free stream plus smooth seeded
disturbances of 10 % of the free-stream speed on every velocity component): a uniform stream
plus 1e-3 noise leaves the cross-stream momenta near zero, and their relative error then
measures only the absolute round-off of the pressure term.
"""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from cases import rel_l2

pytestmark = pytest.mark.gpu

CGRID_CELLS = (10, 30, 20, 4)
CGRID_DT = 5e-7
CGRID_STEPS, CGRID_EVERY = 20, 4


def per_var_max(a, b, elems):
    """max over variables of max_{elems, points} |a - b| / max_{elems, points} |b|."""
    a = a.detach().double().cpu()[elems]
    b = b.detach().double().cpu()[elems]
    num = (a - b).abs().amax(dim=(0, 2))
    den = b.abs().amax(dim=(0, 2)).clamp_min(1e-300)
    return float((num / den).max())


def boundary_elements(mesh, tag):
    return np.nonzero((np.asarray(mesh.face_bc) == tag).any(axis=1))[0]


# ----------------------------------------------------------------------------- reduced C-grid
@pytest.fixture(scope="module")
def cgrid():
    """Oracle trajectory of the reduced C-grid: states after 1 and 20 steps, probe series and
    forces sampled every 4 steps, and the residual of the initial state."""
    import bench
    from oracle import OracleSystem
    mesh, fp, aoa = bench.naca_workload(cells=CGRID_CELLS)
    probe = mesh.info["probe"][None, :]
    s = OracleSystem(mesh, 4, fp, equations="ns", probes=probe)
    x = s.solpt_coords()
    u0 = torch.tensor(fi.developed_state(x, fp, 21, periods=[None, None, mesh.info["span"]])).permute(0, 2, 1)
    u0 = u0.contiguous()
    dt = torch.tensor([CGRID_DT], dtype=torch.float64)
    R0 = s.residual(u0)
    u1, P1, F1 = s.run(u0, dt, 1, sample_every=CGRID_EVERY)
    u20, P, F = s.run(u1, dt, CGRID_STEPS - 1, sample_every=CGRID_EVERY, step0=1)
    return {"mesh": mesh, "fp": fp, "probe": probe, "u0": u0, "R0": R0, "u1": u1, "u20": u20,
            "P": torch.cat([P1, P]), "F": torch.cat([F1, F])}


def _cgrid_run(c, precision, gpu):
    from paper_2312_14167_amd import Solver
    sol = Solver(c["mesh"], 4, c["fp"], equations="ns", precision=precision, probes=c["probe"],
                 max_samples=CGRID_STEPS, forces=True)
    dt = torch.tensor([CGRID_DT], dtype=torch.float64, device=gpu)
    u = c["u0"].to(device=gpu, dtype=sol.dtype)
    tiles = sol.autotune(u, dt, reps=1)
    R = sol.rhs(u)
    sol.reset_accumulators()
    sol.rk_step(u, dt, 1, sample_every=CGRID_EVERY)
    u1 = u.clone()
    sol.rk_step(u, dt, CGRID_STEPS - 1, sample_every=CGRID_EVERY)
    torch.cuda.synchronize()
    st = sol.probe_oaspl(p_ref=2e-5)
    ser = sol.probe_series(CGRID_STEPS)
    sol.close()
    return tiles, R, u1, u, st, ser


def test_reduced_cgrid_fp64_1_and_20_steps(cgrid, gpu):
    c = cgrid
    tiles, R, u1, u20, st, ser = _cgrid_run(c, "fp64", gpu)
    eR, e1, e20 = rel_l2(R, c["R0"]), rel_l2(u1, c["u1"]), rel_l2(u20, c["u20"])
    P, F = c["P"].numpy(), c["F"].numpy()
    print(f"C-grid 50x20x4 p=4 FP64 (tiles {tiles}): residual {eR:.3e}, 1 step {e1:.3e}, 20 steps {e20:.3e}")
    assert eR <= 1e-11 and e1 <= 1e-12 and e20 <= 1e-12, (eR, e1, e20)
    assert st["n_samples"] == len(P) == CGRID_STEPS // CGRID_EVERY
    dp = float(np.abs(ser.T - P).max() / np.abs(P).max())
    Fm = F.mean(axis=0)
    dF = float(np.abs(st["mean_force"] - Fm).max() / np.abs(Fm).max())
    print(f"  probe series rel {dp:.3e}, mean force rel {dF:.3e}")
    assert dp <= 1e-13 and dF <= 1e-11, (dp, dF)


def test_reduced_cgrid_fp32_1_and_20_steps(cgrid, gpu):
    c = cgrid
    tiles, R, u1, u20, st, ser = _cgrid_run(c, "fp32", gpu)
    eR, e1, e20 = rel_l2(R, c["R0"]), rel_l2(u1, c["u1"]), rel_l2(u20, c["u20"])
    P, F = c["P"].numpy(), c["F"].numpy()
    dp = float(np.abs(ser.T - P).max() / np.abs(P).max())
    Fm = F.mean(axis=0)
    dF = float(np.abs(st["mean_force"] - Fm).max() / np.abs(Fm).max())
    print(f"C-grid 50x20x4 p=4 FP32 (tiles {tiles}): residual {eR:.3e}, 1 step {e1:.3e}, 20 steps {e20:.3e}; "
          f"probe series rel {dp:.3e}, mean force rel {dF:.3e}")
    assert e1 <= 1e-5 and e20 <= 1e-5, (e1, e20)
    assert eR <= 2e-4, eR
    # FP64 accumulators of FP32 states: the probe pressure carries the state's FP32 rounding
    assert dp <= 2e-6 and dF <= 1e-6, (dp, dF)


def test_reduced_cgrid_boundary_elements_pointwise(cgrid, gpu):
    """Maximum error over every solution point of the elements with a wall face, and of those with
    a far-field face, per variable: residual and the state after one step."""
    from paper_2312_14167_amd import Solver
    c = cgrid
    tiles, R, u1, u20, st, ser = _cgrid_run(c, "fp64", gpu)
    for tag, name in ((fi.BC_WALL, "wall"), (fi.BC_FARFIELD, "far field")):
        el = boundary_elements(c["mesh"], tag)
        eR = per_var_max(R, c["R0"], el)
        e1 = per_var_max(u1, c["u1"], el)
        print(f"C-grid {name} elements ({len(el)}): pointwise residual {eR:.3e}, 1 step {e1:.3e}")
        assert len(el) > 0 and eR <= 5e-11 and e1 <= 1e-12, (name, eR, e1)


# ----------------------------------------------------------------------------- batched cavities
CAV = [(1.6, 0.2), (2.4, 0.14), (3.3, 0.1)]
CAV_DT = np.array([2e-4, 1.5e-4, 1e-4])
CAV_STEPS = 8


@pytest.fixture(scope="module")
def cavities():
    from oracle import OracleSystem
    ms = [fi.cavity(a, h=h, q=2, upstream=2.0, top=3.0, outflow=4.0, top_buffer=1.0, out_buffer=1.5) for a, h in CAV]
    mesh = fi.concat_meshes(ms)
    fp = fi.freestream_params(2, 0.15, 1500.0, n_mesh=3)
    fp.vel_inf[1] = [np.cos(0.05), np.sin(0.05)]
    fp.p_inf[2] *= 1.02
    probes = np.array([[0.5, 1.79]] * 3)
    s = OracleSystem(mesh, 4, fp, equations="ns", probes=probes, probe_mesh=[0, 1, 2])
    x = s.solpt_coords()
    u0 = torch.tensor(fi.developed_state(x, fp, 23, mesh=mesh)).permute(0, 2, 1).contiguous()
    R0 = s.residual(u0)
    u1, P1, F1 = s.run(u0, torch.tensor(CAV_DT), 1, sample_every=1)
    uN, P, F = s.run(u1, torch.tensor(CAV_DT), CAV_STEPS - 1, sample_every=1, step0=1)
    return {"mesh": mesh, "fp": fp, "probes": probes, "u0": u0, "R0": R0, "u1": u1, "uN": uN,
            "P": torch.cat([P1, P]).numpy(), "F": torch.cat([F1, F]).numpy(), "counts": [m.n_elem for m in ms]}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_uneven_cavities_p4(cavities, precision, gpu):
    from paper_2312_14167_amd import Solver
    c = cavities
    sol = Solver(c["mesh"], 4, c["fp"], equations="ns", precision=precision, probes=c["probes"],
                 probe_mesh=np.arange(3), max_samples=CAV_STEPS, forces=True)
    dt = torch.tensor(CAV_DT, dtype=torch.float64, device=gpu)
    u = c["u0"].to(device=gpu, dtype=sol.dtype)
    tiles = sol.autotune(u, dt, reps=1)
    R = sol.rhs(u)
    sol.reset_accumulators()
    sol.rk_step(u, dt, 1, sample_every=1)
    u1 = u.clone()
    sol.rk_step(u, dt, CAV_STEPS - 1, sample_every=1)
    torch.cuda.synchronize()
    st = sol.probe_oaspl(p_ref=2e-5)
    ser = sol.probe_series(CAV_STEPS)
    eR, e1, eN = rel_l2(R, c["R0"]), rel_l2(u1, c["u1"]), rel_l2(u, c["uN"])
    P, F = c["P"], c["F"]
    dp = float(np.abs(ser.T - P).max() / np.abs(P).max())
    Fm = F.mean(axis=0)
    dF = float(np.abs(st["mean_force"] - Fm).max() / np.abs(Fm).max())
    dprms = float(np.abs(st["prms"] - P.std(axis=0)).max() / P.std(axis=0).max())
    walls = boundary_elements(c["mesh"], fi.BC_WALL)
    ew = per_var_max(R, c["R0"], walls)
    print(f"3 cavities {c['counts']} p=4 {precision} (tiles {tiles}): residual {eR:.3e}, 1 step {e1:.3e}, "
          f"{CAV_STEPS} steps {eN:.3e}; wall elements pointwise residual {ew:.3e}; probe series {dp:.3e}, "
          f"p_rms {dprms:.3e}, mean force {dF:.3e}")
    assert st["n_samples"] == CAV_STEPS
    if precision == "fp64":
        assert eR <= 1e-11 and e1 <= 1e-12 and eN <= 1e-12, (eR, e1, eN)
        assert ew <= 1e-11 and dp <= 1e-13 and dF <= 1e-11 and dprms <= 1e-9, (ew, dp, dF, dprms)
    else:
        # p_RMS of FP32 states: the FP64 probe pressure carries the state's rounding,
        # ~ eps_32 p_inf absolute, against the series' fluctuation sigma
        sig = float(P.std(axis=0).min())
        assert e1 <= 1e-5 and eN <= 1e-5, (e1, eN)
        assert eR <= 3e-4 and ew <= 1.5e-4 and dp <= 2e-6 and dF <= 1e-6, (eR, ew, dp, dF)
        assert dprms <= 2 * 6e-8 * float(c["fp"].p_inf.max()) / sig, (dprms, sig)
    sol.close()


# ----------------------------------------------------------------------------- non-finite state
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_in_state_reports_nonfinite(precision, gpu):
    """A NaN written from the host into the probe's element: the sampled probe pressure is not
    finite, so fr_probe_oaspl returns FR_ERR_NONFINITE; after a reset and a finite state it
    returns FR_OK again."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd._lib import FR_ERR_NONFINITE, FrError
    m = fi.o_grid(24, 8, q=4, r1=6.0, stretch=1.2, seed=3)
    fp = fi.freestream_params(2, 0.2, 1000.0)
    s = OracleSystem(m, 4, fp, equations="ns", probes=[[0.0, 3.0]])
    e = s.probes[0][0]
    u0 = torch.tensor(fi.developed_state(s.solpt_coords(), fp, 3)).permute(0, 2, 1).contiguous()
    sol = Solver(m, 4, fp, equations="ns", precision=precision, probes=[[0.0, 3.0]], max_samples=4, forces=True)
    dt = torch.tensor([2e-4], dtype=torch.float64, device=gpu)
    u = u0.to(device=gpu, dtype=sol.dtype)
    sol.reset_accumulators()
    sol.rk_step(u, dt, 1, sample_every=1)
    assert sol.probe_oaspl(p_ref=2e-5)["n_samples"] == 1
    bad = u.clone()
    bad[e, 0, 3] = float("nan")
    sol.rk_step(bad, dt, 1, sample_every=1)
    with pytest.raises(FrError) as exc:
        sol.probe_oaspl(p_ref=2e-5)
    assert exc.value.status == FR_ERR_NONFINITE
    sol.reset_accumulators()
    sol.rk_step(u, dt, 1, sample_every=1)
    st = sol.probe_oaspl(p_ref=2e-5)
    assert st["n_samples"] == 1 and np.isfinite(st["prms"]).all()
    sol.close()
