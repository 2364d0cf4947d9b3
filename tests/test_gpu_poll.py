"""A MADS poll of the airfoil problem evaluated as one batched solve: the candidates' objectives
from the concatenated-mesh solver equal those of separate single-design solves, and Algorithm 1
runs on top of the batched evaluator."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GRID = dict(n_wake=3, n_foil=8, n_normal=3, n_span=2, q=2, r_out=4.0, x_out=6.0, h_wall=0.05)


def test_batched_poll_equals_separate_solves(gpu):
    from paper_2312_14167_amd.poll import naca_poll
    designs = np.array([[0.0, 4.0, 12.0, 6.0], [2.0, 4.0, 12.0, 6.0], [0.0, 6.0, 10.0, 4.0]])
    kw = dict(grid=GRID, p=2, steps=12, dt=2e-4, precision="fp64", cl_base=0.6, cd_base=0.05)
    b = naca_poll(designs, **kw)
    assert b["finite"] and b["n_samples"] == 12
    for k, x in enumerate(designs):
        s = naca_poll(x[None, :], **kw)
        print(f"design {x}: OASPL {b['oaspl'][k]:.6f} / {s['oaspl'][0]:.6f}, CL {b['cl'][k]:.6e}, CD {b['cd'][k]:.6e}")
        assert abs(b["oaspl"][k] - s["oaspl"][0]) <= 1e-9 * abs(s["oaspl"][0])
        np.testing.assert_allclose([b["cl"][k], b["cd"][k]], [s["cl"][0], s["cd"][0]], rtol=1e-10, atol=1e-14)
        assert abs(b["objective"][k] - s["objective"][0]) <= 1e-9 * abs(s["objective"][0])


def test_mads_iterations_on_batched_polls(gpu):
    from paper_2312_14167_amd.mads import minimize
    from paper_2312_14167_amd.poll import naca_poll
    calls = []

    def evaluate(P):
        calls.append(len(P))
        r = naca_poll(P, grid=GRID, p=2, steps=12, dt=2e-4, precision="fp64", cl_base=0.6, cd_base=0.05)
        return r["objective"]
    st = minimize(evaluate, [0.0, 4.0, 12.0, 6.0], 1.0, lower=[-10, 4, 6, 0], upper=[10, 9, 18, 12], max_polls=2)
    assert calls[0] == 1 and all(c <= 8 for c in calls[1:]) and len(st.history) == 2
    assert np.isfinite(st.f)


def test_batched_poll_matches_oracle(gpu):
    """Each candidate's OASPL (Eqs. (9)-(12)), mean C_L and C_D (Eq. (8)) and penalised objective
    from the batched poll against the FP64 oracle run on that candidate's own mesh: probe series ->
    OASPL, time-mean wall force -> coefficients (oracle functions), then the objective."""
    import torch

    import fr_inputs as fi
    from oracle import OracleSystem, airfoil_objective, force_coefficients, oaspl_from_series
    from paper_2312_14167_amd.poll import naca_candidate_mesh, naca_poll
    designs = np.array([[0.0, 4.0, 12.0, 6.0], [2.0, 4.0, 12.0, 6.0], [-1.0, 6.0, 10.0, 3.0]])
    steps, dt, span = 12, 2e-4, 0.2
    b = naca_poll(designs, grid=GRID, p=2, steps=steps, dt=dt, precision="fp64", cl_base=0.6, cd_base=0.05)
    for k, x in enumerate(designs):
        m = naca_candidate_mesh(x, GRID)
        fp = fi.freestream_params(3, 0.2, 23000.0)
        a = np.deg2rad(x[3])
        fp.vel_inf[0] = [np.cos(a), np.sin(a), 0.0]
        s = OracleSystem(m, 2, fp, equations="ns", probes=[[1.0, -2.0, 0.5 * span]])
        u0 = torch.tensor(fi.freestream_state(s.solpt_coords(), fp)).permute(0, 2, 1).contiguous()
        _, P, F = s.run(u0, torch.tensor([dt], dtype=torch.float64), steps, sample_every=1)
        oaspl = oaspl_from_series(P[:, 0].numpy(), 2e-5 * fp.p_inf[0] / 101325.0)
        ed = fp.vel_inf[0] / np.linalg.norm(fp.vel_inf[0])
        el = np.array([-ed[1], ed[0], 0.0])
        cd, cl = force_coefficients(F.numpy().mean(axis=0), fp.rho_inf, fp.vel_inf, np.stack([ed, el])[None],
                                    [span])[0]
        obj = airfoil_objective(oaspl, cl, cd, 0.6, 0.05)
        # scale of the coefficients' round-off: the pressure integral ~ p_inf over the dynamic pressure
        cscale = fp.p_inf[0] / (0.5 * fp.rho_inf[0])
        print(f"design {x}: OASPL {b['oaspl'][k]:.9f} / oracle {oaspl:.9f} dB; C_L {b['cl'][k]:.9e} / {cl:.9e}; "
              f"C_D {b['cd'][k]:.9e} / {cd:.9e}; objective {b['objective'][k]:.9f} / {obj:.9f}")
        # p_RMS of a pressure of size p_inf fluctuating by sigma carries FP64 rounding of relative
        # size eps p_inf / sigma (sigma ~ 1e-8 here: 12 steps from a uniform start), and the dB value
        # 20 log10(p_RMS / p_ref) moves by 20 / ln 10 times that
        sig = float(P[:, 0].numpy().std())
        tol_db = 20.0 / np.log(10.0) * 1.1e-16 * fp.p_inf[0] / sig
        assert abs(b["oaspl"][k] - oaspl) <= tol_db, (b["oaspl"][k] - oaspl, tol_db)
        assert abs(b["cl"][k] - cl) <= 1e-11 * cscale and abs(b["cd"][k] - cd) <= 1e-11 * cscale
        assert abs(b["objective"][k] - obj) <= tol_db + 1e-11 * abs(obj)
