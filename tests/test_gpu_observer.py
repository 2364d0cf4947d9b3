"""Spanwise observer statistics: several probes along the span of the extruded C-grid sampled by
the FP64 accumulator over RK4 steps; the library's host statistics of the GPU series (cumulative
p_RMS vectors, observer OASPL averaged over the span, Welch PSD) against the oracle's statistics
of the oracle's own trajectory.  The fluctuation sigma is ~1e-3 of p_inf, so relative agreement of
the series to ~1e-13 gives ~1e-9 on RMS-derived quantities."""
import numpy as np
import pytest
import torch

from cases import make_case

pytestmark = pytest.mark.gpu


def test_spanwise_observer_oaspl_and_psd_match_oracle(gpu):
    from oracle import OracleSystem, cumulative_prms, observer_oaspl, welch_psd
    from paper_2312_14167_amd import Solver
    m, p, fp, eq, init, dt, _ = make_case("ns_cgrid_p4")
    zs = [0.01, 0.06, 0.11, 0.16]
    probes = [[1.0, -2.0, z] for z in zs] + [[0.2, 0.8, z] for z in zs]
    groups = np.array([0] * 4 + [1] * 4)
    K = 48
    s = OracleSystem(m, p, fp, equations=eq, probes=probes)
    u0 = torch.tensor(init(s.solpt_coords())).permute(0, 2, 1).contiguous()
    _, P, _ = s.run(u0, torch.tensor(dt), K, sample_every=1, forces=False)
    P = P.numpy().T                                     # [n_probe, K]
    sol = Solver(m, p, fp, equations=eq, probes=probes, max_samples=K)
    u = u0.to(gpu).clone()
    sol.reset_accumulators()
    sol.rk_step(u, torch.tensor(dt, dtype=torch.float64, device=gpu), K, sample_every=1)
    st = sol.probe_statistics(p_ref=2e-5, groups=groups, n_windows=3, sample_dt=float(dt[0]), cap=K)
    rp, rd = observer_oaspl(P, groups, 2, 2e-5)
    cum = np.stack([cumulative_prms(P[a]) for a in range(len(probes))])
    f, psd = welch_psd(P[0], 3, float(dt[0]))
    e_cum = float(np.abs(st["prms_cumulative"][:, 1:] - cum[:, 1:]).max() / np.abs(cum[:, 1:]).max())
    e_rms = float(np.abs(st["observer_prms"] - rp).max() / rp.max())
    e_psd = float(np.abs(st["psd"][0] - psd).max() / psd.max())
    print(f"observer OASPL {st['observer_oaspl']} dB; rel err: cumulative {e_cum:.2e}, observer RMS {e_rms:.2e}, "
          f"PSD {e_psd:.2e}")
    assert e_cum <= 1e-8 and e_rms <= 1e-8 and e_psd <= 1e-7
    np.testing.assert_allclose(st["observer_oaspl"], rd, rtol=0, atol=1e-7)
    np.testing.assert_allclose(st["freq"], f, rtol=1e-13)
