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
