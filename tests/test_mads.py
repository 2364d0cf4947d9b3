"""The MADS host driver (Algorithm 1 with OrthoMADS poll directions) on closed-form problems:
Halton points, orthogonal integer positive-spanning directions, the mesh-size rules and the stop
rule, convergence on a bounded quadratic, and the penalised airfoil objective."""
import numpy as np

from paper_2312_14167_amd.mads import MadsState, halton, minimize, naca_objective, orthomads_directions


def test_halton_radical_inverses():
    np.testing.assert_allclose(halton(1, 3), [0.5, 1 / 3, 0.2])
    np.testing.assert_allclose(halton(6, 2), [0.375, 2 / 9])  # 6 = 110b -> .011b ; 6 = 20_3 -> .02_3


def test_orthomads_directions_orthogonal_integer_and_spanning():
    rng = np.random.default_rng(0)
    for t in range(1, 30):
        for n in (1, 2, 4):
            for maximal in (True, False):
                D = orthomads_directions(t, n, 16.0, maximal)
                assert D.dtype.kind == "i"
                H = D[:, :n]
                G = H.T @ H
                assert np.all(G == np.diag(np.diag(G))) and np.all(np.diag(G) == np.diag(G)[0])
                assert D.shape[1] == (2 * n if maximal else n + 1)
                for _ in range(20):  # positive spanning: every direction has a poll column within 90 deg
                    v = rng.normal(size=n)
                    assert (v @ D).max() > 0


def test_mesh_size_rules_and_poll_size():
    st = MadsState(x=np.zeros(2), f=1.0, delta_m0=1.0, delta_m=1.0, maximal=True)
    pts = st.poll_points()
    assert pts.shape == (4, 2)
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0)         # Delta^p = sqrt(Delta^m) = 1
    st.update(pts, np.full(4, 2.0))                               # failure
    assert st.delta_m == 0.25 and st.f == 1.0
    f = np.full(4, 2.0)
    f[1] = 0.5
    pts = st.poll_points()
    st.update(pts, f)                                             # success
    assert st.delta_m == 1.0 and st.f == 0.5 and np.allclose(st.x, pts[1])
    st.update(st.poll_points(), np.array([0.1, 1, 1, 1]))
    assert st.delta_m == 4.0
    st.poll_points()
    assert st.delta_m == 1.0                                      # capped at Delta^m_0
    mn = MadsState(x=np.zeros(3), f=1.0, delta_m0=1.0, delta_m=1.0 / 16, maximal=False)
    assert mn.poll_size() == 3 * 0.25                             # n sqrt(Delta^m)
    assert mn.poll_points().shape == (4, 3)


def test_minimize_bounded_quadratic_converges():
    c = np.array([0.7, -1.3, 2.2])
    w = np.array([1.0, 3.0, 0.5])
    calls = []

    def batch(P):
        calls.append(len(P))
        return ((P - c) ** 2 * w).sum(axis=1)
    for maximal in (True, False):
        calls.clear()
        st = minimize(batch, np.zeros(3), 1.0, lower=[-5, -5, -5], upper=[5, 5, 5], maximal=maximal, max_polls=400)
        assert np.abs(st.x - c).max() < 2e-2, (maximal, st.x)
        assert calls[0] == 1 and max(calls[1:]) == (6 if maximal else 4)   # one batch per poll
    # a bound excludes the minimiser: the driver stays feasible and reaches the bound
    st = minimize(batch, np.zeros(3), 1.0, lower=[-5, -5, -5], upper=[5, 5, 1.0], max_polls=400)
    assert st.x[2] <= 1.0 and abs(st.x[2] - 1.0) < 2e-2


def test_naca_penalised_objective():
    f = naca_objective([100.0, 100.0], [0.7, 0.6], [0.05, 0.06], cl_base=0.65, cd_base=0.055)
    np.testing.assert_allclose(f, [100 + 8000 * 0.05 ** 2, 100 + 8000 * 0.05 ** 2 + 400000 * 0.005 ** 2])
