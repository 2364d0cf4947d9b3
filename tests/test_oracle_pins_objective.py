"""Pins of the oracle's force coefficients (Eq. (8)) and of the airfoil case's penalised objective
(CPU only): hand-computed values, invariance under a rotation of flow and force together, and
the two branches of the objective with their junction."""
import math

import numpy as np

from oracle import airfoil_objective, force_coefficients


def test_force_coefficient_hand_computed():
    """F = (3, 4), rho = 1.2, U = (2, 0), area 0.5: dynamic pressure 0.5 * 1.2 * 4 = 2.4, so
    C_x = 3 / (2.4 * 0.5) = 2.5 and C_y = 4 / 1.2 = 10/3; along (0.6, 0.8): (1.8 + 3.2) / 1.2."""
    c = force_coefficients(np.array([[3.0, 4.0]]), [1.2], [[2.0, 0.0]],
                           np.array([[[1.0, 0.0], [0.0, 1.0], [0.6, 0.8]]]), [0.5])
    np.testing.assert_allclose(c[0], [2.5, 10.0 / 3.0, 5.0 / 1.2], rtol=1e-15)


def test_force_coefficients_invariant_under_rotation():
    """Drag along the free stream and lift normal to it do not change when the free stream and the
    force rotate together (angle of attack applied to both), in 2-D and 3-D (rotation about z);
    several meshes at once with their own free streams and areas."""
    rng = np.random.default_rng(3)
    for d in (2, 3):
        n = 4
        F = rng.normal(size=(n, d))
        U = np.zeros((n, d))
        U[:, 0] = rng.uniform(0.5, 2.0, n)
        rho = rng.uniform(0.8, 1.2, n)
        area = rng.uniform(0.1, 1.0, n)

        def dirs(Uv):
            e = Uv / np.linalg.norm(Uv, axis=1, keepdims=True)
            lift = np.zeros_like(e)
            lift[:, 0], lift[:, 1] = -e[:, 1], e[:, 0]
            return np.stack([e, lift], axis=1)
        c0 = force_coefficients(F, rho, U, dirs(U), area)
        a = rng.uniform(0, 2 * np.pi, n)
        R = np.zeros((n, d, d))
        R[:, 0, 0], R[:, 0, 1], R[:, 1, 0], R[:, 1, 1] = np.cos(a), -np.sin(a), np.sin(a), np.cos(a)
        if d == 3:
            R[:, 2, 2] = 1.0
        Fr = np.einsum('nij,nj->ni', R, F)
        Ur = np.einsum('nij,nj->ni', R, U)
        c1 = force_coefficients(Fr, rho, Ur, dirs(Ur), area)
        np.testing.assert_allclose(c1, c0, rtol=1e-12, atol=1e-14)
        # the drag coefficient is the streamwise force over 1/2 rho U^2 A
        np.testing.assert_allclose(c0[:, 0], F[:, 0] / (0.5 * rho * U[:, 0] ** 2 * area), rtol=1e-14)


def test_airfoil_objective_branches():
    """Below or at the baseline drag only the lift penalty applies; above it the drag penalty is
    added; the objective is continuous where the drag crosses its baseline."""
    assert math.isclose(airfoil_objective(110.0, 0.66, 0.05, 0.65, 0.055), 110.0 + 8000.0 * 0.01 ** 2,
                        rel_tol=1e-14)
    assert math.isclose(airfoil_objective(110.0, 0.65, 0.06, 0.65, 0.055), 110.0 + 400000.0 * 0.005 ** 2,
                        rel_tol=1e-15)
    f0 = airfoil_objective(100.0, 0.7, 0.05, 0.6, 0.05)
    f1 = airfoil_objective(100.0, 0.7, 0.05 + 1e-12, 0.6, 0.05)
    assert math.isclose(f0, 100.0 + 8000.0 * 0.1 ** 2, rel_tol=1e-14) and abs(f1 - f0) < 1e-12
