"""Thin host driver of the gradient-free optimiser (the MADS iteration of Algorithm 1 with the
OrthoMADS poll directions), whose poll candidates are evaluated together as one batched solve.

Algorithm 1 (Optimization Framework section):
* the mesh size Delta^m is capped at its initial value Delta^m_0;
* poll size Delta^p = n sqrt(Delta^m) (minimal positive basis) or sqrt(Delta^m) (maximal);
* the candidates of one poll are evaluated together (all at once, "in parallel");
* success (a candidate below the incumbent): Delta^m <- 4 Delta^m and the best candidate becomes
  the incumbent; failure: Delta^m <- Delta^m / 4;
* stop when Delta^m < 1e-6 and the design changed by less than 1 % between two iterations.

Poll directions (OrthoMADS, cited by the paper): the t-th point u of the Halton sequence gives
the direction q = round(a (2u - 1) / |2u - 1|) with a chosen so |q|^2 is the largest integer
vector norm not above Delta^p / Delta^m; the Householder matrix H = |q|^2 I - 2 q q^T has
orthogonal integer columns, and the poll points are x + Delta^m h for the columns h of [H, -H]
(maximal basis, 2n points) or of [H, -sum of H's columns] (minimal basis, n + 1 points).  Points
outside the bounds are not evaluated (extreme barrier: +inf).  Readings where the paper is
silent: the Halton index advances by one per iteration; the incumbent design is the best point
ever evaluated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_PRIMES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def halton(t: int, n: int) -> np.ndarray:
    """t-th point (t >= 1) of the n-dimensional Halton sequence (radical inverses in the first n
    primes)."""
    if n > len(_PRIMES):
        raise ValueError("at most 12 design parameters")
    out = np.zeros(n)
    for k in range(n):
        b, f, i, r = _PRIMES[k], 1.0, t, 0.0
        while i > 0:
            f /= b
            r += f * (i % b)
            i //= b
        out[k] = r
    return out


def orthomads_directions(t: int, n: int, ratio: float, maximal: bool) -> np.ndarray:
    """Integer poll directions (columns) for Halton index t and ratio Delta^p / Delta^m."""
    u = 2.0 * halton(t, n) - 1.0
    nu = np.linalg.norm(u)
    if nu == 0.0:
        u, nu = np.ones(n), math.sqrt(n)
    d = u / nu
    # the columns of H have norm |q|^2, so the poll distance Delta^m |q|^2 matches Delta^p when
    # |q| ~ sqrt(ratio): largest a with |round(a d)| <= sqrt(ratio) (at least a unit vector)
    ratio = math.sqrt(max(ratio, 1.0))
    q = np.round(d).astype(np.int64)
    a, step = 1.0, 1.0
    while step > 1e-3:
        cand = np.round((a + step) * d).astype(np.int64)
        if np.linalg.norm(cand) <= max(ratio, 1.0):
            a += step
            q = cand
        else:
            step /= 2.0
    if not q.any():
        q[int(np.argmax(np.abs(d)))] = 1
    H = float(q @ q) * np.eye(n, dtype=np.int64) - 2 * np.outer(q, q)
    H = H.astype(np.int64)
    if maximal:
        return np.concatenate([H, -H], axis=1)
    return np.concatenate([H, -H.sum(axis=1, keepdims=True)], axis=1)


@dataclass
class MadsState:
    x: np.ndarray                      # incumbent design
    f: float                           # incumbent objective
    delta_m0: float
    delta_m: float
    maximal: bool = True
    lower: np.ndarray | None = None
    upper: np.ndarray | None = None
    k: int = 0                         # poll iteration
    successes: int = 0
    history: list = field(default_factory=list)
    x_prev: np.ndarray | None = None

    @property
    def n(self) -> int:
        return len(self.x)

    def poll_size(self) -> float:
        return self.n * math.sqrt(self.delta_m) if not self.maximal else math.sqrt(self.delta_m)

    def poll_points(self) -> np.ndarray:
        """Candidate designs of the current poll, [n_candidates, n]."""
        self.delta_m = min(self.delta_m, self.delta_m0)
        D = orthomads_directions(self.k + 1, self.n, self.poll_size() / self.delta_m, self.maximal)
        return self.x[None, :] + self.delta_m * D.T

    def feasible(self, pts: np.ndarray) -> np.ndarray:
        ok = np.ones(len(pts), dtype=bool)
        if self.lower is not None:
            ok &= (pts >= self.lower).all(axis=1)
        if self.upper is not None:
            ok &= (pts <= self.upper).all(axis=1)
        return ok

    def update(self, pts: np.ndarray, f: np.ndarray) -> bool:
        """Apply Algorithm 1's success / failure rule to the evaluated poll."""
        self.x_prev = self.x.copy()
        i = int(np.argmin(f))
        success = bool(f[i] < self.f)
        if success:
            self.x, self.f = pts[i].copy(), float(f[i])
            self.delta_m *= 4.0
            self.successes += 1
        else:
            self.delta_m /= 4.0
        self.k += 1
        self.history.append({"k": self.k, "f": self.f, "x": self.x.copy(), "delta_m": self.delta_m,
                             "success": success, "n_candidates": len(pts)})
        return success

    def converged(self, tol_mesh: float = 1e-6, tol_change: float = 0.01) -> bool:
        if self.x_prev is None or self.delta_m >= tol_mesh:
            return False
        scale = np.where(np.abs(self.x_prev) > 0, np.abs(self.x_prev), 1.0)
        return bool(np.max(np.abs(self.x - self.x_prev) / scale) < tol_change)


def minimize(evaluate_batch, x0, delta_m0: float, lower=None, upper=None, maximal: bool = True,
             max_polls: int = 200, tol_mesh: float = 1e-6) -> MadsState:
    """Algorithm 1.  ``evaluate_batch(points [m, n]) -> objectives [m]`` evaluates all candidates
    of one poll together (the batched solve); the baseline is evaluated first on its own."""
    x0 = np.asarray(x0, float)
    f0 = float(np.asarray(evaluate_batch(x0[None, :]))[0])
    st = MadsState(x=x0.copy(), f=f0, delta_m0=delta_m0, delta_m=delta_m0, maximal=maximal,
                   lower=None if lower is None else np.asarray(lower, float),
                   upper=None if upper is None else np.asarray(upper, float))
    for _ in range(max_polls):
        pts = st.poll_points()
        ok = st.feasible(pts)
        f = np.full(len(pts), np.inf)
        if ok.any():
            f[ok] = np.asarray(evaluate_batch(pts[ok]), float)
        st.update(pts, f)
        if st.converged(tol_mesh):
            break
    return st


def naca_objective(oaspl: np.ndarray, cl: np.ndarray, cd: np.ndarray, cl_base: float, cd_base: float,
                   eps1: float = 8000.0, eps2: float = 400000.0) -> np.ndarray:
    """Penalised airfoil objective of the NACA optimisation: OASPL + eps1 (C_L - C_L,base)^2, plus
    eps2 (C_D - C_D,base)^2 when the mean drag exceeds the baseline's."""
    oaspl, cl, cd = (np.asarray(a, float) for a in (oaspl, cl, cd))
    f = oaspl + eps1 * (cl - cl_base) ** 2
    return np.where(cd > cd_base, f + eps2 * (cd - cd_base) ** 2, f)
