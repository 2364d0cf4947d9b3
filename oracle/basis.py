"""1-D and tensor-product FR operators (oracle; test infrastructure only).

Flux reconstruction as introduced by Huynh (cited in the flow-solver
subsection): inside an element the solution is the Lagrange interpolant
through the solution points; the flux derivative is corrected with the
derivative of a correction function g that is 1 at its own face and 0 at the
opposite face.  Reading taken: Gauss-Legendre solution points and Huynh's
g_DG, g_R = (P_{p+1} + P_p) / 2 (right face) and g_L(x) = g_R(-x).
"""
from __future__ import annotations

import itertools

import numpy as np


def gauss_legendre(P: int):
    """P Gauss-Legendre points and weights on [-1, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(P)
    return x, w


def gll_nodes(q: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes of degree q: -1, roots of P_q', +1."""
    if q == 1:
        return np.array([-1.0, 1.0])
    r = np.sort(np.polynomial.legendre.Legendre.basis(q).deriv().roots().real)
    return np.concatenate([[-1.0], r, [1.0]])


def lagrange_eval(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[a, j] = l_j(x_a), the Lagrange basis through ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    L = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_deriv(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dL[a, j] = l_j'(x_a) by the product rule (sum over the dropped factor)."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    dL = np.zeros((len(x), n))
    for j in range(n):
        for r in range(n):
            if r == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[r]))
            for m in range(n):
                if m != j and m != r:
                    term = term * (x - nodes[m]) / (nodes[j] - nodes[m])
            dL[:, j] += term
    return dL


def correction_deriv(p: int, x: np.ndarray) -> np.ndarray:
    """g_R'(x) for Huynh's g_DG right correction function (1 at x = +1, 0 at x = -1)."""
    leg = np.polynomial.legendre.Legendre
    g = 0.5 * (leg.basis(p + 1) + leg.basis(p))
    return g.deriv()(np.asarray(x, float))


class TensorOps:
    """Dense tensor-product operators of one element in ``dim`` dimensions at degree ``p``.

    Solution points: lexicographic multi-index (i_0 fastest).  Face f lies on reference
    coordinate k = f // 2 at side s = -1 (f even) or +1 (f odd); its flux points carry the
    Gauss points of the other coordinates in lexicographic order (lowest coordinate
    fastest); flux point index = f * P**(dim-1) + t.
    """

    def __init__(self, dim: int, p: int):
        self.dim, self.p = dim, p
        P = p + 1
        self.P = P
        self.xi, self.w = gauss_legendre(P)
        self.Ns = P ** dim
        self.Nfp = P ** (dim - 1)
        self.Nf = 2 * dim * self.Nfp
        self.nv = dim + 2
        self.D1 = lagrange_deriv(self.xi, self.xi)            # D1[a, b] = l_b'(xi_a)
        self.lm = lagrange_eval(self.xi, np.array([-1.0]))[0]  # l_b(-1)
        self.lp = lagrange_eval(self.xi, np.array([1.0]))[0]   # l_b(+1)
        self.sol_idx = np.array(list(itertools.product(range(P), repeat=dim)))[:, ::-1]  # [Ns, dim], i_0 fastest
        # flux points: (face, tangential multi-index)
        fk, fs, ft = [], [], []
        for f in range(2 * dim):
            k = f // 2
            s = -1 if f % 2 == 0 else 1
            others = [m for m in range(dim) if m != k]
            for t in itertools.product(range(P), repeat=dim - 1):
                t = t[::-1]  # lowest remaining coordinate fastest
                fk.append(k)
                fs.append(s)
                ft.append(dict(zip(others, t)))
        self.fpt_k = np.array(fk)
        self.fpt_s = np.array(fs)
        self.fpt_t = ft
        Ns, Nf = self.Ns, self.Nf
        # D_k: derivative along reference coordinate k
        self.Dk = np.zeros((dim, Ns, Ns))
        for k in range(dim):
            for i in range(Ns):
                for j in range(Ns):
                    ii, jj = self.sol_idx[i], self.sol_idx[j]
                    if all(ii[m] == jj[m] for m in range(dim) if m != k):
                        self.Dk[k, i, j] = self.D1[ii[k], jj[k]]
        gp = correction_deriv(p, self.xi)   # g_R'(xi_a)
        gm = correction_deriv(p, -self.xi)  # g_R'(-xi_a)
        self.M0 = np.zeros((Nf, Ns))
        self.Lift = np.zeros((Ns, Nf))      # g_R'(s_f xi_i^(k_f)) on the line of f
        self.LiftG = np.zeros((dim, Ns, Nf))  # s_f g_R'(s_f xi_i^(k)) for faces with k_f = k
        for f in range(Nf):
            k, s, t = self.fpt_k[f], self.fpt_s[f], self.fpt_t[f]
            for i in range(Ns):
                ii = self.sol_idx[i]
                if all(ii[m] == t[m] for m in t):
                    self.M0[f, i] = (self.lp if s > 0 else self.lm)[ii[k]]
                    g = gp[ii[k]] if s > 0 else gm[ii[k]]
                    self.Lift[i, f] = g
                    self.LiftG[k, i, f] = s * g
        # face quadrature weight of each flux point (product of tangential Gauss weights)
        self.fpt_w = np.array([np.prod([self.w[t[m]] for m in t]) if t else 1.0 for t in self.fpt_t])
        self.sol_w = np.prod(self.w[self.sol_idx], axis=1)

    def ref_solpts(self) -> np.ndarray:
        return self.xi[self.sol_idx]  # [Ns, dim]

    def ref_fpts(self) -> np.ndarray:
        pts = np.zeros((self.Nf, self.dim))
        for f in range(self.Nf):
            pts[f, self.fpt_k[f]] = self.fpt_s[f]
            for m, tm in self.fpt_t[f].items():
                pts[f, m] = self.xi[tm]
        return pts

    def interp_weights(self, xi_p: np.ndarray) -> np.ndarray:
        """Tensor Lagrange weights of all solution points at reference point ``xi_p``."""
        w = np.ones(self.Ns)
        for k in range(self.dim):
            lk = lagrange_eval(self.xi, np.array([xi_p[k]]))[0]
            w = w * lk[self.sol_idx[:, k]]
        return w
