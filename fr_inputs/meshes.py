"""Seeded synthetic high-order meshes (quads / hexes with curved geometry).

Mesh description format (the input contract shared by the oracle and the library)
----------------------------------------------------------------------------------
* ``node_xyz``  float64 ``[n_node, dim]`` physical node coordinates.
* ``elem_nodes`` int64 ``[n_elem, (q+1)**dim]``: the element's geometry nodes,
  which sit at the tensor-product Gauss-Lobatto-Legendre (GLL) points of degree
  ``q`` of the reference cube ``[-1, 1]**dim``, listed lexicographically with the
  first reference coordinate fastest.  Every element must be right-handed.
* ``face_bc`` int32 ``[n_elem, 2*dim]``: per reference face ``f`` (face ``f`` lies
  on reference coordinate ``k = f // 2`` at ``-1`` for even ``f`` and ``+1`` for odd
  ``f``) a tag: ``FACE_AUTO`` (matched geometrically with another element's face,
  directly or after a periodic translation), ``BC_WALL`` (adiabatic no-slip wall)
  or ``BC_FARFIELD`` (characteristic far field).
* ``periodic_vec`` float64 ``[n_per, dim]``: translations under which two
  ``FACE_AUTO`` faces are identified.
* ``mesh_elem_begin`` int64 ``[n_mesh + 1]``: disjoint element ranges when several
  independent meshes are concatenated (one design per range).

The synthetic workloads follow the shapes of the paper's cases (Sections 3-5):
an O-grid around a cylinder (tandem-cylinder section), an extruded C-grid around
a NACA 4-digit section (airfoil section) and a family of open cavities (cavity
section); plus periodic boxes for the closed-form tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FACE_AUTO = 0
BC_WALL = 1
BC_FARFIELD = 2


@dataclass
class MeshDesc:
    dim: int
    q: int
    node_xyz: np.ndarray
    elem_nodes: np.ndarray
    face_bc: np.ndarray
    periodic_vec: np.ndarray
    mesh_elem_begin: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.elem_nodes.shape[0])

    @property
    def n_mesh(self) -> int:
        return int(self.mesh_elem_begin.shape[0] - 1)


def gll_points(q: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points of degree q on [-1, 1] (q+1 points, ascending).

    Used only to *place* geometry nodes; the endpoints are exactly +-1 and the
    interior points are the roots of P_q'.
    """
    if q < 1:
        raise ValueError("geometry degree must be >= 1")
    if q == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(q).deriv().roots()
    pts = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    # symmetrise to remove root-finder noise
    return 0.5 * (pts - pts[::-1])


def _param_nodes(lines: np.ndarray, q: int, wrap: bool):
    """Node parameter values along one structured direction.

    Returns (values, cell, frac): the parameter value of every node, the cell it is
    attributed to and its local fraction in [0, 1] (for continuity-preserving maps).
    """
    n = len(lines) - 1
    g = (gll_points(q) + 1.0) * 0.5
    nn = n * q + (0 if wrap else 1)
    vals = np.empty(nn)
    cell = np.empty(nn, dtype=np.int64)
    frac = np.empty(nn)
    for c in range(n):
        for a in range(q + (1 if (c == n - 1 and not wrap) else 0)):
            idx = c * q + a
            if idx >= nn:
                continue
            vals[idx] = lines[c] + g[a] * (lines[c + 1] - lines[c])
            cell[idx] = c
            frac[idx] = g[a]
    return vals, cell, frac


def _structured(lines, q, mapfn, wrap, keep=None, bcfn=None, periodic_vec=None, info=None):
    """Build a structured (possibly masked / wrapped) high-order mesh.

    ``lines[k]``: cell boundaries of direction k in parameter space.
    ``mapfn(P, C, T)``: P param coords ``[..., d]``, C cell indices, T local fractions
    -> physical coordinates ``[..., d]``.
    ``keep(I)``: boolean mask over element grid indices ``I`` (tuple of arrays).
    ``bcfn(I, f)``: tag array for face f of elements with grid indices I.
    """
    d = len(lines)
    ncell = [len(l) - 1 for l in lines]
    pv = [_param_nodes(np.asarray(lines[k], float), q, wrap[k]) for k in range(d)]
    nnode_dim = [len(p[0]) for p in pv]
    # node grid, dim 0 fastest
    grids = np.meshgrid(*[p[0] for p in pv], indexing="ij")
    cells = np.meshgrid(*[p[1] for p in pv], indexing="ij")
    fracs = np.meshgrid(*[p[2] for p in pv], indexing="ij")
    P = np.stack(grids, axis=-1)
    C = np.stack(cells, axis=-1)
    T = np.stack(fracs, axis=-1)
    X = mapfn(P, C, T)
    # flatten with dim 0 fastest: transpose so that index order is (..., i1, i0)
    X = np.transpose(X, tuple(range(d - 1, -1, -1)) + (d,)).reshape(-1, d)

    def node_id(idx):
        nid = np.zeros_like(idx[0])
        stride = 1
        for k in range(d):
            nid = nid + (idx[k] % nnode_dim[k]) * stride
            stride *= nnode_dim[k]
        return nid

    egrid = np.meshgrid(*[np.arange(n) for n in ncell], indexing="ij")
    egrid = [np.transpose(g, tuple(range(d - 1, -1, -1))).reshape(-1) for g in egrid]
    if keep is not None:
        m = keep(tuple(egrid))
        egrid = [g[m] for g in egrid]
    ne = len(egrid[0])
    loc = np.meshgrid(*[np.arange(q + 1)] * d, indexing="ij")
    loc = [np.transpose(l, tuple(range(d - 1, -1, -1))).reshape(-1) for l in loc]
    idx = [egrid[k][:, None] * q + loc[k][None, :] for k in range(d)]
    en = node_id(idx)
    # compact unused nodes
    used = np.unique(en)
    remap = -np.ones(X.shape[0], dtype=np.int64)
    remap[used] = np.arange(len(used))
    en = remap[en]
    X = X[used]
    fb = np.zeros((ne, 2 * d), dtype=np.int32)
    if bcfn is not None:
        for f in range(2 * d):
            fb[:, f] = bcfn(tuple(egrid), f)
    pvec = np.zeros((0, d)) if periodic_vec is None else np.asarray(periodic_vec, float).reshape(-1, d)
    inf = dict(info or {})
    inf["grid_index"] = np.stack(egrid, axis=1)
    return MeshDesc(dim=d, q=q, node_xyz=np.ascontiguousarray(X), elem_nodes=np.ascontiguousarray(en.astype(np.int64)),
                    face_bc=fb, periodic_vec=pvec, mesh_elem_begin=np.array([0, ne], dtype=np.int64), info=inf)


def periodic_box(dim: int, n, lo=-5.0, hi=5.0, q: int = 1, curv: float = 0.0, seed: int | None = None,
                 bc: str = "periodic") -> MeshDesc:
    """Structured box [lo, hi]^dim with n cells per direction.

    ``curv`` > 0 applies a smooth, periodic-compatible sinusoidal deformation
    (amplitude ``curv`` times the cell size) so the elements are curved; with a
    seed the phases are random.  ``bc='periodic'`` identifies opposite sides;
    ``'farfield'`` tags every boundary face as far field; ``'channel'`` is periodic in
    x (and z) with adiabatic walls at the y-bounds.
    """
    n = [n] * dim if np.isscalar(n) else list(n)
    L = hi - lo
    lines = [np.linspace(lo, hi, n[k] + 1) for k in range(dim)]
    rng = np.random.default_rng(seed) if seed is not None else None
    ph = rng.uniform(0, 2 * np.pi, size=(dim, dim)) if rng is not None else np.zeros((dim, dim))
    h = L / max(n)

    def mapfn(P, C, T):
        # smooth deformation vanishing on the box boundary; in 3-D it depends on (x, y) only
        # and moves only x and y (an extruded curved mesh)
        X = P.copy()
        if curv != 0.0:
            s = np.ones(P.shape[:-1])
            for k in range(min(dim, 2)):
                s = s * np.sin(2 * np.pi * (P[..., k] - lo) / L)
            for k in range(min(dim, 2)):
                X[..., k] = P[..., k] + curv * h * s * np.cos(ph[k, 0])
        return X

    def bcfn(I, f):
        k, side = f // 2, f % 2
        at = (I[k] == 0) if side == 0 else (I[k] == n[k] - 1)
        tag = np.zeros(len(I[0]), dtype=np.int32)
        if bc == "farfield":
            tag[at] = BC_FARFIELD
        elif bc == "channel" and k == 1:
            tag[at] = BC_WALL
        return tag

    if bc == "periodic":
        pv = [L * np.eye(dim)[k] for k in range(dim)]
    elif bc == "channel":
        pv = [L * np.eye(dim)[k] for k in range(dim) if k != 1]
    else:
        pv = []
    return _structured(lines, q, mapfn, [False] * dim, bcfn=bcfn, periodic_vec=pv,
                       info={"kind": "box", "n": n, "lo": lo, "hi": hi, "curv": curv})


def o_grid(n_theta: int, n_r: int, r0: float = 0.5, r1: float = 30.0, stretch: float = 1.04, q: int = 4,
           perturb: float = 0.05, seed: int = 1, wall: str = "wall") -> MeshDesc:
    """O-grid around a cylinder of radius r0 out to r1 (2-D quads).

    Radial lines are geometrically stretched (ratio ``stretch``); interior corners
    get seeded displacements of at most ``perturb`` times the local spacing in r
    and in arc length, blended bilinearly inside each cell (the wall and the outer
    ring are not moved).  Reference direction 0 is radial, 1 is circumferential,
    so elements are right-handed.  ``wall='farfield'`` tags the inner ring as far
    field instead of a wall (free-stream tests).
    """
    s = stretch
    h0 = (r1 - r0) * (s - 1.0) / (s ** n_r - 1.0)
    rl = r0 + h0 * (s ** np.arange(n_r + 1) - 1.0) / (s - 1.0)
    rl[-1] = r1
    tl = np.linspace(0.0, 2 * np.pi, n_theta + 1)
    rng = np.random.default_rng(seed)
    dr = np.zeros((n_r + 1, n_theta))
    dt = np.zeros((n_r + 1, n_theta))
    dth = 2 * np.pi / n_theta
    for j in range(1, n_r):
        loc = min(rl[j] - rl[j - 1], rl[j + 1] - rl[j])
        dr[j] = rng.uniform(-perturb, perturb, n_theta) * loc
        dt[j] = rng.uniform(-perturb, perturb, n_theta) * dth
    # dt is an angular displacement: arc displacement = r * dt <= perturb * r * dth

    def mapfn(P, C, T):
        cr, ct = C[..., 0], C[..., 1]
        tr, tt = T[..., 0], T[..., 1]
        c0 = ct % n_theta
        c1 = (ct + 1) % n_theta

        def blend(a):
            return ((1 - tr) * (1 - tt) * a[cr, c0] + tr * (1 - tt) * a[cr + 1, c0]
                    + (1 - tr) * tt * a[cr, c1] + tr * tt * a[cr + 1, c1])
        r = P[..., 0] + blend(dr)
        th = P[..., 1] + blend(dt)
        return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)

    def bcfn(I, f):
        tag = np.zeros(len(I[0]), dtype=np.int32)
        if f == 0:
            tag[I[0] == 0] = BC_WALL if wall == "wall" else BC_FARFIELD
        elif f == 1:
            tag[I[0] == n_r - 1] = BC_FARFIELD
        return tag

    return _structured([rl, tl], q, mapfn, [False, True], bcfn=bcfn,
                       info={"kind": "o_grid", "n_theta": n_theta, "n_r": n_r, "r0": r0, "r1": r1,
                             "stretch": stretch, "perturb": perturb, "seed": seed,
                             "probe": np.array([0.0, 3.0]), "ref_length": 2 * r0})


def _stretched(x0, x1, h_first, ratio, ratio_buffer=None, x_buffer=None):
    """Cell boundaries from x0 towards x1 (either direction), first cell h_first,
    geometric growth ``ratio``; beyond |x - x0| > x_buffer the growth is ``ratio_buffer``.
    The last cell is merged so the final boundary is exactly x1."""
    sgn = 1.0 if x1 > x0 else -1.0
    L = abs(x1 - x0)
    pts = [0.0]
    h = h_first
    while pts[-1] + h < L - 1e-12:
        pts.append(pts[-1] + h)
        r = ratio
        if ratio_buffer is not None and x_buffer is not None and pts[-1] > x_buffer:
            r = ratio_buffer
        h *= r
    if len(pts) > 1 and L - pts[-1] < 0.5 * h / max(ratio, 1.0):
        pts[-1] = L
    else:
        pts.append(L)
    return x0 + sgn * np.array(pts)


def cavity(aspect: float, h: float = 0.1, q: int = 4, upstream: float = 5.0, top: float = 15.0,
           outflow: float = 60.0, top_buffer: float = 5.0, out_buffer: float = 50.0) -> MeshDesc:
    """Open cavity (2-D): cavity of width 1 (x in [0, 1]) and depth ``aspect`` below a flat
    plate (y = 0) that starts ``upstream`` widths ahead; domain top at ``top``, outflow at
    ``1 + outflow``.  Cells of size ``h`` in the cavity, growth 1.05 in the resolved region
    and 1.075 in the buffers (top ``top_buffer`` and last ``out_buffer`` widths).
    Walls: plate, cavity walls; far field: inlet, top, outlet.
    """
    W, D = 1.0, float(aspect)
    nxc = max(2, int(round(W / h)))
    xc = np.linspace(0.0, W, nxc + 1)
    hx = W / nxc
    xu = _stretched(0.0, -upstream, hx, 1.05)[::-1]
    xd = _stretched(W, W + outflow, hx, 1.05, 1.075, outflow - out_buffer)
    xl = np.concatenate([xu[:-1], xc, xd[1:]])
    nyc = max(2, int(round(D / h)))
    yc = np.linspace(-D, 0.0, nyc + 1)
    ya = _stretched(0.0, top, D / nyc, 1.05, 1.075, top - top_buffer)
    yl = np.concatenate([yc, ya[1:]])
    i_c0 = len(xu) - 1
    i_c1 = i_c0 + nxc
    j_0 = nyc

    def keep(I):
        inside_cav = (I[0] >= i_c0) & (I[0] < i_c1)
        return (I[1] >= j_0) | inside_cav

    def mapfn(P, C, T):
        return P.copy()

    def bcfn(I, f):
        i, j = I
        tag = np.zeros(len(i), dtype=np.int32)
        if f == 0:
            tag[i == 0] = BC_FARFIELD
        elif f == 1:
            tag[i == len(xl) - 2] = BC_FARFIELD
        elif f == 2:  # -y face
            solid_below = (j == 0) | ((j == j_0) & ((i < i_c0) | (i >= i_c1)))
            tag[solid_below] = BC_WALL
        elif f == 3:
            tag[j == len(yl) - 2] = BC_FARFIELD
        return tag

    m = _structured([xl, yl], q, mapfn, [False, False], keep=keep, bcfn=bcfn,
                    info={"kind": "cavity", "aspect": D, "h": h, "probe": np.array([0.5, 1.79]),
                          "ref_length": W})
    # side walls of the cavity: faces whose neighbour cell is removed
    gi = m.info["grid_index"]
    i, j = gi[:, 0], gi[:, 1]
    below = j < j_0
    m.face_bc[below & (i == i_c0), 0] = BC_WALL
    m.face_bc[below & (i == i_c1 - 1), 1] = BC_WALL
    return m


def naca4(m: float, pc: float, t: float, n: int = 400):
    """Textbook NACA 4-digit section (closed trailing edge) as callables.

    Returns ``surf(s)`` mapping s in [0, 2] to a point: s in [0, 1] runs over the lower
    surface from the trailing edge to the leading edge, s in [1, 2] over the upper surface
    back to the trailing edge, with cosine spacing in x.
    """
    def thick(x):
        return 5 * t * (0.2969 * np.sqrt(np.maximum(x, 0)) - 0.1260 * x - 0.3516 * x ** 2
                        + 0.2843 * x ** 3 - 0.1036 * x ** 4)

    def camber(x):
        if m == 0.0:
            return np.zeros_like(x), np.zeros_like(x)
        yc = np.where(x < pc, m / pc ** 2 * (2 * pc * x - x ** 2),
                      m / (1 - pc) ** 2 * ((1 - 2 * pc) + 2 * pc * x - x ** 2))
        dy = np.where(x < pc, 2 * m / pc ** 2 * (pc - x), 2 * m / (1 - pc) ** 2 * (pc - x))
        return yc, dy

    def surf(s):
        s = np.asarray(s, float)
        lower = s <= 1.0
        sl = np.where(lower, s, 2.0 - s)
        x = 0.5 * (1 + np.cos(np.pi * sl))  # s=0 -> x=1 (TE), s=1 -> x=0 (LE)
        yt = thick(x)
        yc, dy = camber(x)
        th = np.arctan(dy)
        sg = np.where(lower, -1.0, 1.0)
        xs = x - sg * yt * np.sin(th)
        ys = yc + sg * yt * np.cos(th)
        return np.stack([xs, ys], axis=-1)
    return surf


def c_grid_naca(n_wake: int = 40, n_foil: int = 120, n_normal: int = 80, n_span: int = 12, q: int = 2,
                camber: float = 0.0, camber_pos: float = 0.4, thickness: float = 0.12, span: float = 0.2,
                r_out: float = 10.0, x_out: float = 20.0, h_wall: float = 2e-3, seed: int | None = None) -> MeshDesc:
    """Extruded C-grid around a NACA 4-digit section (3-D hexes, spanwise periodic).

    Around-direction (reference 0): lower wake (``n_wake`` cells, from the outflow to
    the trailing edge), the section (``n_foil``: lower TE -> LE -> upper TE), upper wake.
    Normal direction (reference 1): ``n_normal`` cells from the wall / wake cut to a C-shaped
    outer boundary (half circle of radius ``r_out`` about mid-chord, straight to
    ``x = x_out``), geometrically stretched from ``h_wall``.  Spanwise (reference 2):
    ``n_span`` cells over ``span`` chords, periodic.  With ``seed``, the maximum camber is drawn
    from U[0, 0.04] (overriding ``camber``).
    """
    if seed is not None:
        rng = np.random.default_rng(seed)
        camber = float(rng.uniform(0.0, 0.04))
    surf = naca4(camber, camber_pos, thickness)
    na = 2 * n_wake + n_foil
    xc = 0.5
    # wake parameter: cells clustered near the trailing edge
    wr = 1.06

    def wake_x(u):  # u in [0,1]: 0 at TE, 1 at outflow
        return 1.0 + (x_out - 1.0) * (wr ** (u * n_wake) - 1.0) / (wr ** n_wake - 1.0)

    def inner(s):
        s = np.asarray(s, float)
        out = np.empty(s.shape + (2,))
        lw = s < n_wake
        up = s > n_wake + n_foil
        fo = ~(lw | up)
        u = (n_wake - s[lw]) / n_wake
        out[lw] = np.stack([wake_x(u), np.zeros_like(u)], axis=-1)
        u = (s[up] - n_wake - n_foil) / n_wake
        out[up] = np.stack([wake_x(u), np.zeros_like(u)], axis=-1)
        out[fo] = surf(2.0 * (s[fo] - n_wake) / n_foil)
        return out

    def outer(s):
        s = np.asarray(s, float)
        out = np.empty(s.shape + (2,))
        lw = s < n_wake
        up = s > n_wake + n_foil
        fo = ~(lw | up)
        u = (n_wake - s[lw]) / n_wake
        out[lw] = np.stack([xc + (wake_x(u) - 1.0) / (x_out - 1.0) * (x_out - xc), -r_out * np.ones_like(u)], -1)
        u = (s[up] - n_wake - n_foil) / n_wake
        out[up] = np.stack([xc + (wake_x(u) - 1.0) / (x_out - 1.0) * (x_out - xc), r_out * np.ones_like(u)], -1)
        a = (s[fo] - n_wake) / n_foil  # 0 -> bottom, 1 -> top, through the front
        ang = -0.5 * np.pi - np.pi * a
        out[fo] = np.stack([xc + r_out * np.cos(ang), r_out * np.sin(ang)], -1)
        return out

    # normal distribution: geometric from h_wall to reach 1 at n_normal
    def gfun(tn):
        # tn in [0, n_normal]; returns fraction in [0,1]
        L = r_out
        r = 1.0
        # solve h_wall*(r^n-1)/(r-1) = L for r
        lo_r, hi_r = 1.0 + 1e-9, 2.0
        for _ in range(200):
            mid = 0.5 * (lo_r + hi_r)
            if h_wall * (mid ** n_normal - 1) / (mid - 1) > L:
                hi_r = mid
            else:
                lo_r = mid
        r = 0.5 * (lo_r + hi_r)
        return (r ** tn - 1.0) / (r ** n_normal - 1.0)

    Lz = span * 1.0
    lines = [np.arange(na + 1, dtype=float), np.arange(n_normal + 1, dtype=float),
             np.linspace(0.0, Lz, n_span + 1)]

    def mapfn(P, C, T):
        s, tn, z = P[..., 0], P[..., 1], P[..., 2]
        pi_, po = inner(s), outer(s)
        g = gfun(tn)[..., None]
        xy = pi_ + g * (po - pi_)
        return np.concatenate([xy, z[..., None]], axis=-1)

    def bcfn(I, f):
        i, j, k = I
        tag = np.zeros(len(i), dtype=np.int32)
        if f == 0:
            tag[i == 0] = BC_FARFIELD
        elif f == 1:
            tag[i == na - 1] = BC_FARFIELD
        elif f == 2:
            foil = (i >= n_wake) & (i < n_wake + n_foil)
            tag[(j == 0) & foil] = BC_WALL
        elif f == 3:
            tag[j == n_normal - 1] = BC_FARFIELD
        return tag

    te = surf(np.array([0.0]))[0]
    return _structured(lines, q, mapfn, [False, False, False], bcfn=bcfn,
                       periodic_vec=[np.array([0.0, 0.0, Lz])],
                       info={"kind": "c_grid_naca", "camber": camber, "camber_pos": camber_pos,
                             "thickness": thickness, "span": Lz, "probe": np.array([te[0], te[1] - 2.0, 0.5 * Lz]),
                             "ref_length": 1.0, "ref_area": Lz})


def concat_meshes(meshes) -> MeshDesc:
    """Concatenate independent meshes of equal dim and q into one description with
    disjoint element ranges (the batched form advances them together).  Faces are only ever
    paired within one mesh, so the meshes may overlap in space; periodic meshes must share
    their translation vectors (e.g. the same span)."""
    d, q = meshes[0].dim, meshes[0].q
    pv = np.asarray(meshes[0].periodic_vec, float).reshape(-1, d)
    xs, ens, fbs, begins = [], [], [], [0]
    off = 0
    for m in meshes:
        if m.dim != d or m.q != q:
            raise ValueError("meshes must share dim and geometry degree")
        mv = np.asarray(m.periodic_vec, float).reshape(-1, d)
        if mv.shape != pv.shape or not np.allclose(mv, pv, rtol=0, atol=1e-12):
            raise ValueError("concatenated meshes must share their periodic translations")
        xs.append(m.node_xyz)
        ens.append(m.elem_nodes + off)
        fbs.append(m.face_bc)
        off += m.node_xyz.shape[0]
        begins.append(begins[-1] + m.n_elem)
    return MeshDesc(dim=d, q=q, node_xyz=np.concatenate(xs), elem_nodes=np.concatenate(ens),
                    face_bc=np.concatenate(fbs), periodic_vec=pv.copy(),
                    mesh_elem_begin=np.array(begins, dtype=np.int64),
                    info={"kind": "batch", "parts": [m.info for m in meshes]})


def sponge_degrees(mesh: MeshDesc, radii=(0.5, 1.0, 2.0, 3.0), p_max: int = 4) -> np.ndarray:
    """Solution degree per element falling with distance from the chord segment (0, 0)-(1, 0) in
    the x-y plane: p_max inside radii[0], one less per band, 0 beyond the last radius (the
    airfoil case's sponge: high degree at the airfoil, degree 0 towards the outer boundaries).
    The distance is the element centroid's (mean of its nodes) in-plane distance, so on an
    extruded mesh the degree is constant along the span."""
    c = mesh.node_xyz[mesh.elem_nodes].mean(axis=1)
    x, y = c[:, 0], c[:, 1]
    dist = np.hypot(x - np.clip(x, 0.0, 1.0), y)
    band = np.searchsorted(np.asarray(radii, float), dist, side="right")
    return np.clip(p_max - band, 0, p_max).astype(np.int64)
