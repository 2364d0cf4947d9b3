"""Parity at the full workload sizes, in the launch configuration bench.py times.

The residual of an element depends only on the elements within two faces of it (its own state,
its neighbours' flux-point states and their viscous normal fluxes, which depend on their
neighbours' flux-point states).  So the FP64 oracle, run on the index-space box of radius 2
around a sampled element (faces leaving the box tagged far field), reproduces that element's
residual exactly, and is compared with the full-size GPU residual element by element.
"""
import os
import sys

import numpy as np
import pytest
import torch

import fr_inputs as fi
from cases import rel_l2

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _patch(mesh, centre, nbr_boxes):
    """Sub-mesh of the elements whose grid index lies in one of the boxes (lists of per-direction
    index sets); AUTO faces whose partner is outside become far field."""
    gi = mesh.info["grid_index"]
    keep = np.zeros(mesh.n_elem, dtype=bool)
    for box in nbr_boxes:
        m = np.ones(mesh.n_elem, dtype=bool)
        for k, idx in enumerate(box):
            m &= np.isin(gi[:, k], idx)
        keep |= m
    sel = np.nonzero(keep)[0]
    used = np.unique(mesh.elem_nodes[sel])
    remap = -np.ones(mesh.node_xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(len(used))
    sub = fi.MeshDesc(dim=mesh.dim, q=mesh.q, node_xyz=mesh.node_xyz[used], elem_nodes=remap[mesh.elem_nodes[sel]],
                      face_bc=mesh.face_bc[sel].copy(), periodic_vec=mesh.periodic_vec.copy(),
                      mesh_elem_begin=np.array([0, len(sel)], dtype=np.int64))
    return sel, sub


def _close_patch(sub, oracle_cls, p, fp):
    """Tag AUTO faces of the patch without a partner inside it (they lie >= 3 faces from the
    centre) as far field, then build the oracle on the patch."""
    from scipy.spatial import cKDTree
    d = sub.dim
    cents = _face_centres(sub.node_xyz, sub.elem_nodes, d, sub.q)
    auto = np.argwhere(sub.face_bc == fi.FACE_AUTO)
    pts = cents[auto[:, 0], auto[:, 1]]
    tree = cKDTree(pts)
    scale = float(np.ptp(sub.node_xyz, axis=0).max())
    shifts = [np.zeros(d)] + [sg * v for v in sub.periodic_vec for sg in (1.0, -1.0)]
    for a, (e, f) in enumerate(auto):
        found = False
        for sh in shifts:
            if any(b != a for b in tree.query_ball_point(pts[a] + sh, 1e-9 * scale)):
                found = True
                break
        if not found:
            sub.face_bc[e, f] = fi.BC_FARFIELD
    return oracle_cls(sub, p, fp, equations="ns")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Bound on one element's residual, relative L2.  The small parity meshes use 1e-11; the
# full-size meshes have cells 1e-2 to 1e-3 of their coordinate range (wall cells of the C-grid
# and the O-grid), and the metric terms, differences of node coordinates over a cell, lose
# about one more decimal digit there (measured up to 7.7e-12 on the C-grid and 3.9e-11 on the
# O-grid, against <= 6.2e-13 on the small meshes).
FULL_SIZE_TOL = 1e-10


def test_naca_cgrid_full_size_sampled_residual(gpu):
    import bench
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    mesh, fp, _ = bench.naca_workload(scale=1.0)
    sol = Solver(mesh, 4, fp, equations="ns", precision="fp64")
    u = bench.initial_state(sol, fp, mesh, 5)
    R = sol.rhs(u.to(gpu)).cpu()
    gi = mesh.info["grid_index"]
    na, nn, nz = gi[:, 0].max() + 1, gi[:, 1].max() + 1, gi[:, 2].max() + 1
    rng = np.random.default_rng(0)
    # wall next to the trailing edge, wake cut, leading edge, outflow, outer boundary, random interior
    picks = [(40, 0, 0), (20, 0, 5), (100, 0, 11), (0, 10, 3), (150, 79, 6),
             tuple(int(x) for x in rng.integers([0, 0, 0], [na, nn, nz]))]
    xs = sol.solpt_coords()
    for (i, j, k) in picks:
        e = int(np.nonzero((gi[:, 0] == i) & (gi[:, 1] == j) & (gi[:, 2] == k))[0][0])
        ib = [x for x in range(i - 2, i + 3) if 0 <= x < na]
        jb = [x for x in range(j - 2, j + 3) if 0 <= x < nn]
        kb = [x % nz for x in range(k - 2, k + 3)]
        boxes = [[ib, jb, kb]]
        if j <= 2:  # across the wake cut
            boxes.append([[na - 1 - x for x in ib if 0 <= na - 1 - x < na], [0, 1, 2], kb])
        sel, sub = _patch(mesh, e, boxes)
        s = _close_patch(sub, OracleSystem, 4, fp)
        le = int(np.nonzero(sel == e)[0][0])
        up = u[sel]
        Rp = s.residual(up)
        np.testing.assert_allclose(s.solpt_coords()[le], xs[e], atol=1e-12)
        err = _rel(R[e].numpy(), Rp[le].numpy())
        print(f"element {e} grid {(i, j, k)}: patch of {len(sel)}; residual rel L2 {err:.3e}")
        assert err <= FULL_SIZE_TOL, err


def test_cylinder_ogrid_full_size_sampled_residual_and_fp32(gpu):
    import bench
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    mesh, fp = bench.cylinder_workload()
    sol = Solver(mesh, 4, fp, equations="ns", precision="fp64")
    u = bench.initial_state(sol, fp, mesh, 7)
    R = sol.rhs(u.to(gpu)).cpu()
    gi = mesh.info["grid_index"]
    nr, nt = gi[:, 0].max() + 1, gi[:, 1].max() + 1
    for (ir, it) in [(0, 0), (0, 77), (64, 40), (127, 120), (3, 159)]:
        e = int(np.nonzero((gi[:, 0] == ir) & (gi[:, 1] == it))[0][0])
        rb = [x for x in range(ir - 2, ir + 3) if 0 <= x < nr]
        tb = [x % nt for x in range(it - 2, it + 3)]
        sel, sub = _patch(mesh, e, [[rb, tb]])
        s = _close_patch(sub, OracleSystem, 4, fp)
        le = int(np.nonzero(sel == e)[0][0])
        Rp = s.residual(u[sel])[le].numpy()
        err = _rel(R[e].numpy(), Rp)
        print(f"cylinder element {(ir, it)}: residual rel L2 {err:.3e}")
        assert err <= FULL_SIZE_TOL, err
    # FP32 at full size: one RK4 step against the oracle's FP64 step, per variable.
    s_full = OracleSystem(mesh, 4, fp, equations="ns")
    s32 = Solver(mesh, 4, fp, equations="ns", precision="fp32")
    dt = 2e-5
    dtg = torch.tensor([dt], dtype=torch.float64, device=gpu)
    # (a) a state with a developed flow's magnitudes (10 % disturbances on every velocity component)
    ud = torch.tensor(fi.developed_state(s_full.solpt_coords(), fp, 7)).permute(0, 2, 1).contiguous()
    uref = s_full.rk4_step(ud, torch.tensor([dt], dtype=torch.float64))
    u32 = ud.float().to(gpu)
    s32.rk_step(u32, dtg, 1)
    e_dev = rel_l2(u32, uref)
    # (b) the bench's start, a uniform stream with 1e-3 momentum noise: the cross-stream momentum
    # is noise only, so its error is the absolute FP32 round-off of the pressure term
    # (~ eps_32 p_inf dt / h) over a norm 1e-3 of the momentum's; reported per component and
    # against the momentum vector's norm
    uref_b = s_full.rk4_step(u, torch.tensor([dt], dtype=torch.float64))
    u32b = u.float().to(gpu)
    s32.rk_step(u32b, dtg, 1)
    e2 = ((u32b.double().cpu() - uref_b) ** 2).sum(dim=(0, 2))
    n2 = (uref_b ** 2).sum(dim=(0, 2))
    per_comp = (e2 / n2).sqrt().numpy()
    d = sol.dim
    mom_vec = float((e2[1:1 + d].sum() / n2[1:1 + d].sum()).sqrt())
    print(f"cylinder full size FP32 one step vs oracle: developed state per-variable rel L2 {e_dev:.3e}; "
          f"uniform-stream start per component {np.array2string(per_comp, precision=2)}, "
          f"momentum vector {mom_vec:.3e}")
    assert e_dev <= 1e-5, e_dev
    assert max(per_comp[0], per_comp[-1], mom_vec) <= 1e-5, per_comp


def test_vortex_full_size_20_steps(gpu):
    """The 32 x 32 p = 3 isentropic-vortex case in full: 20 RK4 steps at dt = 2.12e-3 against the
    oracle (<= 1e-12) and the translated closed form (same error as the oracle's)."""
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    m = fi.periodic_box(2, 32, q=1)
    fp = fi.vortex_params()
    s = OracleSystem(m, 3, fp, equations="euler")
    x = s.solpt_coords()
    u0 = torch.tensor(fi.vortex_state(x)).permute(0, 2, 1).contiguous()
    dt = 2.12e-3
    uref, _, _ = s.run(u0, torch.tensor([dt], dtype=torch.float64), 20, sample_every=0)
    sol = Solver(m, 3, fp, equations="euler")
    u = u0.to(gpu).clone()
    sol.rk_step(u, torch.tensor([dt], dtype=torch.float64, device=gpu), 20)
    ue = torch.tensor(fi.vortex_state(x, t=20 * dt)).permute(0, 2, 1)
    num = ((u.cpu() - uref) ** 2).sum(dim=(0, 2)).sqrt()
    den = (uref ** 2).sum(dim=(0, 2)).sqrt()
    assert float((num / den).max()) <= 1e-12
    eg = float((u.cpu() - ue).abs().max())
    eo = float((uref - ue).abs().max())
    print(f"vortex: |GPU - exact| {eg:.3e}, |oracle - exact| {eo:.3e}")
    assert abs(eg - eo) <= 1e-12 and eg < 1e-4


def test_naca_sponge_full_size_sampled_residual(gpu):
    """The variable-degree solver on the full C-grid with the bench's sponge degrees (4 near the
    section to 0 beyond 8 chords): sampled elements next to degree jumps, at the wall and at the
    outer boundary against the variable-degree oracle on the index-space patch around them (the
    degrees of the patch's elements kept)."""
    import bench
    from oracle.vardeg import VarDegreeOracle
    from paper_2312_14167_amd.vardeg import VarDegreeSolver
    mesh, fp, _ = bench.naca_workload(scale=1.0)
    deg = fi.sponge_degrees(mesh, radii=bench.SPONGE_RADII)
    sol = VarDegreeSolver(mesh, deg, fp, precision="fp64")
    parts = []
    for g, x in enumerate(sol.solpt_coords()):
        ug = fi.freestream_state(x, fp)
        ug[..., 1:-1] += fi.noise_like(ug.shape, 5 + g, 1e-3)[..., 1:-1]
        parts.append(torch.tensor(ug).permute(0, 2, 1).contiguous())
    R = [r.cpu() for r in sol.split(sol.rhs(sol.join(parts)))]
    where = {}  # element -> (group, local index)
    for g, el in enumerate(sol.elems):
        for l, e in enumerate(el):
            where[int(e)] = (g, l)
    gi = mesh.info["grid_index"]
    na, nn, nz = gi[:, 0].max() + 1, gi[:, 1].max() + 1, gi[:, 2].max() + 1
    index = {tuple(int(v) for v in gi[e]): e for e in range(mesh.n_elem)}

    def jump(e, lo, hi):
        i, j, k = (int(v) for v in gi[e])
        if deg[e] != hi:
            return False
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            n = index.get((i + di, j + dj, k))
            if n is not None and deg[n] == lo:
                return True
        return False
    picks = []
    for lo, hi in ((3, 4), (2, 3), (1, 2), (0, 1)):
        picks.append(next(e for e in range(0, mesh.n_elem, 7) if jump(e, lo, hi)))
    picks.append(index[(100, 0, 4)])                                  # wall at the leading edge
    picks.append(next(e for e in range(mesh.n_elem) if gi[e, 1] == nn - 1 and gi[e, 2] == 7))  # outer boundary
    for e in picks:
        i, j, k = (int(v) for v in gi[e])
        ib = [x for x in range(i - 2, i + 3) if 0 <= x < na]
        jb = [x for x in range(j - 2, j + 3) if 0 <= x < nn]
        kb = [x % nz for x in range(k - 2, k + 3)]
        boxes = [[ib, jb, kb]]
        if j <= 2:  # across the wake cut
            boxes.append([[na - 1 - x for x in ib if 0 <= na - 1 - x < na], [0, 1, 2], kb])
        sel, sub = _patch(mesh, e, boxes)
        v = _close_patch(sub, lambda m_, p_, f_, equations: VarDegreeOracle(m_, deg[sel], f_, equations=equations),
                         None, fp)
        # the patch's state, group by group in the oracle's order
        up = []
        for G in v.groups:
            rows = [parts[where[int(sel[le])][0]][where[int(sel[le])][1]] for le in G.elems]
            up.append(torch.stack(rows))
        Rp = v.residual(up)
        le = int(np.nonzero(sel == e)[0][0])
        gp, lp = int(v.gidx[le]), int(v.lidx[le])
        g, l = where[e]
        err = _rel(R[g][l].numpy(), Rp[gp][lp].numpy())
        print(f"sponge element {e} grid {(i, j, k)} degree {deg[e]}: patch of {len(sel)} "
              f"(degrees {sorted(set(deg[sel].tolist()))}); residual rel L2 {err:.3e}")
        assert err <= FULL_SIZE_TOL, err


def _face_centres(node_xyz, elem_nodes, d, q):
    """[n_elem][2 d][d] face centres (mean of each face's corner nodes)."""
    import itertools
    cents = np.zeros((elem_nodes.shape[0], 2 * d, d))
    for f in range(2 * d):
        k, side = f // 2, f % 2
        corners = []
        for bits in itertools.product([0, q], repeat=d - 1):
            idx, b = [0] * d, 0
            for m in range(d):
                if m == k:
                    idx[m] = q * side
                else:
                    idx[m] = bits[b]
                    b += 1
            corners.append(sum(idx[m] * (q + 1) ** m for m in range(d)))
        cents[:, f] = node_xyz[elem_nodes[:, corners]].mean(axis=1)
    return cents


def _neighbours(mesh, b0, b1):
    """Face neighbours (global element indices) of the elements of one mesh of a batch
    (elements b0..b1-1; faces pair only inside their own mesh)."""
    from scipy.spatial import cKDTree
    cents = _face_centres(mesh.node_xyz, mesh.elem_nodes[b0:b1], mesh.dim, mesh.q)
    auto = np.argwhere(mesh.face_bc[b0:b1] == fi.FACE_AUTO)
    pts = cents[auto[:, 0], auto[:, 1]]
    scale = float(np.ptp(mesh.node_xyz[np.unique(mesh.elem_nodes[b0:b1])], axis=0).max())
    tree = cKDTree(pts)
    nbr = [[] for _ in range(b1 - b0)]
    for a, b in tree.query_pairs(1e-9 * scale):
        ea, eb = auto[a, 0], auto[b, 0]
        nbr[ea].append(b0 + eb)
        nbr[eb].append(b0 + ea)
    return nbr


def _rings(nbr, b0, e, n):
    """Elements within n face steps of element e, in increasing index: the patch keeps the
    elements' relative order, so every pair keeps its L side (the smaller element, face), which
    decides the one-sided LDG flux."""
    seen, front = {e}, [e]
    for _ in range(n):
        nxt = []
        for x in front:
            for y in nbr[x - b0]:
                if y not in seen:
                    seen.add(y)
                    nxt.append(y)
        front = nxt
    return np.array(sorted(seen), dtype=np.int64)


def _submesh(mesh, sel):
    used = np.unique(mesh.elem_nodes[sel])
    remap = -np.ones(mesh.node_xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(len(used))
    return fi.MeshDesc(dim=mesh.dim, q=mesh.q, node_xyz=mesh.node_xyz[used], elem_nodes=remap[mesh.elem_nodes[sel]],
                       face_bc=mesh.face_bc[sel].copy(), periodic_vec=mesh.periodic_vec.copy(),
                       mesh_elem_begin=np.array([0, len(sel)], dtype=np.int64))


def test_batched_cavities_full_size_sampled(gpu):
    """The bench's batched poll at full size (16 cavities, 367k quads, p = 4, one solver): sampled
    elements (next to a wall, next to the far field, interior) of three cavities.  FP64: the
    residual against the oracle on the two-step neighbourhood (exact, as above).  FP32, at the
    autotuned tiles the bench times: one RK4 step against the oracle's FP64 step on the ten-step
    neighbourhood (a stage's residual reaches two face steps, so the four stages of a step leave
    the centre untouched by the patch's outer boundary), per element: density and energy per
    variable, momentum as a vector (its cross-stream part is 1e-3 noise)."""
    import dataclasses

    import bench
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    bm, bfp, bprobes, counts = bench.cavity_batch()
    s64 = Solver(bm, 4, bfp, equations="ns", precision="fp64")
    u = bench.initial_state(s64, bfp, bm, 5)
    R = s64.rhs(u.to(gpu)).cpu()
    xs = s64.solpt_coords()
    dt = 1e-5
    dtg = torch.full((bm.n_mesh,), dt, dtype=torch.float64, device=gpu)
    s32 = Solver(bm, 4, bfp, equations="ns", precision="fp32", probes=bprobes, probe_mesh=np.arange(bm.n_mesh),
                 max_samples=8, forces=True)
    u32 = u.float().to(gpu)
    tiles = s32.autotune(u32, dtg, reps=2, kinds=bench.FORWARD_KINDS)
    s32.rk_step(u32, dtg, 1, sample_every=1)
    u1 = u32.double().cpu()
    d = bm.dim
    rng = np.random.default_rng(1)
    for m in (0, 7, 15):
        b0, b1 = int(bm.mesh_elem_begin[m]), int(bm.mesh_elem_begin[m + 1])
        nbr = _neighbours(bm, b0, b1)
        fb = bm.face_bc[b0:b1]
        walls = np.nonzero((fb == fi.BC_WALL).any(axis=1))[0]
        far = np.nonzero((fb == fi.BC_FARFIELD).any(axis=1))[0]
        picks = [b0 + int(walls[len(walls) // 2]), b0 + int(far[len(far) // 3]), b0 + int(rng.integers(0, b1 - b0))]
        fp_m = dataclasses.replace(bfp, rho_inf=bfp.rho_inf[m:m + 1], vel_inf=bfp.vel_inf[m:m + 1],
                                   p_inf=bfp.p_inf[m:m + 1], mu=bfp.mu[m:m + 1])
        for e in picks:
            sel = _rings(nbr, b0, e, 2)
            le = int(np.nonzero(sel == e)[0][0])
            s = _close_patch(_submesh(bm, sel), OracleSystem, 4, fp_m)
            np.testing.assert_allclose(s.solpt_coords()[le], xs[e], atol=1e-12)
            err = _rel(R[e].numpy(), s.residual(u[sel])[le].numpy())
            sel10 = _rings(nbr, b0, e, 10)
            le10 = int(np.nonzero(sel10 == e)[0][0])
            s10 = _close_patch(_submesh(bm, sel10), OracleSystem, 4, fp_m)
            ref = s10.rk4_step(u[sel10], torch.tensor([dt], dtype=torch.float64))[le10]
            diff = (u1[e] - ref) ** 2
            e_rho = float(diff[0].sum().sqrt() / (ref[0] ** 2).sum().sqrt())
            e_en = float(diff[-1].sum().sqrt() / (ref[-1] ** 2).sum().sqrt())
            e_mom = float(diff[1:1 + d].sum().sqrt() / (ref[1:1 + d] ** 2).sum().sqrt())
            print(f"cavity {m} element {e} (patches {len(sel)} / {len(sel10)}): FP64 residual rel L2 {err:.3e}; "
                  f"FP32 step rho {e_rho:.2e} energy {e_en:.2e} momentum {e_mom:.2e}")
            assert err <= FULL_SIZE_TOL, err
            assert max(e_rho, e_en, e_mom) <= 5e-7, (e_rho, e_en, e_mom)  # 10x the measured 5.5e-8
    print("FP32 tiles", {k: (v["elements_per_workgroup"], v["waves_per_simd_bound"]) for k, v in tiles.items()})


def _cgrid_step_check(gpu, precision, bar):
    """One RK4 step of the C-grid at full size (autotuned tiles, probe and force sampling) from
    the bench's start against the oracle's FP64 step on the index box of radius 10 around sampled
    elements; returns the per-element errors (density, energy, momentum as a vector)."""
    import bench
    from oracle import OracleSystem
    from paper_2312_14167_amd import Solver
    mesh, fp, _ = bench.naca_workload(scale=1.0)
    sol = Solver(mesh, 4, fp, equations="ns", precision=precision, probes=mesh.info["probe"][None, :],
                 max_samples=8, forces=True)
    u = bench.initial_state(sol, fp, mesh, 5)
    dt = 5e-7
    dtg = torch.full((1,), dt, dtype=torch.float64, device=gpu)
    ug = u.to(device=gpu, dtype=sol.dtype)
    tiles = sol.autotune(ug, dtg, reps=2, kinds=bench.FORWARD_KINDS)
    sol.rk_step(ug, dtg, 1, sample_every=1)
    u1 = ug.double().cpu()
    gi = mesh.info["grid_index"]
    na, nn, nz = gi[:, 0].max() + 1, gi[:, 1].max() + 1, gi[:, 2].max() + 1
    rng = np.random.default_rng(3)
    # wall of the section, outer boundary, interior (boxes clear of the wake cut)
    picks = [(100, 0, 11), (150, 79, 6), (int(rng.integers(60, 140)), int(rng.integers(11, 69)), int(rng.integers(0, nz)))]
    d = mesh.dim
    for (i, j, k) in picks:
        e = int(np.nonzero((gi[:, 0] == i) & (gi[:, 1] == j) & (gi[:, 2] == k))[0][0])
        ib = [x for x in range(i - 10, i + 11) if 0 <= x < na]
        jb = [x for x in range(j - 10, j + 11) if 0 <= x < nn]
        sel, sub = _patch(mesh, e, [[ib, jb, list(range(nz))]])
        s = _close_patch(sub, OracleSystem, 4, fp)
        le = int(np.nonzero(sel == e)[0][0])
        ref = s.rk4_step(u[sel], torch.tensor([dt], dtype=torch.float64))[le]
        diff = (u1[e] - ref) ** 2
        e_rho = float(diff[0].sum().sqrt() / (ref[0] ** 2).sum().sqrt())
        e_en = float(diff[-1].sum().sqrt() / (ref[-1] ** 2).sum().sqrt())
        e_mom = float(diff[1:1 + d].sum().sqrt() / (ref[1:1 + d] ** 2).sum().sqrt())
        print(f"C-grid {precision} element {(i, j, k)} (box of {len(sel)}): step rho {e_rho:.2e} energy {e_en:.2e} "
              f"momentum {e_mom:.2e}")
        assert max(e_rho, e_en, e_mom) <= bar, (e_rho, e_en, e_mom)
    print(f"{precision} tiles", {k: (v["elements_per_workgroup"], v["waves_per_simd_bound"], v["engine"])
                                 for k, v in tiles.items()})


def test_naca_cgrid_full_size_fp64_step(gpu):
    """The headline FP64 step at full size in the launch configuration the bench times, on sampled
    neighbourhoods (see _cgrid_step_check)."""
    _cgrid_step_check(gpu, "fp64", 1e-12)


def test_naca_cgrid_full_size_fp32_step(gpu):
    """The FP32 form at the headline size in the launch configuration the bench times (192k
    hexes, autotuned tiles, FP64 probe and force sampling): one RK4 step from the bench's start
    against the oracle's FP64 step on the index-space box of radius 10 around sampled elements (a
    stage's residual reaches two face steps, so four stages leave the centre untouched by the
    box's outer boundary; the whole span, periodic).  Per element: density and energy per
    variable, momentum as a vector (its cross-stream part is 1e-3 noise)."""
    _cgrid_step_check(gpu, "fp32", 5e-7)  # about 10x the measured 3.6e-8


def test_naca_sponge_full_size_fp32_step(gpu):
    """The sponge's FP32 step at full size as the bench runs it (192k hexes, degrees 4 -> 0, FP64
    probe and force sampling): one RK4 step from the bench's start against the variable-degree
    oracle's FP64 step on the index box of radius 10 (whole span) around elements next to a 3/4
    and a 0/1 degree jump (boxes clear of the wake cut).  Per element: density and energy per
    variable, momentum as a vector."""
    import bench
    from oracle.vardeg import VarDegreeOracle
    from paper_2312_14167_amd.vardeg import VarDegreeSolver
    mesh, fp, _ = bench.naca_workload(scale=1.0)
    deg = fi.sponge_degrees(mesh, radii=bench.SPONGE_RADII)
    sol = VarDegreeSolver(mesh, deg, fp, precision="fp32", probes=mesh.info["probe"][None, :], max_samples=8,
                          forces=True)
    parts = []
    for g, x in enumerate(sol.solpt_coords()):
        ug = fi.freestream_state(x, fp)
        ug[..., 1:-1] += fi.noise_like(ug.shape, 5 + g, 1e-3)[..., 1:-1]
        parts.append(torch.tensor(ug).permute(0, 2, 1).contiguous())
    dt = 5e-7
    u32 = sol.join([p_.float() for p_ in parts])
    sol.rk_step(u32, torch.full((1,), dt, dtype=torch.float64, device=gpu), 1, sample_every=1)
    U1 = [x.double().cpu() for x in sol.split(u32)]
    where = {}
    for g, el in enumerate(sol.elems):
        for l, e in enumerate(el):
            where[int(e)] = (g, l)
    gi = mesh.info["grid_index"]
    na, nn, nz = gi[:, 0].max() + 1, gi[:, 1].max() + 1, gi[:, 2].max() + 1
    index = {tuple(int(v) for v in gi[e]): e for e in range(mesh.n_elem)}

    def jump(e, lo, hi):
        i, j, k = (int(v) for v in gi[e])
        if deg[e] != hi or not (11 <= j <= nn - 12 and 10 <= i <= na - 11):
            return False
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            n = index.get((i + di, j + dj, k))
            if n is not None and deg[n] == lo:
                return True
        return False
    d = mesh.dim
    for lo, hi in ((3, 4), (0, 1)):
        e = next(e for e in range(0, mesh.n_elem, 3) if jump(e, lo, hi))
        i, j, k = (int(v) for v in gi[e])
        ib = [x for x in range(i - 10, i + 11) if 0 <= x < na]
        jb = [x for x in range(j - 10, j + 11) if 0 <= x < nn]
        sel, sub = _patch(mesh, e, [[ib, jb, list(range(nz))]])
        v = _close_patch(sub, lambda m_, p_, f_, equations: VarDegreeOracle(m_, deg[sel], f_, equations=equations),
                         None, fp)
        up = []
        for G in v.groups:
            rows = [parts[where[int(sel[le])][0]][where[int(sel[le])][1]] for le in G.elems]
            up.append(torch.stack(rows))
        ref_all = v.rk4_step(up, torch.tensor([dt], dtype=torch.float64))
        le = int(np.nonzero(sel == e)[0][0])
        ref = ref_all[int(v.gidx[le])][int(v.lidx[le])]
        g, l = where[e]
        diff = (U1[g][l] - ref) ** 2
        e_rho = float(diff[0].sum().sqrt() / (ref[0] ** 2).sum().sqrt())
        e_en = float(diff[-1].sum().sqrt() / (ref[-1] ** 2).sum().sqrt())
        e_mom = float(diff[1:1 + d].sum().sqrt() / (ref[1:1 + d] ** 2).sum().sqrt())
        print(f"sponge FP32 element {(i, j, k)} degree {deg[e]} next to {lo} (box of {len(sel)}): step rho "
              f"{e_rho:.2e} energy {e_en:.2e} momentum {e_mom:.2e}", flush=True)
        assert max(e_rho, e_en, e_mom) <= 5e-7, (e_rho, e_en, e_mom)  # about 10x the measured 3.1e-8
