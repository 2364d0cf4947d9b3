#!/usr/bin/env python3
"""FR RK-stage throughput on one MI355X.

One step = one classical RK4 step (four FR residual stages and updates) of the whole mesh,
with the probe pressure and wall force sampled in FP64 before the step: the full hot path.
Headline workload: 3-D Navier-Stokes FR at p = 4 on an extruded C-grid around a seeded NACA
4-digit section, 200 x 80 x 12 = 192,000 hexes (24.0M solution points x 5 variables), Re 23000,
M 0.2, in FP64.  Reported beside it: the same in FP32 (FP64 accumulators), a batched poll of 16
open-cavity meshes advanced together, per-kernel roofline fractions, and the FP64 CPU oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FR RK-stage GDoF/s (p=4 hex, FP64 vs FP32 vs batched); adjoint/fwd time"
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "naca_cgrid_p4_fp64_traffic.json")
KERNEL_SOURCES = ["fr_kernels.hip", "fr_device.hpp", "fr_solver.hpp"]


def kernel_source_digest() -> str:
    """sha256 over the sources of the forward kernels (the counters of profiles/ go stale when
    these change)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_14167_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary,
    or None when there is none or the kernels changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_digest() or kernel not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel]
    return k["read_bytes"] + k["write_bytes"]
KNAMES = ["interp", "common_sol", "ns_grad", "face_flux", "div_rk", "euler_vol_rk", "probe", "wall_force"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------ workloads
def naca_workload(scale: float = 1.0, seed: int = 2, cells=None):
    """The seeded C-grid workload: 200 x 80 x 12 hexes at scale 1 (2 x 40 wake + 120 around the
    section, 80 normal, 12 spanwise); ``cells`` = (n_wake, n_foil, n_normal, n_span) overrides the
    scaled counts (the section, angle of attack and extents stay those of the seed)."""
    import fr_inputs as fi
    rng = np.random.default_rng(seed)
    aoa = float(rng.uniform(0.0, 6.0))
    nw, nf, nn, ns = (max(2, int(round(40 * scale))), max(4, int(round(120 * scale))),
                      max(2, int(round(80 * scale))), max(2, int(round(12 * scale))))
    if cells is not None:
        nw, nf, nn, ns = cells
    m = fi.c_grid_naca(n_wake=nw, n_foil=nf, n_normal=nn, n_span=ns, q=2, seed=seed)
    fp = fi.freestream_params(3, 0.2, 23000.0, aoa_deg=aoa)
    return m, fp, aoa


def cavity_batch(n: int = 16, seed: int = 3):
    """16 open cavities, depth/width ratio seeded in [1.5, 3.5], quad counts seeded in 6k-40k."""
    import fr_inputs as fi
    rng = np.random.default_rng(seed)
    ms = []
    for _ in range(n):
        a = float(rng.uniform(1.5, 3.5))
        target = int(rng.uniform(6000, 40000))
        lo, hi = 0.005, 0.2
        for _ in range(30):
            h = np.sqrt(lo * hi)
            ne = fi.cavity(a, h=h, q=1).n_elem
            if ne > target:
                lo = h
            else:
                hi = h
        ms.append(fi.cavity(a, h=np.sqrt(lo * hi), q=2))
    m = fi.concat_meshes(ms)
    fp = fi.freestream_params(2, 0.15, 1500.0, n_mesh=n)
    probes = np.array([[0.5, 1.79]] * n)
    return m, fp, probes, [x.n_elem for x in ms]


def cylinder_workload(n_theta=160, n_r=128, p=4, q=4, seed=1):
    """O-grid around a unit-diameter cylinder, radius 0.5 to 30, radial stretching 1.04, interior
    corners perturbed <= 5 % of the local spacing, Re 1000, M 0.2, probe 3 D above."""
    import fr_inputs as fi
    m = fi.o_grid(n_theta, n_r, r0=0.5, r1=30.0, stretch=1.04, q=q, perturb=0.05, seed=seed)
    fp = fi.freestream_params(2, 0.2, 1000.0)
    return m, fp


def initial_state(sol, fp, mesh, seed: int):
    import torch
    import fr_inputs as fi
    x = sol.solpt_coords()
    u = np.empty(x.shape[:-1] + (fp.dim + 2,))
    for k in range(mesh.n_mesh):
        lo, hi = mesh.mesh_elem_begin[k], mesh.mesh_elem_begin[k + 1]
        u[lo:hi] = fi.freestream_state(x[lo:hi], fp, k)
    noise = fi.noise_like(u.shape, seed, 1e-3)
    u[..., 1:-1] += noise[..., 1:-1]
    return torch.tensor(u).permute(0, 2, 1).contiguous()


# ------------------------------------------------------------------------------------ accounting
def algorithmic_bytes(info, dim, T, eq, ldg_beta=0.5):
    """Minimum HBM bytes per launch of each kernel (every input read once, every output written
    once; RK kernels averaged over the four stages of a step).  With the one-sided LDG flux
    (beta = +-1/2) only one side of each interior face pair takes the neighbour's u_f and
    supplies a viscous normal flux, and that side forms the pair's whole common flux inside the
    Navier-Stokes volume kernel (no face kernel runs); the stage kernels then write u_f only on
    the faces whose values the flux side takes and on boundary faces when a face's values fill at
    least two cache lines (one byte of face flags per element tells which)."""
    Ne, NV, Ns, Nf, npair, nbnd, nwall, nmesh = info
    NM = dim * dim + 1
    I = 4
    one_sided = abs(ldg_beta) == 0.5
    # u_f written: face blocks of at least 256 bytes skip the faces no later kernel reads
    skip = (NV * Nf // (2 * dim)) * T >= 256
    uf_vals = (npair + nbnd) * NV if (eq == "ns" and one_sided and skip) else Ne * Nf * NV
    b = {}
    b["interp"] = Ne * NV * Ns * T + uf_vals * T + Ne
    # u, metrics, neighbour codes -> vol
    vol_part = Ne * ((2 * NV * Ns + NM * Ns) * T + Nf * I)
    if eq == "ns" and one_sided:
        # neighbour u_f on the flux side; normals and |N| there and on boundary points; fvn on
        # boundary points; every flux point's common flux
        b["ns_grad"] = (vol_part + npair * NV * T + (npair + nbnd) * (dim + 1) * T + nbnd * NV * T
                        + Ne * Nf * NV * T)
        b["face_flux"] = 0.0
    else:
        needed = 2 * npair + nbnd
        b["ns_grad"] = vol_part + 2 * npair * NV * T + needed * (dim + NV) * T
        vis = 2 * NV if eq == "ns" else 0
        b["face_flux"] = (npair * ((2 * NV + vis + dim + 1) * T + 2 * I)
                          + nbnd * ((NV + (NV if eq == "ns" else 0) + dim + 1) * T + I)
                          + (2 * npair + nbnd) * NV * T)
    rk_rw = (4 * (NV * Ns + NV * Nf + Ns + NV * Ns) + 3 * NV * Ns       # reads: vol/u, fhat, invJ, u0; acc
             + 3 * 2 * NV * Ns + NV * Ns) / 4.0                          # writes: acc + stage state / u0
    b["div_rk"] = Ne * (rk_rw * T + I + 1) + uf_vals * T                 # + u_f of the new stage state
    b["euler_vol_rk"] = Ne * ((rk_rw + (NM - 1) * Ns) * T + I + 1) + uf_vals * T
    b["probe"] = 0.0
    b["wall_force"] = nwall * ((NV + dim + dim + 1) * T + 8 + I)
    return b


def staged_model(info, kern):
    """The same launches priced with a staged pipeline's bytes (3-D p = 4 NS, FP64: interp, common
    solution, gradient + flux, viscous interface, divergence + RK each storing its outputs once;
    19225 values per element per stage, 12600 of them in the work the volume kernel fuses), for
    comparison with the fused model the roofline uses."""
    ne, nv, ns = info[0], info[1], info[2]
    if not (nv == 5 and ns == 125 and "ns_grad" in kern and "div_rk" in kern):
        return None
    g_ms = kern["ns_grad"][0] / kern["ns_grad"][1]
    d_ms = kern["div_rk"][0] / kern["div_rk"][1]
    fused_part, stage = 12600 * 8 * ne, 19225 * 8 * ne
    return {"values_per_element_stage": 19225, "ns_grad_part_values": 12600,
            "ns_grad_GB_s": fused_part / (g_ms * 1e-3) / 1e9, "ns_grad_frac": fused_part / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "stage_GB_s": stage / ((g_ms + d_ms) * 1e-3) / 1e9}


def time_steps(sol, u, dt, steps, warmup, sample_every=1):
    import torch
    sol.reset_accumulators()
    for _ in range(warmup):
        sol.rk_step(u, dt, 1, sample_every=sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.rk_step(u, dt, steps, sample_every=sample_every)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_profile(sol, u, dt, steps):
    """Per-kernel average durations over `steps` RK4 steps, from HIP events recorded on the launch
    stream around every kernel."""
    import ctypes as C

    import torch
    from paper_2312_14167_amd._lib import check, lib
    L = lib()
    L.fr_profile_enable.argtypes = [C.c_void_p, C.c_int32]
    L.fr_profile_read.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    ms = np.zeros(8)
    n = np.zeros(8, dtype=np.int64)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(L.fr_profile_enable(sol._h, 1))
    check(L.fr_profile_read(sol._h, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p), st))
    sol.rk_step(u, dt, steps, sample_every=1)
    check(L.fr_profile_read(sol._h, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p), st))
    check(L.fr_profile_enable(sol._h, 0))
    return {KNAMES[k]: (ms[k], int(n[k])) for k in range(8) if n[k] > 0}


def solver_info(sol):
    import ctypes as C
    from paper_2312_14167_amd._lib import check, lib
    L = lib()
    L.fr_solver_info.argtypes = [C.c_void_p, C.c_void_p]
    info = np.zeros(8, dtype=np.int64)
    check(L.fr_solver_info(sol._h, info.ctypes.data_as(C.c_void_p)))
    return [int(x) for x in info]


def cpu_baseline(budget_s: float = 20.0):
    """The FP64 oracle, as it is, on a bounded sample of the headline workload: a reduced C-grid of
    the same kind (p = 4 hexes, NS), one RK4 step."""
    import torch
    from oracle import OracleSystem
    m, fp, _ = naca_workload(scale=0.25)
    s = OracleSystem(m, 4, fp, equations="ns")
    x = s.solpt_coords()
    import fr_inputs as fi
    u = torch.tensor(fi.freestream_state(x, fp) + fi.noise_like(x.shape[:-1] + (5,), 1, 1e-3)).permute(0, 2, 1)
    u = u.contiguous()
    s.residual(u)  # warm-up
    t0 = time.perf_counter()
    n = 0
    while True:
        s.rk4_step(u, torch.tensor([1e-6], dtype=torch.float64))
        n += 1
        if time.perf_counter() - t0 > budget_s / 2 or n >= 4:
            break
    t = (time.perf_counter() - t0) / n
    dof = m.n_elem * 125 * 5
    return {"value": dof * 4 / t / 1e9, "unit": "GDoF-stage/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"one RK4 step (4 FR residuals, FP64, dense per-element operators) of a reduced C-grid "
                      f"around the same section: {m.n_elem} p=4 hexes, NS, {n} repetition(s) averaged"}


# ------------------------------------------------------------------------------------ main
FORWARD_KINDS = ("ns_volume", "ns_lift_rk", "euler_volume_rk")


def run_variant(mesh, fp, precision, steps, warmup, probes=None, probe_mesh=None, seed=5, profile=False,
                autotune=True):
    import torch
    from paper_2312_14167_amd import Solver
    t0 = time.perf_counter()
    sol = Solver(mesh, 4, fp, equations="ns", precision=precision, probes=probes, probe_mesh=probe_mesh,
                 max_samples=max(steps + warmup, 1), forces=True)
    log(f"  built {precision} solver in {time.perf_counter() - t0:.1f}s")
    u = initial_state(sol, fp, mesh, seed).to(device="cuda", dtype=sol.dtype)
    # stable explicit dt: the trailing-edge cells of the C-grid are ~7e-4 chords long
    dt = torch.full((mesh.n_mesh,), 5e-7 if mesh.dim == 3 else 1e-5, dtype=torch.float64, device="cuda")
    tiles = sol.autotune(u, dt, reps=3, kinds=FORWARD_KINDS) if autotune else None
    if tiles:
        log("  autotuned: " + ", ".join(f"{k} E={v['elements_per_workgroup']} waves={v['waves_per_simd_bound'] or 'default'} "
                                         f"{v['engine']}{' (remembered)' if v['from_cache'] else ''}"
                                         for k, v in tiles.items()))
    t = time_steps(sol, u, dt, steps, warmup)
    info = solver_info(sol)
    dof = info[0] * info[1] * info[2]
    out = {"sec": t, "gdofs": dof * 4 * steps / t / 1e9, "ms_per_step": 1e3 * t / steps, "info": info,
           "finite": bool(torch.isfinite(u).all()), "tiles": tiles}
    if profile:
        out["kernels"] = kernel_profile(sol, u, dt, max(2, min(steps, 10)))
    st = sol.probe_oaspl(p_ref=2e-5 * fp.p_inf[0] / 101325.0)
    out["n_samples"] = st["n_samples"]
    sol.close()
    del u
    torch.cuda.empty_cache()
    return out


SPONGE_RADII = (2.0, 4.0, 6.0, 8.0)   # chords from the section: P4 inside 2, P0 beyond 8


def run_sponge(mesh, fp, precision, steps, warmup, seed=5):
    """The C-grid with the sponge's degrees (4 near the section falling to 0 towards the outer
    boundary and the far wake): one solver per degree group, mortar kernels between degrees, the
    whole RK4 step one graph; FP64 probe and wall-force sampling every step."""
    import torch
    import fr_inputs as fi
    from paper_2312_14167_amd import VarDegreeSolver
    deg = fi.sponge_degrees(mesh, radii=SPONGE_RADII)
    t0 = time.perf_counter()
    sol = VarDegreeSolver(mesh, deg, fp, precision=precision, probes=mesh.info["probe"][None, :],
                          max_samples=max(steps + warmup, 1), forces=True)
    log(f"  built {precision} variable-degree solver in {time.perf_counter() - t0:.1f}s: degrees {sol.degrees}, "
        f"elements {sol.n_elem}, {sol.n_mortar} mortar faces")
    parts = []
    for g, x in enumerate(sol.solpt_coords()):
        u = fi.freestream_state(x, fp)
        noise = fi.noise_like(u.shape, seed + g, 1e-3)
        u[..., 1:-1] += noise[..., 1:-1]
        parts.append(torch.tensor(u).permute(0, 2, 1).contiguous())
    u = sol.join(parts)
    dt = torch.full((1,), 5e-7, dtype=torch.float64, device="cuda")
    t = time_steps(sol, u, dt, steps, warmup)
    dof = sum(n * 5 * (p + 1) ** 3 for n, p in zip(sol.n_elem, sol.degrees))
    f, ns = sol.mean_force()
    out = {"gdofs": dof * 4 * steps / t / 1e9, "ms_per_step": 1e3 * t / steps, "dof": dof,
           "degrees": sol.degrees, "elements": sol.n_elem, "mortar_faces": sol.n_mortar,
           "finite": bool(torch.isfinite(u).all()) and bool(np.isfinite(f).all()), "n_samples": ns}
    sol.close()
    del u
    torch.cuda.empty_cache()
    return out


def mfma_comparison(mesh, fp, steps, warmup, seed=5):
    """FP32 headline with the NS volume kernel's divergence on the vector ALU and on the matrix
    cores (v_mfma_f32_16x16x4f32), at the same tile sizes and register budget: ms per step and
    the volume kernel's average launch time for each."""
    import torch
    from paper_2312_14167_amd import Solver
    sol = Solver(mesh, 4, fp, equations="ns", precision="fp32", probes=mesh.info["probe"][None, :],
                 max_samples=max(steps + warmup, 1) * 8, forces=True)
    u0 = initial_state(sol, fp, mesh, seed).to(device="cuda", dtype=sol.dtype)
    dt = torch.full((1,), 5e-7, dtype=torch.float64, device="cuda")
    cands = sol.tune_candidates(0)
    out = {}
    for c, (E, Wb, eng) in enumerate(cands):
        if Wb != 0 or E == cands[2][0] and c == 2:
            continue
        sol.tune_select(0, c)
        u = u0.clone()
        t = time_steps(sol, u, dt, steps, warmup)
        kern = kernel_profile(sol, u, dt, max(2, min(steps, 5)))
        name = f"{'mfma' if eng else 'valu'}_E{E}"
        out[name] = {"ms_per_step": 1e3 * t / steps, "ns_grad_avg_ms": kern["ns_grad"][0] / kern["ns_grad"][1]}
        log(f"  {name}: {out[name]['ms_per_step']:.3f} ms/step, volume kernel {out[name]['ns_grad_avg_ms']:.4f} ms")
    sol.close()
    return out


def interface_forms(mesh, fp, steps, warmup, seed=5):
    """The headline C-grid (FP64) in the two forms that run the standalone interface kernel
    `k_face_flux` (left/right flux-point states gathered per pair): the two-sided LDG flux (beta = 0,
    every flux point supplies a viscous normal flux) and the Euler equations.  Per-kernel average
    launch times and fractions of the HBM roofline on each kernel's algorithmic bytes."""
    import dataclasses

    import torch
    from paper_2312_14167_amd import Solver
    out = {}
    for name, eq, beta in (("ns_two_sided_ldg", "ns", 0.0), ("euler", "euler", fp.ldg_beta)):
        f2 = dataclasses.replace(fp, ldg_beta=beta)
        sol = Solver(mesh, 4, f2, equations=eq, precision="fp64", probes=mesh.info["probe"][None, :],
                     max_samples=max(steps + warmup, 1) * 8, forces=(eq == "ns"))
        u = initial_state(sol, f2, mesh, seed).to(device="cuda", dtype=sol.dtype)
        dt = torch.full((1,), 5e-7, dtype=torch.float64, device="cuda")
        t = time_steps(sol, u, dt, steps, warmup)
        kern = kernel_profile(sol, u, dt, max(2, min(steps, 10)))
        info = solver_info(sol)
        ab = algorithmic_bytes(info, 3, 8, eq, beta)
        r = {"ms_per_step": 1e3 * t / steps, "gdofs": info[0] * info[1] * info[2] * 4 * steps / t / 1e9, "kernels": {}}
        for k, (ms, n) in kern.items():
            e = {"avg_ms": ms / n}
            if ab.get(k, 0) > 0:
                e["algorithmic_GB"] = ab[k] / 1e9
                e["frac"] = ab[k] / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS
            r["kernels"][k] = e
        out[name] = r
        sol.close()
        del u
        torch.cuda.empty_cache()
    return out


def adjoint_ratio(K=200, C=20):
    """Forward RK4 trajectory with probe sampling vs its checkpointed adjoint (gradient of the
    time-mean square probe-pressure fluctuation w.r.t. the initial state), cylinder O-grid
    80 x 64, p = 3, FP64."""
    import torch
    from paper_2312_14167_amd import Solver
    from paper_2312_14167_amd.adjoint import FRTrajectory
    m, fp = cylinder_workload(80, 64, p=3, q=3)
    probe = np.array([[0.0, 3.0]])
    sol = Solver(m, 3, fp, equations="ns", probes=probe, max_samples=K, forces=False)
    u0 = initial_state(sol, fp, m, 9).cuda()
    dt = torch.tensor([1e-4], dtype=torch.float64, device="cuda")
    # warm-up with the timed shapes (graph capture, work and record-buffer allocation)
    X = torch.tensor(m.node_xyz, dtype=torch.float64, device="cuda", requires_grad=True)
    for nodes in (None, X):
        ug = u0.clone().requires_grad_(True)
        P = FRTrajectory.apply(ug, sol, dt, K, C, nodes)
        ((P - P.mean(0)) ** 2).mean(0).sum().backward()
    torch.cuda.synchronize()
    ug = u0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    P = FRTrajectory.apply(ug, sol, dt, K, C, None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J = ((P - P.mean(0)) ** 2).mean(0).sum()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = ug.grad
    # the same with the mesh-node gradient (each stage VJP also evaluates its residual in the
    # two-sided form and accumulates metric / normal adjoints; one node mapping per step)
    ug = u0.clone().requires_grad_(True)
    X = torch.tensor(m.node_xyz, dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    P = FRTrajectory.apply(ug, sol, dt, K, C, X)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    ((P - P.mean(0)) ** 2).mean(0).sum().backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    return {"forward_s": t1 - t0, "backward_s": t2 - t1, "adjoint_over_forward": (t2 - t1) / (t1 - t0),
            "forward_plus_adjoint_over_forward": (t2 - t0) / (t1 - t0),
            "with_node_gradient": {"forward_s": t4 - t3, "backward_s": t5 - t4,
                                   "adjoint_over_forward": (t5 - t4) / (t4 - t3),
                                   "grad_finite": bool(torch.isfinite(X.grad).all())},
            "steps": K, "checkpoint_every": C, "quads": m.n_elem, "p": 3, "objective": float(J.detach()),
            "grad_finite": bool(torch.isfinite(g).all()),
            "workload": "cylinder O-grid 80 x 64, p=3, FP64, 200 RK4 steps, checkpoint every 20"}


def cylinder_precision_drift(n_steps=5000):
    """FP32 vs FP64 state after n_steps RK4 steps on the 160 x 128 p = 4 cylinder O-grid."""
    import torch
    from paper_2312_14167_amd import Solver
    m, fp = cylinder_workload()
    probe = np.array([[0.0, 3.0]])
    out = {}
    res = {}
    for prec in ("fp64", "fp32"):
        sol = Solver(m, 4, fp, equations="ns", precision=prec, probes=probe, max_samples=n_steps, forces=True)
        u = initial_state(sol, fp, m, 7).to(device="cuda", dtype=sol.dtype)
        dt = torch.tensor([2e-5], dtype=torch.float64, device="cuda")
        sol.rk_step(u, dt, 2, sample_every=1)
        sol.reset_accumulators()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.rk_step(u, dt, n_steps, sample_every=1)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        info = solver_info(sol)
        st = sol.probe_oaspl(p_ref=2e-5 * fp.p_inf[0] / 101325.0)
        res[prec] = u.double()
        out[prec] = {"gdofs": info[0] * info[1] * info[2] * 4 * n_steps / t / 1e9, "ms_per_step": 1e3 * t / n_steps,
                     "oaspl_db": float(st["oaspl"][0]), "mean_force": st["mean_force"][0].tolist(),
                     "finite": bool(torch.isfinite(u).all())}
        sol.close()
    a, b = res["fp32"], res["fp64"]
    rel = float((((a - b) ** 2).sum(dim=(0, 2)).sqrt() / (b ** 2).sum(dim=(0, 2)).sqrt()).max())
    out["fp32_vs_fp64_rel_l2"] = rel
    out["steps"] = n_steps
    out["workload"] = "cylinder O-grid 160 x 128 (20,480 quads), p=4, Re 1000, M 0.2, dt 2e-5"
    return out


def sequential_cavities(bm, bfp, counts, steps, precision="fp32"):
    """The batched poll's 16 meshes advanced one after the other (16 solvers)."""
    import torch
    import fr_inputs as fi
    from paper_2312_14167_amd import Solver
    total = 0.0
    dof = 0
    for k in range(bm.n_mesh):
        lo, hi = bm.mesh_elem_begin[k], bm.mesh_elem_begin[k + 1]
        used = np.unique(bm.elem_nodes[lo:hi])
        remap = -np.ones(bm.node_xyz.shape[0], dtype=np.int64)
        remap[used] = np.arange(len(used))
        mk = fi.MeshDesc(dim=2, q=bm.q, node_xyz=bm.node_xyz[used], elem_nodes=remap[bm.elem_nodes[lo:hi]],
                         face_bc=bm.face_bc[lo:hi], periodic_vec=np.zeros((0, 2)),
                         mesh_elem_begin=np.array([0, hi - lo]))
        fpk = fi.FlowParams(dim=2, rho_inf=bfp.rho_inf[k:k + 1], vel_inf=bfp.vel_inf[k:k + 1],
                            p_inf=bfp.p_inf[k:k + 1], mu=bfp.mu[k:k + 1])
        sol = Solver(mk, 4, fpk, equations="ns", precision=precision, probes=np.array([[0.5, 1.79]]),
                     max_samples=steps + 4, forces=True)
        u = initial_state(sol, fpk, mk, 5).to(device="cuda", dtype=sol.dtype)
        dt = torch.full((1,), 1e-5, dtype=torch.float64, device="cuda")
        sol.autotune(u, dt, reps=2, kinds=FORWARD_KINDS)
        total += time_steps(sol, u, dt, steps, 2)
        info = solver_info(sol)
        dof += info[0] * info[1] * info[2]
        sol.close()
    return {"sec": total, "gdofs": dof * 4 * steps / total / 1e9, "ms_per_step": 1e3 * total / steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-drift", action="store_true", help="skip the 5000-step FP32/FP64 cylinder run")
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = 192,000 hexes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--only", choices=["adjoint", "drift", "batched", "fp32", "sponge", "mfma", "interface"],
                    help="run one secondary measurement alone (for profiling) and print its JSON")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "reps": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the path runs as one process on one "
              f"MI355X; sharding across GPUs is not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2312_14167_amd import Solver  # noqa: F401  (fails loudly without libfrmi.so)
    K, W = args.steps, args.warmup
    if args.only:
        if args.only == "adjoint":
            r = adjoint_ratio()
        elif args.only == "fp32":
            mesh, fp, aoa = naca_workload(scale=args.scale)
            r = run_variant(mesh, fp, "fp32", K, W, probes=mesh.info["probe"][None, :], profile=True)
            r = {"gdofs": r["gdofs"], "ms_per_step": r["ms_per_step"], "tiles": r["tiles"],
                 "kernels": {k: v[0] / v[1] for k, v in r["kernels"].items()}}
        elif args.only == "drift":
            r = cylinder_precision_drift()
        elif args.only == "mfma":
            mesh, fp, aoa = naca_workload(scale=args.scale)
            r = mfma_comparison(mesh, fp, K, W)
        elif args.only == "sponge":
            mesh, fp, aoa = naca_workload(scale=args.scale)
            r = {pr: run_sponge(mesh, fp, pr, K, W) for pr in ("fp64", "fp32")}
        elif args.only == "interface":
            mesh, fp, aoa = naca_workload(scale=args.scale)
            r = interface_forms(mesh, fp, K, W)
        else:
            bm, bfp, bprobes, counts = cavity_batch()
            r = run_variant(bm, bfp, "fp32", K, W, probes=bprobes, probe_mesh=np.arange(16))
            r = {k: v for k, v in r.items() if k in ("gdofs", "ms_per_step")}
        print(json.dumps({"only": args.only, **r}), flush=True)
        return
    log("building the 3-D C-grid workload")
    t0 = time.perf_counter()
    mesh, fp, aoa = naca_workload(scale=args.scale)
    probe = mesh.info["probe"][None, :]
    log(f"  mesh: {mesh.n_elem} hexes ({time.perf_counter() - t0:.1f}s)")
    log("FP64 headline")
    r64 = run_variant(mesh, fp, "fp64", K, W, probes=probe, profile=True)
    log(f"  {r64['gdofs']:.2f} GDoF-stage/s, {r64['ms_per_step']:.2f} ms/step")
    info = r64["info"]
    ab = algorithmic_bytes(info, 3, 8, "ns", fp.ldg_beta)
    kern = r64["kernels"]
    dom = max(kern, key=lambda k: kern[k][0])
    avg_ms = kern[dom][0] / kern[dom][1]
    per_kernel = {}
    for k, (ms, n) in kern.items():
        if ab.get(k, 0) > 0:
            gbs = ab[k] / (ms / n * 1e-3) / 1e9
            per_kernel[k] = {"avg_ms": ms / n, "launches": n, "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS,
                             "share": ms / sum(v[0] for v in kern.values())}
        else:
            per_kernel[k] = {"avg_ms": ms / n, "launches": n}
    achieved = ab[dom] / (avg_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": r64["gdofs"],
        "unit": "GDoF-stage/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"3-D Navier-Stokes FR, p=4 hexes, extruded C-grid around a seeded NACA 4-digit "
                                f"section ({mesh.info['camber']*100:.2f}% camber, 12% thick, AoA {aoa:.2f} deg), "
                                f"{mesh.n_elem} hexes = {info[0]*info[2]/1e6:.2f}M solution points x 5 variables, "
                                f"Re 23000, M 0.2; one step = RK4 (4 residual stages) with FP64 probe + "
                                f"wall-force sampling"),
                   "dof": info[0] * info[1] * info[2], "stages_per_step": 4},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                     "algorithmic_bytes_per_launch": ab[dom], "avg_launch_ms": avg_ms,
                     "staged_model": staged_model(info, kern)},
        "kernels": per_kernel,
        "tiles": r64.get("tiles"),
    }
    if not args.no_variants:
        log("FP32 (FP64 accumulators)")
        r32 = run_variant(mesh, fp, "fp32", K, W, probes=probe)
        log(f"  {r32['gdofs']:.2f} GDoF-stage/s")
        result["variants"] = {"fp32": {"value": r32["gdofs"], "ms_per_step": r32["ms_per_step"],
                                       "speedup_vs_fp64": r32["gdofs"] / r64["gdofs"], "tiles": r32.get("tiles")}}
        log(f"sponge: degrees 4 -> 0 with distance from the section (radii {SPONGE_RADII} chords)")
        sp = {}
        for pr, ref in (("fp64", r64), ("fp32", r32)):
            rs_ = run_sponge(mesh, fp, pr, K, W)
            rs_["step_time_vs_uniform_p4"] = rs_["ms_per_step"] / ref["ms_per_step"]
            sp[pr] = rs_
            log(f"  {pr}: {rs_['gdofs']:.2f} GDoF-stage/s, {rs_['ms_per_step']:.2f} ms/step "
                f"({rs_['step_time_vs_uniform_p4']:.2f} of uniform p=4)")
        result["variants"]["sponge_p4_to_p0"] = {"radii_chords": list(SPONGE_RADII), **sp}
        log("interface kernel forms: two-sided LDG and Euler on the same C-grid (FP64)")
        itf = interface_forms(mesh, fp, K, W)
        for name, r_ in itf.items():
            log(f"  {name}: {r_['gdofs']:.2f} GDoF-stage/s; face kernel "
                f"{r_['kernels']['face_flux']['frac']:.3f} of the HBM roofline")
        result["variants"]["interface_forms_fp64"] = itf
        del mesh
        log("batched poll: 16 cavities, FP32, one launch per kernel over all meshes")
        bm, bfp, bprobes, counts = cavity_batch()
        rb = run_variant(bm, bfp, "fp32", K, W, probes=bprobes, probe_mesh=np.arange(16))
        log(f"  {rb['gdofs']:.2f} GDoF-stage/s over {bm.n_elem} quads")
        log("16 sequential FP32 solves of the same meshes")
        rs = sequential_cavities(bm, bfp, counts, K)
        log(f"  {rs['gdofs']:.2f} GDoF-stage/s")
        log("16 sequential FP64 solves of the same meshes")
        rs64 = sequential_cavities(bm, bfp, counts, K, precision="fp64")
        log(f"  {rs64['gdofs']:.2f} GDoF-stage/s")
        result["variants"]["batched_16_cavities_fp32"] = {
            "value": rb["gdofs"], "ms_per_step": rb["ms_per_step"], "quads": counts, "total_quads": bm.n_elem,
            "tiles": rb.get("tiles"),
            "sequential_fp32_value": rs["gdofs"], "sequential_fp32_ms_per_step": rs["ms_per_step"],
            "speedup_vs_sequential_fp32": rs["ms_per_step"] / rb["ms_per_step"],
            "sequential_fp64_value": rs64["gdofs"], "sequential_fp64_ms_per_step": rs64["ms_per_step"],
            "speedup_vs_sequential_fp64": rs64["ms_per_step"] / rb["ms_per_step"]}
        log("adjoint / forward time (cylinder 80 x 64, p=3, 200 steps)")
        ra = adjoint_ratio()
        log(f"  forward {ra['forward_s']:.3f}s backward {ra['backward_s']:.3f}s ratio {ra['adjoint_over_forward']:.2f}; "
            f"with node gradient {ra['with_node_gradient']['adjoint_over_forward']:.2f}")
        result["variants"]["adjoint"] = ra
        if not args.no_drift:
            log("FP32 vs FP64 after 5000 steps (cylinder 160 x 128, p=4)")
            rd = cylinder_precision_drift()
            log(f"  rel L2 {rd['fp32_vs_fp64_rel_l2']:.3e}; fp64 {rd['fp64']['gdofs']:.2f}, "
                f"fp32 {rd['fp32']['gdofs']:.2f} GDoF-stage/s")
            result["variants"]["cylinder_5000_steps"] = rd
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline()
        log(f"  {result['cpu_baseline']['value']:.5f} GDoF-stage/s on {result['cpu_baseline']['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
