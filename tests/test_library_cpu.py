"""CPU-side checks of the C ABI: the library loads, exports every symbol of include/fr.h, the
ctypes structures match the C layout, and host-side validation errors are reported before any
device work (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import fr_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr.h")


def _lib():
    from paper_2312_14167_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfrmi.so not built")
    return _lib


def test_every_declared_symbol_is_exported():
    L = _lib().lib()
    text = open(HEADER).read()
    names = set(re.findall(r"\b(fr_[a-z_]+)\s*\(", text))
    names -= {"fr_status"}
    assert {"fr_build_operators", "fr_rhs", "fr_rk_step", "fr_probe_oaspl", "fr_rhs_vjp"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n


def test_ctypes_layout_matches_c_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fr.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(fr_mesh_desc), sizeof(fr_params),'
                   ' offsetof(fr_mesh_desc, mesh_elem_begin), offsetof(fr_params, n_probe),'
                   ' offsetof(fr_params, forces), offsetof(fr_mesh_desc, n_mesh)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    lb = _lib()
    want = [C.sizeof(lb.fr_mesh_desc), C.sizeof(lb.fr_params), lb.fr_mesh_desc.mesh_elem_begin.offset,
            lb.fr_params.n_probe.offset, lb.fr_params.forces.offset, lb.fr_mesh_desc.n_mesh.offset]
    assert got == want


def _build(mesh, p=2, probes=None, eq=1):
    lb = _lib()
    L = lb.lib()
    keep = []

    def a(x, dt):
        x = np.ascontiguousarray(np.asarray(x, dt))
        keep.append(x)
        return x.ctypes.data_as(C.c_void_p) if x.size else None
    pv = np.asarray(mesh.periodic_vec).reshape(-1, mesh.dim)
    md = lb.fr_mesh_desc(dim=mesh.dim, p=p, geom_q=mesh.q, n_periodic=pv.shape[0], n_elem=mesh.n_elem,
                         n_node=mesh.node_xyz.shape[0], node_xyz=a(mesh.node_xyz, np.float64),
                         elem_nodes=a(mesh.elem_nodes, np.int64), face_bc=a(mesh.face_bc, np.int32),
                         periodic_vec=a(pv, np.float64), n_mesh=1, reserved0=0, mesh_elem_begin=None)
    fp = fi.freestream_params(mesh.dim, 0.2, 100.0)
    prm = lb.fr_params(equations=eq, precision=0, gamma=1.4, prandtl=0.71, ldg_beta=0.5, ldg_tau=0.1,
                       rho_inf=a(fp.rho_inf, np.float64), vel_inf=a(fp.vel_inf, np.float64),
                       p_inf=a(fp.p_inf, np.float64), mu=a(fp.mu, np.float64),
                       n_probe=0 if probes is None else len(probes), max_samples=4,
                       probe_xyz=None if probes is None else a(probes, np.float64), probe_mesh=None,
                       forces=0, reserved0=0)
    h = C.c_void_p()
    st = L.fr_build_operators(C.byref(md), C.byref(prm), C.byref(h))
    return st, L.fr_last_error().decode(), h


def test_host_validation_errors_without_gpu():
    lb = _lib()
    L = lb.lib()
    # NULL arguments
    assert L.fr_build_operators(None, None, None) == lb.FR_ERR_ARG
    assert L.fr_rhs(None, None, None, None) == lb.FR_ERR_ARG
    assert L.fr_rk_step(None, None, None, 1, 0, None) == lb.FR_ERR_ARG
    assert L.fr_rhs_vjp(None, None, None, None, None, None) == lb.FR_ERR_ARG
    shp = (C.c_int64 * 3)()
    assert L.fr_state_shape(None, shp) == lb.FR_ERR_ARG
    # unsupported degree
    m = fi.periodic_box(2, 3, q=1)
    st, msg, _ = _build(m, p=7)
    assert st == lb.FR_ERR_UNSUPPORTED
    # unmatched face
    m = fi.periodic_box(2, 3, q=1)
    m.periodic_vec = m.periodic_vec[:1]
    st, msg, _ = _build(m)
    assert st == lb.FR_ERR_MESH and "unmatched" in msg
    # inverted element
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    m.elem_nodes[0] = m.elem_nodes[0][[1, 0, 3, 2]]
    st, msg, _ = _build(m)
    assert st == lb.FR_ERR_MESH and "Jacobian" in msg
    # probe outside the mesh
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    st, msg, _ = _build(m, probes=np.array([[50.0, 0.0]]))
    assert st == lb.FR_ERR_MESH and "probe" in msg
    # unknown face tag
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    m.face_bc[0, 0] = 9
    st, msg, _ = _build(m)
    assert st == lb.FR_ERR_ARG
    L.fr_destroy(None)


# ----------------------------------------------------------------------------- host statistics
def _dp(a):
    return a.ctypes.data_as(C.c_void_p)


def test_host_statistics_match_the_oracle():
    """fr_stats_* (plain host code of the library) against the oracle's definitions on seeded
    series shaped like probe pressure records (p_inf ~ 17.9 plus small fluctuations)."""
    from oracle import cumulative_prms, observer_oaspl, welch_psd
    L = _lib().lib()
    rng = np.random.default_rng(12)
    n = 2500
    t = np.arange(n) * 0.02
    S = np.stack([17.857 + 1e-3 * np.sin(2.1 * t + a) + 2e-4 * rng.normal(size=n) for a in range(6)])
    S = np.ascontiguousarray(S)
    # cumulative RMS vectors
    out = np.zeros(n)
    assert L.fr_stats_prms_cumulative(_dp(S[2]), n, _dp(out)) == 0
    ref = cumulative_prms(S[2])
    np.testing.assert_allclose(out, ref, rtol=1e-9, atol=0)
    # spanwise observers: probes 0-2 and 3-5
    grp = np.array([0, 0, 0, 1, 1, 1], dtype=np.int32)
    prms = np.zeros(2)
    db = np.zeros(2)
    assert L.fr_stats_observer_oaspl(_dp(S), 6, n, _dp(grp), 2, 2e-5, _dp(prms), _dp(db)) == 0
    rp, rd = observer_oaspl(S, grp, 2, 2e-5)
    np.testing.assert_allclose(prms, rp, rtol=1e-9)
    np.testing.assert_allclose(db, rd, rtol=0, atol=1e-9)
    # Welch PSD
    cap = 2000
    f = np.zeros(cap)
    P = np.zeros(cap)
    nf = C.c_int64()
    assert L.fr_stats_psd_welch(_dp(S[4]), n, 6, 0.02, _dp(f), _dp(P), cap, C.byref(nf)) == 0
    fr, Pr = welch_psd(S[4], 6, 0.02)
    assert nf.value == len(fr)
    np.testing.assert_allclose(f[:nf.value], fr, rtol=1e-13)
    np.testing.assert_allclose(P[:nf.value], Pr, rtol=1e-8, atol=1e-10 * Pr.max())


def test_host_statistics_argument_errors():
    L = _lib().lib()
    x = np.ones(10)
    out = np.zeros(10)
    nf = C.c_int64()
    assert L.fr_stats_prms_cumulative(None, 10, _dp(out)) == -1
    assert L.fr_stats_prms_cumulative(_dp(x), 0, _dp(out)) == -1
    assert L.fr_stats_psd_welch(_dp(x), 5, 6, 0.1, _dp(out), _dp(out), 10, C.byref(nf)) == -1  # too short
    y = np.ones(100)
    assert L.fr_stats_psd_welch(_dp(y), 100, 3, 0.1, _dp(out), _dp(out), 10, C.byref(nf)) == -1  # cap < L/2+1
    assert nf.value == 26
    grp = np.array([0, 2], dtype=np.int32)
    two = np.ones((2, 10))
    assert L.fr_stats_observer_oaspl(_dp(two), 2, 10, _dp(grp), 2, 1.0, _dp(out), _dp(out)) == -1
    # a work area no host can hold is refused with FR_ERR_OOM before any sample is read (the
    # exception stays inside the library)
    huge = 1 << 62
    assert L.fr_stats_psd_welch(_dp(y), huge, 1, 0.1, _dp(out), _dp(out), huge, C.byref(nf)) == -6
    assert L.fr_stats_observer_oaspl(_dp(two), 2, huge, _dp(np.zeros(2, dtype=np.int32)), 1, 1.0, _dp(out),
                                     _dp(out)) == -6


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits non-zero with a message that says so
    (before touching a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr, r.stderr


def test_trajectory_adjoint_needs_one_stored_sample_per_step():
    """The trajectory adjoint reads back one probe sample per step, so a solver whose device series
    holds fewer samples than the steps (or that has no probes) is refused before any step runs."""
    import torch
    from paper_2312_14167_amd.adjoint import FRTrajectory

    class _Small:
        n_probe, max_samples = 2, 3

    class _NoProbe:
        n_probe, max_samples = 0, 0

    for s in (_Small(), _NoProbe()):
        with pytest.raises(ValueError, match="max_samples"):
            FRTrajectory.apply(torch.zeros(4, dtype=torch.float64), s, torch.zeros(1, dtype=torch.float64),
                               5, 1, None)


def test_algorithmic_bytes_follow_the_face_flags():
    """The bench's byte model: with the one-sided LDG and faces of at least 256 bytes (3-D p = 4)
    the stage kernels write u_f only on the pairs' provider faces and the boundary; with smaller
    faces (2-D p = 4 FP32) or the two-sided LDG every face is written."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    # two hexes sharing one face: 25 flux-point pairs, 250 boundary points
    Ne, NV, Ns, Nf, npair, nbnd = 2, 5, 125, 150, 25, 250
    info = (Ne, NV, Ns, Nf, npair, nbnd, 0, 1)
    one = bench.algorithmic_bytes(info, 3, 8, "ns", 0.5)
    two = bench.algorithmic_bytes(info, 3, 8, "ns", 0.3)
    assert one["interp"] == Ne * NV * Ns * 8 + (npair + nbnd) * NV * 8 + Ne
    assert two["interp"] == Ne * NV * Ns * 8 + Ne * Nf * NV * 8 + Ne
    assert two["div_rk"] - one["div_rk"] == (Ne * Nf - npair - nbnd) * NV * 8
    # 2-D p = 4 in FP32: a face is 4 x 5 x 4 = 80 bytes, every face written
    info2 = (Ne, 4, 25, 20, 5, 30, 0, 1)
    b2 = bench.algorithmic_bytes(info2, 2, 4, "ns", 0.5)
    assert b2["interp"] == Ne * 4 * 25 * 4 + Ne * 20 * 4 * 4 + Ne


def _vdeg_build(m, deg, eq="ns", probes=None, n_mesh_override=None):
    from paper_2312_14167_amd.solver import marshal
    lb = _lib()
    L = lb.lib()
    fp = fi.freestream_params(m.dim, 0.2, 100.0 if eq == "ns" else None)
    md, prm, keep = marshal(m, 0, fp, eq, "fp64", probes, None, 4 if probes is not None else 0, False)
    if n_mesh_override:
        md.n_mesh = n_mesh_override
    d = np.ascontiguousarray(np.asarray(deg, dtype=np.int32))
    h = C.c_void_p()
    st = L.fr_vdeg_build(C.byref(md), d.ctypes.data_as(C.c_void_p), C.byref(prm), C.byref(h))
    return st, L.fr_last_error().decode(), h


def test_variable_degree_host_validation_without_gpu():
    """fr_vdeg_build refuses bad arguments before any device work: NULL pointers, degrees outside
    0..4, the Euler equations and several meshes (not built), the internal mortar face tag given
    as input, and a probe outside the mesh."""
    lb = _lib()
    L = lb.lib()
    assert L.fr_vdeg_build(None, None, None, None) == lb.FR_ERR_ARG
    h = C.c_void_p()
    assert L.fr_vdeg_build(None, None, None, C.byref(h)) == lb.FR_ERR_ARG
    m = fi.periodic_box(2, 3, q=1, bc="farfield")
    deg = np.full(m.n_elem, 2)
    deg[0] = 5
    st, msg, _ = _vdeg_build(m, deg)
    assert st == lb.FR_ERR_ARG and "degree" in msg
    st, msg, _ = _vdeg_build(m, np.full(m.n_elem, 2), eq="euler")
    assert st == lb.FR_ERR_UNSUPPORTED
    st, msg, _ = _vdeg_build(m, np.full(m.n_elem, 2), n_mesh_override=2)
    assert st == lb.FR_ERR_UNSUPPORTED
    m2 = fi.periodic_box(2, 3, q=1, bc="farfield")
    m2.face_bc[0, 0] = 3
    st, msg, _ = _vdeg_build(m2, np.full(m2.n_elem, 2))
    assert st == lb.FR_ERR_ARG and "tag" in msg
    st, msg, _ = _vdeg_build(m, np.full(m.n_elem, 2), probes=np.array([[50.0, 0.0]]))
    assert st == lb.FR_ERR_MESH and "probe" in msg
    assert L.fr_vdeg_rhs(None, None, None, None) == lb.FR_ERR_ARG
    assert L.fr_vdeg_rk_step(None, None, None, 1, 0, None) == lb.FR_ERR_ARG
    L.fr_vdeg_destroy(None)
