"""Python binding of the FR library: same operations as the C ABI, torch tensors for device
memory and the current HIP stream.  Every step of the path runs in libfrmi's kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import FR_EULER, FR_FP32, FR_FP64, FR_NAVIER_STOKES, FR_TUNE_MAX, check, fr_mesh_desc, fr_params, lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def marshal(mesh, p: int, flow, equations: str, precision: str, probes=None, probe_mesh=None,
            max_samples: int = 0, forces: bool = False):
    """fr_mesh_desc and fr_params of a mesh and flow; the arrays they point to are returned too and
    must stay alive during the build call (the first one is the node array)."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(np.asarray(a, dtype=dt))
        keep.append(a)
        return a
    node = arr(mesh.node_xyz, np.float64)
    en = arr(mesh.elem_nodes, np.int64)
    fb = arr(mesh.face_bc, np.int32)
    pv = arr(np.asarray(mesh.periodic_vec).reshape(-1, mesh.dim), np.float64)
    mb = arr(mesh.mesh_elem_begin, np.int64)
    md = fr_mesh_desc(dim=mesh.dim, p=p, geom_q=mesh.q, n_periodic=pv.shape[0], n_elem=en.shape[0],
                      n_node=node.shape[0], node_xyz=_ptr(node), elem_nodes=_ptr(en), face_bc=_ptr(fb),
                      periodic_vec=_ptr(pv), n_mesh=mesh.n_mesh, reserved0=0, mesh_elem_begin=_ptr(mb))
    rho = arr(flow.rho_inf, np.float64)
    vel = arr(flow.vel_inf, np.float64)
    pin = arr(flow.p_inf, np.float64)
    mu = arr(flow.mu, np.float64)
    npb = 0
    pxyz = pm = None
    if probes is not None:
        pxyz = arr(np.atleast_2d(probes), np.float64)
        npb = pxyz.shape[0]
        pm = arr(np.zeros(npb) if probe_mesh is None else probe_mesh, np.int32)
    prm = fr_params(equations=FR_NAVIER_STOKES if equations == "ns" else FR_EULER,
                    precision=FR_FP64 if precision == "fp64" else FR_FP32,
                    gamma=flow.gamma, prandtl=flow.prandtl, ldg_beta=flow.ldg_beta, ldg_tau=flow.ldg_tau,
                    rho_inf=_ptr(rho), vel_inf=_ptr(vel), p_inf=_ptr(pin), mu=_ptr(mu),
                    n_probe=npb, max_samples=max(int(max_samples), 1 if npb else 0),
                    probe_xyz=_ptr(pxyz), probe_mesh=_ptr(pm), forces=1 if forces else 0, reserved0=0)
    return md, prm, keep


class Solver:
    """One FR discretisation (one or several concatenated meshes) on the current GPU.

    ``mesh``: mesh description (node coordinates, GLL element nodes, face tags, periodic
    translations, element ranges); ``flow``: per-mesh free stream / viscosity and fluid
    constants.  ``precision`` 'fp64' or 'fp32' (accumulators stay FP64).
    """

    def __init__(self, mesh, p: int, flow, equations: str = "ns", precision: str = "fp64", probes=None,
                 probe_mesh=None, max_samples: int = 0, forces: bool = False):
        L = lib()
        self.dim = mesh.dim
        self.p = p
        self.n_mesh = mesh.n_mesh
        self.equations = equations
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        md, prm, keep = marshal(mesh, p, flow, equations, precision, probes, probe_mesh, max_samples, forces)
        node = keep[0]
        npb = int(prm.n_probe)
        self.n_node = int(node.shape[0])
        self.node_xyz = node.copy()
        self.max_samples = int(prm.max_samples)  # capacity of the device series
        h = C.c_void_p()
        check(L.fr_build_operators(C.byref(md), C.byref(prm), C.byref(h)))
        self._h = h
        shp = (C.c_int64 * 3)()
        check(L.fr_state_shape(h, shp))
        self.shape = tuple(int(x) for x in shp)
        self.n_probe = npb

    # ----------------------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().fr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_state(self, t: torch.Tensor, name: str):
        if not (t.is_cuda and t.dtype == self.dtype and tuple(t.shape) == self.shape and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor of shape {self.shape}")

    def new_state(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def solpt_coords(self) -> np.ndarray:
        out = np.empty((self.shape[0], self.shape[2], self.dim))
        check(lib().fr_solpt_coords(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def rhs(self, u: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._check_state(u, "u")
        r = self.new_state() if out is None else out
        self._check_state(r, "out")
        check(lib().fr_rhs(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(r.data_ptr()), _stream(stream)))
        return r

    def rk_step(self, u: torch.Tensor, dt: torch.Tensor, n_steps: int = 1, sample_every: int = 0, stream=None):
        self._check_state(u, "u")
        if not (dt.is_cuda and dt.dtype == torch.float64 and dt.numel() == self.n_mesh and dt.is_contiguous()):
            raise ValueError("dt must be a contiguous float64 CUDA tensor with one entry per mesh")
        check(lib().fr_rk_step(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(dt.data_ptr()), int(n_steps),
                               int(sample_every), _stream(stream)))
        return u

    def reset_accumulators(self, stream=None):
        check(lib().fr_reset_accumulators(self._h, _stream(stream)))

    def probe_oaspl(self, p_ref: float = 1.0, stream=None) -> dict:
        npb = max(self.n_probe, 1)
        prms = np.zeros(npb)
        oaspl = np.zeros(npb)
        force = np.zeros(self.n_mesh * self.dim)
        n = C.c_int64()
        check(lib().fr_probe_oaspl(self._h, float(p_ref), prms.ctypes.data_as(C.c_void_p),
                                   oaspl.ctypes.data_as(C.c_void_p), force.ctypes.data_as(C.c_void_p),
                                   C.byref(n), _stream(stream)))
        return {"prms": prms[:self.n_probe], "oaspl": oaspl[:self.n_probe],
                "mean_force": force.reshape(self.n_mesh, self.dim), "n_samples": int(n.value)}

    def force_coefficients(self, directions, ref_area, stream=None) -> np.ndarray:
        """Eq. (8): time-mean wall force of each mesh along each direction over the free-stream
        dynamic pressure times ref_area.  directions [n_mesh][n_dir][dim] (or [n_dir][dim] for
        all meshes), ref_area scalar or [n_mesh] -> [n_mesh][n_dir]."""
        d = np.asarray(directions, dtype=np.float64)
        if d.ndim == 2:
            d = np.broadcast_to(d, (self.n_mesh,) + d.shape)
        d = np.ascontiguousarray(d)
        if d.shape[0] != self.n_mesh or d.shape[2] != self.dim:
            raise ValueError("directions must be [n_mesh][n_dir][dim]")
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(ref_area, dtype=np.float64), (self.n_mesh,)))
        out = np.zeros((self.n_mesh, d.shape[1]))
        check(lib().fr_force_coefficients(self._h, int(d.shape[1]), d.ctypes.data_as(C.c_void_p),
                                          a.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p),
                                          _stream(stream)))
        return out

    def probe_series(self, cap: int, stream=None) -> np.ndarray:
        out = np.zeros((max(self.n_probe, 1), cap))
        n = C.c_int64()
        check(lib().fr_probe_series(self._h, out.ctypes.data_as(C.c_void_p), int(cap), C.byref(n), _stream(stream)))
        return out[:self.n_probe, :min(int(n.value), cap, self.max_samples)]

    TUNE_KINDS = ["ns_volume", "ns_lift_rk", "euler_volume_rk", "ns_volume_adjoint"]

    def autotune(self, u: torch.Tensor, dt: torch.Tensor, reps: int = 3, kinds=None, stream=None) -> dict:
        """Time the candidates of the volume kernels on this mesh (tile size x waves-per-SIMD bound,
        and the matrix-core divergence where compiled; u is not modified), keep the fastest (or the
        choice remembered for this shape); returns per kernel the chosen candidate and the ms per
        step of every candidate.  kinds: names from TUNE_KINDS to tune (default: all of the
        solver's)."""
        self._check_state(u, "u")
        self._check_dt(dt)
        choice = np.zeros(16, dtype=np.int32)
        ms = np.zeros(4 * FR_TUNE_MAX)
        mask = 0 if kinds is None else sum(1 << self.TUNE_KINDS.index(k) for k in kinds)
        check(lib().fr_autotune(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(dt.data_ptr()), int(reps), int(mask),
                                choice.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p), _stream(stream)))
        kinds = [k for k in ([0, 1, 3] if self.equations == "ns" else [2])
                 if kinds is None or self.TUNE_KINDS[k] in kinds]
        out = {}
        for k in kinds:
            cands = self.tune_candidates(k)
            if not cands:
                continue
            out[self.TUNE_KINDS[k]] = {
                "elements_per_workgroup": int(choice[4 * k]), "waves_per_simd_bound": int(choice[4 * k + 1]),
                "engine": "mfma" if choice[4 * k + 2] else "valu", "from_cache": bool(choice[4 * k + 3]),
                "candidates": [{"E": c[0], "waves": c[1], "engine": "mfma" if c[2] else "valu",
                                "ms_per_step": float(ms[k * FR_TUNE_MAX + i])} for i, c in enumerate(cands)]}
        return out

    def tune_candidates(self, kind: int):
        """[(elements per workgroup, waves-per-SIMD bound (0: default), engine (1: matrix cores))]"""
        cand = np.zeros(3 * FR_TUNE_MAX, dtype=np.int32)
        n = C.c_int32()
        check(lib().fr_tune_candidates(self._h, int(kind), cand.ctypes.data_as(C.c_void_p), C.byref(n)))
        return [tuple(int(x) for x in cand[3 * i:3 * i + 3]) for i in range(n.value)]

    def tune_select(self, kind: int, index: int):
        check(lib().fr_tune_select(self._h, int(kind), int(index)))

    def probe_statistics(self, p_ref: float, groups=None, n_windows: int = 6, sample_dt: float | None = None,
                         cap: int | None = None) -> dict:
        """Host statistics of the recorded probe series (library host code): the cumulative p_RMS
        vector of every probe (Eqs. (10)-(12)), the OASPL of each observer whose probes are
        grouped by ``groups`` (spanwise average of p_RMS; default: one observer per probe) and,
        with ``sample_dt`` (time between samples), the Welch PSD of every probe."""
        series = np.ascontiguousarray(self.probe_series(cap or 1 << 20))
        npb, n = series.shape
        if n == 0:
            raise ValueError("no samples recorded")
        L = lib()
        cum = np.zeros((npb, n))
        for a in range(npb):
            check(L.fr_stats_prms_cumulative(series[a].ctypes.data_as(C.c_void_p), n,
                                             cum[a].ctypes.data_as(C.c_void_p)))
        grp = np.ascontiguousarray(np.arange(npb) if groups is None else np.asarray(groups), dtype=np.int32)
        ng = int(grp.max()) + 1
        prms = np.zeros(ng)
        oaspl = np.zeros(ng)
        check(L.fr_stats_observer_oaspl(series.ctypes.data_as(C.c_void_p), npb, n, grp.ctypes.data_as(C.c_void_p),
                                        ng, float(p_ref), prms.ctypes.data_as(C.c_void_p),
                                        oaspl.ctypes.data_as(C.c_void_p)))
        out = {"prms_cumulative": cum, "observer_prms": prms, "observer_oaspl": oaspl}
        if sample_dt is not None:
            nf = C.c_int64()
            spec = []
            for a in range(npb):
                f = np.zeros(n)
                P = np.zeros(n)
                check(L.fr_stats_psd_welch(series[a].ctypes.data_as(C.c_void_p), n, int(n_windows), float(sample_dt),
                                           f.ctypes.data_as(C.c_void_p), P.ctypes.data_as(C.c_void_p), n,
                                           C.byref(nf)))
                spec.append(P[:nf.value])
            out["freq"] = f[:nf.value]
            out["psd"] = np.stack(spec)
        return out

    def info(self) -> dict:
        a = np.zeros(8, dtype=np.int64)
        check(lib().fr_solver_info(self._h, a.ctypes.data_as(C.c_void_p)))
        keys = ["n_elem", "nv", "ns", "nf", "n_pairs", "n_boundary", "n_wall", "n_mesh"]
        return dict(zip(keys, (int(x) for x in a)))

    def _xbar_ptr(self, x_bar):
        if x_bar is None:
            return None
        if not (x_bar.is_cuda and x_bar.dtype == torch.float64 and tuple(x_bar.shape) == (self.n_node, self.dim)
                and x_bar.is_contiguous()):
            raise ValueError(f"x_bar must be a contiguous float64 CUDA tensor of shape {(self.n_node, self.dim)}")
        return C.c_void_p(x_bar.data_ptr())

    def _check_dt(self, dt):
        if not (dt.is_cuda and dt.dtype == torch.float64 and dt.numel() == self.n_mesh and dt.is_contiguous()):
            raise ValueError("dt must be a contiguous float64 CUDA tensor with one entry per mesh")

    def probe_vjp(self, u: torch.Tensor, p_bar: torch.Tensor, u_bar: torch.Tensor, x_bar=None, stream=None):
        """u_bar += sum_a p_bar[a] dp_a/du (p_bar: float64 CUDA tensor [n_probe]); with x_bar
        (float64 [n_node, dim]) also x_bar += sum_a p_bar[a] dp_a/dX."""
        self._check_state(u, "u")
        self._check_state(u_bar, "u_bar")
        p_bar = p_bar.to(device=u.device, dtype=torch.float64).contiguous()
        check(lib().fr_probe_vjp(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(p_bar.data_ptr()),
                                 C.c_void_p(u_bar.data_ptr()), self._xbar_ptr(x_bar), _stream(stream)))
        return u_bar

    def rk_step_stages(self, u: torch.Tensor, dt: torch.Tensor, stages: torch.Tensor, states=None, residuals=None,
                       stream=None):
        """RK4 steps of u in place, recording each step's stage states y2, y3, y4 into stages
        ([3, *shape] for one step, [n, 3, *shape] for n steps) and, if given, each step's base
        state into states ([n, *shape]) and its four stage residuals into residuals ([n, 4, *shape]
        or [4, *shape])."""
        self._check_state(u, "u")
        self._check_dt(dt)
        one = tuple(stages.shape) == (3,) + self.shape
        n = 1 if one else int(stages.shape[0])
        if not (stages.is_cuda and stages.dtype == self.dtype and stages.is_contiguous()
                and (one or tuple(stages.shape) == (n, 3) + self.shape)):
            raise ValueError("stages must be a contiguous CUDA tensor of shape (3,) + state shape or (n, 3) + state shape")

        def opt(t, shape, name):
            if t is None:
                return None
            if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.numel() == int(np.prod(shape))):
                raise ValueError(f"{name} must be a contiguous CUDA tensor with the elements of {shape}")
            return C.c_void_p(t.data_ptr())
        sp = opt(states, (n,) + self.shape, "states")
        rp = opt(residuals, (n, 4) + self.shape, "residuals")
        check(lib().fr_rk_step_stages(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(dt.data_ptr()), n, sp,
                                      C.c_void_p(stages.data_ptr()), rp, _stream(stream)))
        return u

    def rk_step_vjp(self, u_n: torch.Tensor, dt: torch.Tensor, u_bar: torch.Tensor, stages=None, x_bar=None,
                    residuals=None, stream=None):
        """u_bar <- (d u_{n+1} / d u_n)^T u_bar for one RK4 step from u_n; with x_bar (float64
        [n_node, dim]) also x_bar += (d u_{n+1} / dX)^T u_bar, using the step's recorded stage
        residuals ([4, *shape]) when given."""
        self._check_state(u_n, "u_n")
        self._check_state(u_bar, "u_bar")
        self._check_dt(dt)
        sp = C.c_void_p(stages.data_ptr()) if stages is not None else None
        rp = C.c_void_p(residuals.data_ptr()) if residuals is not None else None
        check(lib().fr_rk_step_vjp(self._h, C.c_void_p(u_n.data_ptr()), C.c_void_p(dt.data_ptr()), sp, rp,
                                   C.c_void_p(u_bar.data_ptr()), self._xbar_ptr(x_bar), _stream(stream)))
        return u_bar

    def rk_segment_vjp(self, states: torch.Tensor, dt: torch.Tensor, u_bar: torch.Tensor, stages: torch.Tensor,
                       p_bar: torch.Tensor, n_steps: int, x_bar=None, residuals=None, stream=None):
        """Reverse of n_steps RK4 steps with their probe samples (see fr_rk_segment_vjp): states
        [>= n, *shape], stages [>= n, 3, *shape], residuals [>= n, 4, *shape] or None, p_bar
        float64 CUDA [>= n, n_probe]; replayed from a captured graph while the tensors repeat."""
        self._check_state(u_bar, "u_bar")
        self._check_dt(dt)
        n = int(n_steps)
        for t, name, shp in ((states, "states", (self.shape,)), (stages, "stages", ((3,) + self.shape,))):
            if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.shape[0] >= n
                    and tuple(t.shape[1:]) == shp[0]):
                raise ValueError(f"{name} has the wrong shape, dtype or layout")
        if residuals is not None and not (residuals.is_contiguous() and tuple(residuals.shape[1:]) == (4,) + self.shape
                                          and residuals.shape[0] >= n and residuals.dtype == self.dtype):
            raise ValueError("residuals has the wrong shape, dtype or layout")
        if not (p_bar.is_cuda and p_bar.dtype == torch.float64 and p_bar.is_contiguous()
                and tuple(p_bar.shape[1:]) == (self.n_probe,) and p_bar.shape[0] >= n):
            raise ValueError("p_bar must be a contiguous float64 CUDA tensor [n_steps, n_probe]")
        rp = C.c_void_p(residuals.data_ptr()) if residuals is not None else None
        check(lib().fr_rk_segment_vjp(self._h, C.c_void_p(states.data_ptr()), C.c_void_p(dt.data_ptr()),
                                      C.c_void_p(stages.data_ptr()), rp, C.c_void_p(p_bar.data_ptr()), n,
                                      C.c_void_p(u_bar.data_ptr()), self._xbar_ptr(x_bar), _stream(stream)))
        return u_bar

    def geo_adjoint_begin(self, stream=None):
        """Start a deferred mesh-node adjoint (see fr_geo_adjoint_begin)."""
        check(lib().fr_geo_adjoint_begin(self._h, _stream(stream)))

    def geo_adjoint_end(self, x_bar: torch.Tensor, stream=None):
        """x_bar += the node mapping of the metric / normal adjoints accumulated since begin."""
        check(lib().fr_geo_adjoint_end(self._h, self._xbar_ptr(x_bar), _stream(stream)))
        return x_bar

    def rhs_vjp_noalloc(self, u: torch.Tensor, r_bar: torch.Tensor, u_bar: torch.Tensor, stream=None):
        """u_bar += (dR/du)^T r_bar with the library's static per-GPU work area (no device
        allocation; see fr_rhs_vjp_noalloc)."""
        self._check_state(u, "u")
        self._check_state(r_bar, "r_bar")
        self._check_state(u_bar, "u_bar")
        check(lib().fr_rhs_vjp_noalloc(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(r_bar.data_ptr()),
                                       C.c_void_p(u_bar.data_ptr()), _stream(stream)))
        return u_bar

    def rhs_vjp(self, u: torch.Tensor, r_bar: torch.Tensor, u_bar: torch.Tensor, x_bar: torch.Tensor | None = None,
                stream=None):
        self._check_state(u, "u")
        self._check_state(r_bar, "r_bar")
        self._check_state(u_bar, "u_bar")
        check(lib().fr_rhs_vjp(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(r_bar.data_ptr()),
                               C.c_void_p(u_bar.data_ptr()), self._xbar_ptr(x_bar), _stream(stream)))
        return u_bar
