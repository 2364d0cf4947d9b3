"""Python binding of the variable-degree solver (fr_vdeg_* in include/fr.h): one solution degree
per element in 0..4, faces between degrees coupled by mortars on the higher side's points.  The
state is one flat device buffer holding the degree groups in increasing degree (``split`` gives
per-group views [n_elem of the group, nv, (degree + 1)^dim], elements in increasing number)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import check, lib
from .solver import _ptr, _stream, marshal


class VarDegreeSolver:
    def __init__(self, mesh, degree, flow, precision: str = "fp64", probes=None, max_samples: int = 0,
                 forces: bool = False):
        L = lib()
        self.dim = mesh.dim
        self.nv = mesh.dim + 2
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        deg = np.ascontiguousarray(np.asarray(degree, dtype=np.int32))
        if deg.shape != (mesh.n_elem,):
            raise ValueError("one degree per element")
        md, prm, keep = marshal(mesh, 0, flow, "ns", precision, probes, None, max_samples, forces)
        self.n_probe = int(prm.n_probe)
        self.max_samples = int(prm.max_samples)
        h = C.c_void_p()
        check(L.fr_vdeg_build(C.byref(md), _ptr(deg), C.byref(prm), C.byref(h)))
        self._h = h
        ng = C.c_int32()
        dg = (C.c_int32 * 5)()
        ne = (C.c_int64 * 5)()
        off = (C.c_int64 * 6)()
        nm = C.c_int64()
        check(L.fr_vdeg_groups(h, C.byref(ng), dg, ne, off, C.byref(nm)))
        self.n_group = int(ng.value)
        self.degrees = [int(dg[g]) for g in range(self.n_group)]
        self.n_elem = [int(ne[g]) for g in range(self.n_group)]
        self.offset = [int(off[g]) for g in range(self.n_group + 1)]
        self.size = self.offset[-1]
        self.n_mortar = int(nm.value)
        self.elems = []
        for g in range(self.n_group):
            e = np.zeros(self.n_elem[g], dtype=np.int64)
            check(L.fr_vdeg_group_elems(h, g, e.ctypes.data_as(C.c_void_p)))
            self.elems.append(e)

    def close(self):
        if getattr(self, "_h", None):
            lib().fr_vdeg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def group_shape(self, g: int):
        return (self.n_elem[g], self.nv, (self.degrees[g] + 1) ** self.dim)

    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.size, dtype=self.dtype, device="cuda")

    def split(self, flat: torch.Tensor):
        """Views of the groups' states inside the flat buffer."""
        out = []
        for g in range(self.n_group):
            shp = self.group_shape(g)
            n = shp[0] * shp[1] * shp[2]
            out.append(flat[self.offset[g]:self.offset[g] + n].view(shp))
        return out

    def join(self, parts, out: torch.Tensor | None = None) -> torch.Tensor:
        """Flat buffer from per-group states [n_elem, nv, Ns] (any device; copied)."""
        flat = self.new_state() if out is None else out
        for v, p in zip(self.split(flat), parts):
            v.copy_(torch.as_tensor(p).to(dtype=self.dtype).reshape(v.shape))
        return flat

    def solpt_coords(self):
        out = []
        for g in range(self.n_group):
            n, _, ns = self.group_shape(g)
            x = np.empty((n, ns, self.dim))
            check(lib().fr_vdeg_solpt_coords(self._h, g, x.ctypes.data_as(C.c_void_p)))
            out.append(x)
        return out

    def _check(self, t: torch.Tensor, name: str):
        if not (t.is_cuda and t.dtype == self.dtype and t.dim() == 1 and t.numel() == self.size and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor of {self.size} values")

    def rhs(self, u: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._check(u, "u")
        r = self.new_state() if out is None else out
        self._check(r, "out")
        check(lib().fr_vdeg_rhs(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(r.data_ptr()), _stream(stream)))
        return r

    def rk_step(self, u: torch.Tensor, dt: torch.Tensor, n_steps: int = 1, sample_every: int = 0, stream=None):
        self._check(u, "u")
        if not (dt.is_cuda and dt.dtype == torch.float64 and dt.numel() == 1):
            raise ValueError("dt must be a float64 CUDA tensor with one entry")
        check(lib().fr_vdeg_rk_step(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(dt.data_ptr()), int(n_steps),
                                    int(sample_every), _stream(stream)))
        return u

    def reset_accumulators(self, stream=None):
        check(lib().fr_vdeg_reset_accumulators(self._h, _stream(stream)))

    def probe_series(self, cap: int, stream=None) -> np.ndarray:
        out = np.zeros((max(self.n_probe, 1), cap))
        n = C.c_int64()
        check(lib().fr_vdeg_probe_series(self._h, out.ctypes.data_as(C.c_void_p), int(cap), C.byref(n),
                                         _stream(stream)))
        return out[:self.n_probe, :min(int(n.value), cap, self.max_samples)]

    def mean_force(self, stream=None):
        f = np.zeros(self.dim)
        n = C.c_int64()
        check(lib().fr_vdeg_mean_force(self._h, f.ctypes.data_as(C.c_void_p), C.byref(n), _stream(stream)))
        return f, int(n.value)
