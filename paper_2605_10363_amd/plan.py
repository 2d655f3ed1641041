"""Python front end of libkldi: a plan per geometry, evaluations on device tensors."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """kldi_plan_create / kldi_eval / kldi_plan_destroy for one molecular geometry.

    atom_xyz [n_atoms, 3] (bohr); basis with shell_atom, shell_l, prim_ptr, prim_exp, prim_coef;
    grid_xyz [n_points, 3], weights [n_points], point_atom [n_points]; all host arrays (copied).
    """

    def __init__(self, atom_xyz, basis, grid_xyz, weights, point_atom, xc="lda", prec="fp64", t_b=1e-10,
                 t_d=1e-10, rho_cut=1e-14, grid_block=128, ao_block=32, v_segment=0, stream=None):
        self._h = ctypes.c_void_p()
        self._keep = [np.ascontiguousarray(atom_xyz, np.float64),
                      np.ascontiguousarray(basis.shell_atom, np.int32),
                      np.ascontiguousarray(basis.shell_l, np.int32),
                      np.ascontiguousarray(basis.prim_ptr, np.int32),
                      np.ascontiguousarray(basis.prim_exp, np.float64),
                      np.ascontiguousarray(basis.prim_coef, np.float64),
                      np.ascontiguousarray(grid_xyz, np.float64),
                      np.ascontiguousarray(weights, np.float64),
                      np.ascontiguousarray(point_atom, np.int32)]
        ax, sa, sl, pp, pe, pc, gx, gw, ga = self._keep
        b = L.kldi_basis(ax.shape[0], ax.ctypes.data, sl.shape[0], sa.ctypes.data, sl.ctypes.data, pp.ctypes.data,
                         pe.ctypes.data, pc.ctypes.data)
        g = L.kldi_grid(gw.shape[0], gx.ctypes.data, gw.ctypes.data, ga.ctypes.data)
        o = L.kldi_opts()
        L.kldi_opts_default(ctypes.byref(o))
        o.t_b, o.t_d, o.rho_cut = float(t_b), float(t_d), float(rho_cut)
        o.grid_block, o.ao_block = int(grid_block), int(ao_block)
        o.prec, o.xc, o.v_segment = L.PREC[prec], L.XC[xc], int(v_segment)
        self.xc, self.prec = xc, prec
        L.check(L.kldi_plan_create(ctypes.byref(b), ctypes.byref(g), ctypes.byref(o), _stream_handle(stream),
                                   ctypes.byref(self._h)), "kldi_plan_create")
        self.n_ao = int(sl.shape[0] and sum((l + 1) * (l + 2) // 2 for l in sl))
        self.n_points = int(gw.shape[0])

    def info(self) -> dict:
        i = L.kldi_plan_info_t()
        L.check(L.kldi_plan_info(self._h, ctypes.byref(i)), "kldi_plan_info")
        return {k: getattr(i, k) for k, _ in i._fields_}

    def structure(self):
        inf = self.info()
        nt, nb = inf["n_tiles"], inf["n_blocks"]
        ao = np.empty(self.n_ao, np.int32)
        pt = np.empty(self.n_points, np.int64)
        ret = np.empty(nt * nb, np.uint8)
        bmax = np.empty(nt * nb, np.float64)
        L.check(L.kldi_plan_structure(self._h, ao.ctypes.data, pt.ctypes.data, ret.ctypes.data, bmax.ctypes.data),
                "kldi_plan_structure")
        return ao, pt, ret.reshape(nb, nt), bmax.reshape(nb, nt)

    def eval(self, D, rho=True, vxc=True, out=None, stream=None):
        """One EXC evaluation.  D: torch float64 CUDA tensor [n_ao, n_ao].  Returns (rho, exc, vxc)
        device tensors (rho/vxc None when not requested); the work is only enqueued."""
        if not (isinstance(D, torch.Tensor) and D.is_cuda and D.dtype == torch.float64 and D.is_contiguous()):
            raise TypeError("D must be a contiguous float64 CUDA tensor")
        if tuple(D.shape) != (self.n_ao, self.n_ao):
            raise ValueError("D must be [n_ao, n_ao] = [%d, %d]" % (self.n_ao, self.n_ao))
        dev = D.device
        if out is None:
            out = (torch.empty(self.n_points, dtype=torch.float64, device=dev) if rho else None,
                   torch.empty(1, dtype=torch.float64, device=dev),
                   torch.empty(self.n_ao, self.n_ao, dtype=torch.float64, device=dev) if vxc else None)
        r, e, v = out
        L.check(L.kldi_eval(self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(r.data_ptr() if r is not None else 0),
                            ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(v.data_ptr() if v is not None else 0),
                            _stream_handle(stream)), "kldi_eval")
        return r, e, v

    def check(self, stream=None) -> dict:
        s = L.kldi_eval_stats_t()
        st = L.kldi_eval_check(self._h, ctypes.byref(s), _stream_handle(stream))
        out = {k: getattr(s, k) for k, _ in s._fields_}
        L.check(st, "kldi_eval_check")
        return out

    def timing(self, enable=True):
        L.check(L.kldi_plan_timing(self._h, 1 if enable else 0), "kldi_plan_timing")

    def stage_ms(self):
        ms = (ctypes.c_double * len(L.STAGES))()
        n = ctypes.c_int32()
        L.check(L.kldi_eval_timing(self._h, ms, ctypes.byref(n)), "kldi_eval_timing")
        return dict(zip(L.STAGES, list(ms))), int(n.value)

    def close(self):
        if self._h:
            L.kldi_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @classmethod
    def from_problem(cls, p, **kw):
        kw.setdefault("xc", p.xc)
        return cls(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, **kw)
