"""Python front end of libkldi: a plan per geometry (or per batch of geometries), evaluations on
device tensors."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _structs(atom_xyz, basis, grid_xyz, weights, point_atom, keep):
    arrs = [np.ascontiguousarray(atom_xyz, np.float64), np.ascontiguousarray(basis.shell_atom, np.int32),
            np.ascontiguousarray(basis.shell_l, np.int32), np.ascontiguousarray(basis.prim_ptr, np.int32),
            np.ascontiguousarray(basis.prim_exp, np.float64), np.ascontiguousarray(basis.prim_coef, np.float64),
            np.ascontiguousarray(grid_xyz, np.float64), np.ascontiguousarray(weights, np.float64),
            np.ascontiguousarray(point_atom, np.int32)]
    keep.extend(arrs)
    ax, sa, sl, pp, pe, pc, gx, gw, ga = arrs
    b = L.kldi_basis(ax.shape[0], ax.ctypes.data, sl.shape[0], sa.ctypes.data, sl.ctypes.data, pp.ctypes.data,
                     pe.ctypes.data, pc.ctypes.data)
    g = L.kldi_grid(gw.shape[0], gx.ctypes.data, gw.ctypes.data, ga.ctypes.data)
    n_ao = int(sum((int(l) + 1) * (int(l) + 2) // 2 for l in sl))
    return b, g, n_ao, int(gw.shape[0])


def _opts(xc, prec, t_b, t_d, rho_cut, grid_block, ao_block, v_segment, chunk_tiles, schedule):
    o = L.kldi_opts()
    L.kldi_opts_default(ctypes.byref(o))
    o.t_b, o.t_d, o.rho_cut = float(t_b), float(t_d), float(rho_cut)
    o.grid_block, o.ao_block = int(grid_block), int(ao_block)
    o.prec, o.xc, o.v_segment, o.chunk_tiles = L.PREC[prec], L.XC[xc], int(v_segment), int(chunk_tiles)
    o.schedule = L.SCHED[schedule]
    return o


def _check_d(D, n):
    if not (isinstance(D, torch.Tensor) and D.is_cuda and D.dtype == torch.float64 and D.is_contiguous()):
        raise TypeError("D must be a contiguous float64 CUDA tensor")
    if D.numel() != n:
        raise ValueError("D must hold %d elements" % n)


class _PlanBase:
    """Common part of a single-molecule plan and a batch plan (one libkldi plan handle)."""

    n_mol = 1

    def info(self) -> dict:
        i = L.kldi_plan_info_t()
        L.check(L.kldi_plan_info(self._h, ctypes.byref(i)), "kldi_plan_info")
        return {k: getattr(i, k) for k, _ in i._fields_}

    def _eval(self, D, n_d, n_pts, rho, vxc, out, stream, vshape):
        _check_d(D, n_d)
        dev = D.device
        if out is None:
            out = (torch.empty(n_pts, dtype=torch.float64, device=dev) if rho else None,
                   torch.empty(self.n_mol, dtype=torch.float64, device=dev),
                   torch.empty(vshape, dtype=torch.float64, device=dev) if vxc else None)
        r, e, v = out
        L.check(L.kldi_eval(self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(r.data_ptr() if r is not None else 0),
                            ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(v.data_ptr() if v is not None else 0),
                            _stream_handle(stream)), "kldi_eval")
        return r, e, v

    def grad(self, D, exc=None, stream=None):
        """kldi_eval_grad: dE_xc/dR (n_atoms x 3 float64 CUDA tensor) with the grid held fixed."""
        _check_d(D, self.n_ao * self.n_ao)
        g = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=D.device)
        L.check(L.kldi_eval_grad(self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(exc.data_ptr() if exc is not None else 0), _stream_handle(stream)),
                "kldi_eval_grad")
        return g

    def attach_mlp(self, mlp):
        L.check(L.kldi_plan_attach_mlp(self._h, mlp._h if mlp is not None else None), "kldi_plan_attach_mlp")
        self._mlp = mlp

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

    def graph(self, enable=True):
        """Replay a captured HIP graph per evaluation (kldi_plan_graph)."""
        L.check(L.kldi_plan_graph(self._h, 1 if enable else 0), "kldi_plan_graph")

    def autotune(self, D, reps=3, stream=None) -> dict:
        """kldi_plan_autotune with a representative D (packed as for eval)."""
        t = L.kldi_tune_t()
        L.check(L.kldi_plan_autotune(self._h, ctypes.c_void_p(D.data_ptr()), int(reps), _stream_handle(stream),
                                     ctypes.byref(t)), "kldi_plan_autotune")
        return {k: getattr(t, k) for k, _ in t._fields_}

    def close(self):
        if self._h:
            L.kldi_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan(_PlanBase):
    """kldi_plan_create / kldi_eval / kldi_plan_destroy for one molecular geometry.

    atom_xyz [n_atoms, 3] (bohr); basis with shell_atom, shell_l, prim_ptr, prim_exp, prim_coef;
    grid_xyz [n_points, 3], weights [n_points], point_atom [n_points]; all host arrays (copied).
    """

    def __init__(self, atom_xyz, basis, grid_xyz, weights, point_atom, xc="lda", prec="fp64", t_b=1e-10,
                 t_d=1e-10, rho_cut=1e-14, grid_block=128, ao_block=32, v_segment=0, chunk_tiles=0, schedule="grid",
                 shell_order=None, stream=None):
        """shell_order: None (atom order) or the internal sequence of shells (e.g. overlap_order())."""
        self._h = ctypes.c_void_p()
        self._keep = []
        b, g, self.n_ao, self.n_points = _structs(atom_xyz, basis, grid_xyz, weights, point_atom, self._keep)
        self.n_atoms = int(np.asarray(atom_xyz).shape[0])
        o = _opts(xc, prec, t_b, t_d, rho_cut, grid_block, ao_block, v_segment, chunk_tiles, schedule)
        if shell_order is not None:
            so = np.ascontiguousarray(shell_order, np.int32)
            self._keep.append(so)
            o.shell_order = so.ctypes.data
        self.xc, self.prec = xc, prec
        L.check(L.kldi_plan_create(ctypes.byref(b), ctypes.byref(g), ctypes.byref(o), _stream_handle(stream),
                                   ctypes.byref(self._h)), "kldi_plan_create")
        self._keep = None

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
        if tuple(D.shape) != (self.n_ao, self.n_ao):
            raise ValueError("D must be [n_ao, n_ao] = [%d, %d]" % (self.n_ao, self.n_ao))
        return self._eval(D, self.n_ao * self.n_ao, self.n_points, rho, vxc, out, stream, (self.n_ao, self.n_ao))

    def eval_grid(self, D, stream=None):
        """rho and sigma on the grid (device tensors, caller order) -- kldi_eval_grid."""
        _check_d(D, self.n_ao * self.n_ao)
        rho = torch.empty(self.n_points, dtype=torch.float64, device=D.device)
        sigma = torch.empty(self.n_points, dtype=torch.float64, device=D.device)
        L.check(L.kldi_eval_grid(self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                 ctypes.c_void_p(sigma.data_ptr()), _stream_handle(stream)), "kldi_eval_grid")
        return rho, sigma

    @classmethod
    def from_problem(cls, p, **kw):
        kw.setdefault("xc", p.xc)
        return cls(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, **kw)


class Batch(_PlanBase):
    """kldi_batch_create: one plan over many independent molecules (the batching form).

    problems: objects with atom_xyz, basis, grid (xyz, weight, point_atom).  D, rho and Vxc use the
    packed layout of kldi_batch_layout (offsets ao_off, d_off, pt_off); E_xc has one value per molecule.
    """

    def __init__(self, problems, xc="lda", prec="fp64", t_b=1e-10, t_d=1e-10, rho_cut=1e-14, grid_block=128,
                 ao_block=32, v_segment=0, chunk_tiles=0, schedule="grid", stream=None):
        self._h = ctypes.c_void_p()
        keep = []
        n = len(problems)
        bs = (L.kldi_basis * n)()
        gs = (L.kldi_grid * n)()
        self.n_aos, self.n_pts = [], []
        for m, p in enumerate(problems):
            b, g, na, npt = _structs(p.atom_xyz, p.basis, p.grid.xyz, p.grid.weight, p.grid.point_atom, keep)
            bs[m], gs[m] = b, g
            self.n_aos.append(na)
            self.n_pts.append(npt)
        o = _opts(xc, prec, t_b, t_d, rho_cut, grid_block, ao_block, v_segment, chunk_tiles, schedule)
        self.xc, self.prec, self.n_mol = xc, prec, n
        L.check(L.kldi_batch_create(n, bs, gs, ctypes.byref(o), _stream_handle(stream), ctypes.byref(self._h)),
                "kldi_batch_create")
        del keep
        self.ao_off = np.empty(n + 1, np.int64)
        self.d_off = np.empty(n + 1, np.int64)
        self.pt_off = np.empty(n + 1, np.int64)
        L.check(L.kldi_batch_layout(self._h, self.ao_off.ctypes.data, self.d_off.ctypes.data, self.pt_off.ctypes.data),
                "kldi_batch_layout")

    def pack(self, mats, device="cuda"):
        """Packed D (1-D float64 CUDA tensor) from one n_ao x n_ao array per molecule."""
        flat = np.concatenate([np.ascontiguousarray(m, np.float64).ravel() for m in mats])
        assert flat.size == self.d_off[-1]
        return torch.from_numpy(flat).to(device)

    def unpack(self, V):
        """Per-molecule n_ao x n_ao views of a packed Vxc."""
        return [V[self.d_off[m]:self.d_off[m + 1]].view(self.n_aos[m], self.n_aos[m]) for m in range(self.n_mol)]

    def split_rho(self, rho):
        return [rho[self.pt_off[m]:self.pt_off[m + 1]] for m in range(self.n_mol)]

    def eval(self, D, rho=True, vxc=True, out=None, stream=None):
        """One EXC evaluation of every molecule.  D: packed float64 CUDA tensor.  Returns packed rho,
        exc [n_mol] and packed Vxc (device tensors; the work is only enqueued)."""
        return self._eval(D, int(self.d_off[-1]), int(self.pt_off[-1]), rho, vxc, out, stream, (int(self.d_off[-1]),))


def xc_eval(xc, rho, sigma=None, rho_cut=0.0, stream=None):
    """The library's functional on device arrays (kldi_xc_eval): returns (f, v_rho, v_sigma)."""
    n = rho.numel()
    f = torch.empty_like(rho)
    vr = torch.empty_like(rho)
    vs = torch.empty_like(rho) if sigma is not None else None
    L.check(L.kldi_xc_eval(L.XC[xc], ctypes.c_void_p(rho.data_ptr()),
                           ctypes.c_void_p(sigma.data_ptr() if sigma is not None else 0), n, float(rho_cut),
                           ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(vr.data_ptr()),
                           ctypes.c_void_p(vs.data_ptr() if vs is not None else 0), _stream_handle(stream)),
            "kldi_xc_eval")
    return f, vr, vs


def overlap_order(basis, S):
    """kldi_overlap_order: (leaf order of the AOs, shell order) from the overlap matrix S (caller order)."""
    sl = np.ascontiguousarray(basis.shell_l, np.int32)
    n_ao = int(sum((int(l) + 1) * (int(l) + 2) // 2 for l in sl))
    S = np.ascontiguousarray(S, np.float64)
    if S.shape != (n_ao, n_ao):
        raise ValueError("S must be n_ao x n_ao")
    b = L.kldi_basis()
    b.n_shells = sl.shape[0]
    b.shell_l = sl.ctypes.data
    ao = np.empty(n_ao, np.int32)
    so = np.empty(sl.shape[0], np.int32)
    L.check(L.kldi_overlap_order(ctypes.byref(b), S.ctypes.data, ao.ctypes.data, so.ctypes.data), "kldi_overlap_order")
    return ao, so


class Mlp:
    """kldi_mlp_*: the functional surrogate (2-64-64-64-3 SiLU), trained and run by libkldi."""

    N_PARAMS = 8707

    def __init__(self, seed=0):
        self._h = ctypes.c_void_p()
        cfg = L.kldi_mlp_cfg(int(seed))
        L.check(L.kldi_mlp_create(ctypes.byref(cfg), ctypes.byref(self._h)), "kldi_mlp_create")

    def params(self, set_params=None):
        get = np.empty(self.N_PARAMS, np.float32)
        box = np.empty(4)
        tm = np.empty(3)
        ts = np.empty(3)
        sp = None
        if set_params is not None:
            sp = np.ascontiguousarray(set_params, np.float32)
        L.check(L.kldi_mlp_params(self._h, get.ctypes.data, sp.ctypes.data if sp is not None else None, box.ctypes.data,
                                  tm.ctypes.data, ts.ctypes.data), "kldi_mlp_params")
        return get, box, tm, ts

    def loss_grad(self, x, t, stream=None):
        """x: float32 CUDA [n, 2] features, t: float32 CUDA [n, 3] standardised targets."""
        g = np.empty(self.N_PARAMS, np.float32)
        loss = ctypes.c_double()
        L.check(L.kldi_mlp_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                     ctypes.byref(loss), g.ctypes.data, _stream_handle(stream)), "kldi_mlp_loss_grad")
        return loss.value, g

    def step(self, x, t, lr, stream=None):
        """One Adam step on the batch (x, t) (float32 CUDA [n, 2], [n, 3]); returns the loss before it."""
        loss = ctypes.c_double()
        L.check(L.kldi_mlp_step(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                float(lr), ctypes.byref(loss), _stream_handle(stream)), "kldi_mlp_step")
        return loss.value

    def step_static(self, x, t, lr, loss=None, stream=None):
        """kldi_mlp_step_static: the same step without device allocation (n <= 16384); the loss before
        the step goes to `loss` (a float64 CUDA tensor of one element) if given.  Does not synchronise."""
        L.check(L.kldi_mlp_step_static(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                       x.shape[0], float(lr), ctypes.c_void_p(loss.data_ptr() if loss is not None else 0),
                                       _stream_handle(stream)), "kldi_mlp_step_static")

    def train(self, rho, sigma, epochs=10, batch=65536, lr=2e-3, seed=1, xc="pbe", rho_min=1e-8, stream=None):
        cfg = L.kldi_train_cfg(int(epochs), int(batch), float(lr), int(seed), L.XC[xc], float(rho_min))
        losses = np.zeros(max(int(epochs), 1))
        L.check(L.kldi_mlp_train(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                                 rho.numel(), ctypes.byref(cfg), losses.ctypes.data, _stream_handle(stream)),
                "kldi_mlp_train")
        return losses[:epochs]

    def forward(self, rho, sigma, stream=None):
        f = torch.empty_like(rho)
        vr = torch.empty_like(rho)
        vs = torch.empty_like(rho)
        used = torch.empty(rho.numel(), dtype=torch.int32, device=rho.device)
        L.check(L.kldi_mlp_forward(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                                   rho.numel(), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(vr.data_ptr()),
                                   ctypes.c_void_p(vs.data_ptr()), ctypes.c_void_p(used.data_ptr()),
                                   _stream_handle(stream)), "kldi_mlp_forward")
        return f, vr, vs, used

    def close(self):
        if self._h:
            L.kldi_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
