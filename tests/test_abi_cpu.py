"""libkldi's C ABI without a GPU: exported symbols, defaults, and host-side validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_10363_amd", "libkldi.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_2605_10363_amd import build
        build.build()
    from paper_2605_10363_amd import _lib
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kldi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kldi_[a-z_]+)\s*\(", src)))


def test_every_declared_function_is_exported(L):
    names = declared_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_version_and_defaults(L):
    assert L.kldi_version() == 4
    o = L.kldi_opts()
    L.kldi_opts_default(ctypes.byref(o))
    assert o.t_b == 1e-10 and o.t_d == 1e-10 and o.rho_cut == 1e-14
    assert o.grid_block == 128 and o.ao_block == 32 and o.prec == 0 and o.xc == 1
    assert o.v_segment == 0 and o.chunk_tiles == 0 and o.schedule == 0


def _structs(L, p, **kw):
    keep = [np.ascontiguousarray(p.atom_xyz), p.basis.shell_atom.astype(np.int32), p.basis.shell_l.astype(np.int32),
            p.basis.prim_ptr.astype(np.int32), np.ascontiguousarray(p.basis.prim_exp),
            np.ascontiguousarray(p.basis.prim_coef), np.ascontiguousarray(p.grid.xyz),
            np.ascontiguousarray(p.grid.weight), p.grid.point_atom.astype(np.int32)]
    ax, sa, sl, pp, pe, pc, gx, gw, ga = keep
    b = L.kldi_basis(ax.shape[0], ax.ctypes.data, sl.shape[0], sa.ctypes.data, sl.ctypes.data, pp.ctypes.data,
                     pe.ctypes.data, pc.ctypes.data)
    g = L.kldi_grid(gw.shape[0], gx.ctypes.data, gw.ctypes.data, ga.ctypes.data)
    o = L.kldi_opts()
    L.kldi_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return b, g, o, keep


def _create(L, b, g, o):
    h = ctypes.c_void_p(123)
    st = L.kldi_plan_create(ctypes.byref(b) if b is not None else None, ctypes.byref(g) if g is not None else None,
                            ctypes.byref(o) if o is not None else None, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("bad", ["null_basis", "null_grid", "null_opts", "neg_tb", "nan_td", "bad_l", "bad_ptr",
                                 "neg_exp", "bad_atom", "bad_point_atom", "zero_points", "block_not_64",
                                 "bad_prec", "bad_xc", "nan_xyz", "bad_schedule", "neg_segment"])
def test_invalid_arguments_rejected_before_any_launch(L, bad):
    p = synth.tiny_problem(seed=2)
    b, g, o, keep = _structs(L, p)
    if bad == "null_basis":
        b = None
    elif bad == "null_grid":
        g = None
    elif bad == "null_opts":
        o = None
    elif bad == "neg_tb":
        o.t_b = -1.0
    elif bad == "nan_td":
        o.t_d = float("nan")
    elif bad == "bad_l":
        keep[2][0] = 3
    elif bad == "bad_ptr":
        keep[3][1] = keep[3][0]
    elif bad == "neg_exp":
        keep[4][0] = -0.5
    elif bad == "bad_atom":
        keep[1][0] = 99
    elif bad == "bad_point_atom":
        keep[8][3] = -1
    elif bad == "zero_points":
        g.n_points = 0
    elif bad == "block_not_64":
        o.grid_block = 100
    elif bad == "bad_prec":
        o.prec = 7
    elif bad == "bad_xc":
        o.xc = 42
    elif bad == "nan_xyz":
        keep[6][5, 1] = float("nan")
    elif bad == "bad_schedule":
        o.schedule = 5
    elif bad == "neg_segment":
        o.v_segment = -2
    st, h = _create(L, b, g, o)
    assert st == -1, (bad, st, L.kldi_last_error())
    assert h.value is None
    assert len(L.kldi_last_error()) > 0


@pytest.mark.parametrize("field,value", [("grid_block", 512), ("grid_block", 192), ("ao_block", 64)])
def test_unsupported_block_shapes(L, field, value):
    p = synth.tiny_problem(seed=2)
    b, g, o, keep = _structs(L, p, **{field: value})
    st, h = _create(L, b, g, o)
    assert st == -4
    assert h.value is None


def test_null_handles(L):
    assert L.kldi_plan_destroy(None) == 0
    assert L.kldi_eval(None, None, None, None, None, None) == -1
    assert L.kldi_plan_info(None, None) == -1
    assert L.kldi_eval_check(None, None, None) == -1
    assert L.kldi_plan_structure(None, None, None, None, None) == -1


def test_batch_arguments_rejected_before_any_launch(L):
    """kldi_batch_create validates every molecule (and n_mol) before touching the device."""
    ps = [synth.tiny_problem(seed=2), synth.tiny_problem(n_atoms=2, seed=3)]
    parts = [_structs(L, p) for p in ps]
    o = parts[0][2]
    B = (L.kldi_basis * 2)(parts[0][0], parts[1][0])
    G = (L.kldi_grid * 2)(parts[0][1], parts[1][1])
    h = ctypes.c_void_p(123)
    assert L.kldi_batch_create(0, B, G, ctypes.byref(o), None, ctypes.byref(h)) == -1
    assert h.value is None
    parts[1][3][8][0] = 7                       # molecule 1: a point of a missing atom
    G = (L.kldi_grid * 2)(parts[0][1], parts[1][1])
    h = ctypes.c_void_p(123)
    assert L.kldi_batch_create(2, B, G, ctypes.byref(o), None, ctypes.byref(h)) == -1
    assert h.value is None
    assert b"molecule 1" in L.kldi_last_error()
    assert L.kldi_batch_create(2, None, G, ctypes.byref(o), None, ctypes.byref(h)) == -1


def test_null_handles_of_batch_graph_and_tuning(L):
    assert L.kldi_batch_layout(None, None, None, None) == -1
    assert L.kldi_plan_graph(None, 1) == -1
    assert L.kldi_plan_autotune(None, None, 1, None, None) == -1
