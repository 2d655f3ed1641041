"""ctypes binding of libkldi (include/kldi.h): argument marshalling only.

Every step of the EXC evaluation runs inside libkldi's HIP kernels; this module converts Python
arguments to the C structs, passes device pointers of torch tensors and the current HIP stream, and
turns status codes into exceptions.  There is no fallback: if libkldi.so is missing, importing this
module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkldi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libkldi.so is not built (%s); run __graft_entry__.build() first" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

KLDI_OK = 0
STATUS = {0: "KLDI_OK", -1: "KLDI_E_ARG", -2: "KLDI_E_OOM", -3: "KLDI_E_HIP", -4: "KLDI_E_UNSUPPORTED",
          -5: "KLDI_E_STATE", -6: "KLDI_E_NONFINITE"}
XC = {"lda": 1, "pbe": 2, "pbe_x": 3, "mvs": 4, "mvs_x": 5}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 3, "bf16x6": 4}
SCHED = {"grid": 0, "queue": 1}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class kldi_basis(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("atom_xyz", ctypes.c_void_p), ("n_shells", ctypes.c_int32),
                ("shell_atom", ctypes.c_void_p), ("shell_l", ctypes.c_void_p), ("shell_prim_ptr", ctypes.c_void_p),
                ("prim_exp", ctypes.c_void_p), ("prim_coef", ctypes.c_void_p)]


class kldi_grid(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("point_atom", ctypes.c_void_p)]


class kldi_opts(ctypes.Structure):
    _fields_ = [("t_b", ctypes.c_double), ("t_d", ctypes.c_double), ("rho_cut", ctypes.c_double),
                ("grid_block", ctypes.c_int32), ("ao_block", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("xc", ctypes.c_int32), ("v_segment", ctypes.c_int32), ("chunk_tiles", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("shell_order", ctypes.c_void_p)]


class kldi_plan_info_t(ctypes.Structure):
    _fields_ = [("n_ao", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("n_points", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64), ("n_candidate_tiles", ctypes.c_int64),
                ("n_retained_tiles", ctypes.c_int64), ("retained_fraction", ctypes.c_double),
                ("max_tiles_per_block", ctypes.c_int32), ("v_segment", ctypes.c_int32),
                ("n_v_items", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64), ("n_grid_chunks", ctypes.c_int32),
                ("plan_ms", ctypes.c_double), ("n_mol", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("n_x_items", ctypes.c_int64)]


class kldi_tune_t(ctypes.Structure):
    _fields_ = [("v_segment", ctypes.c_int32), ("schedule", ctypes.c_int32), ("ms", ctypes.c_double),
                ("n_tried", ctypes.c_int32)]


class kldi_eval_stats_t(ctypes.Structure):
    _fields_ = [("n_pairs_x", ctypes.c_int64), ("n_pairs_v", ctypes.c_int64), ("gemm_flops", ctypes.c_double),
                ("nonfinite_d", ctypes.c_int32), ("n_points_mlp", ctypes.c_int64),
                ("n_pairs_v_diag", ctypes.c_int64)]


class kldi_mlp_cfg(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64)]


class kldi_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("xc", ctypes.c_int32), ("rho_min", ctypes.c_double)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


kldi_opts_default = _sig("kldi_opts_default", None, [ctypes.POINTER(kldi_opts)])
kldi_plan_create = _sig("kldi_plan_create", ctypes.c_int,
                        [ctypes.POINTER(kldi_basis), ctypes.POINTER(kldi_grid), ctypes.POINTER(kldi_opts),
                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)])
kldi_batch_create = _sig("kldi_batch_create", ctypes.c_int,
                         [ctypes.c_int32, ctypes.POINTER(kldi_basis), ctypes.POINTER(kldi_grid), ctypes.POINTER(kldi_opts),
                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)])
kldi_batch_layout = _sig("kldi_batch_layout", ctypes.c_int,
                         [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_plan_graph = _sig("kldi_plan_graph", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32])
kldi_plan_autotune = _sig("kldi_plan_autotune", ctypes.c_int,
                          [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(kldi_tune_t)])
kldi_plan_destroy = _sig("kldi_plan_destroy", ctypes.c_int, [ctypes.c_void_p])
kldi_plan_info = _sig("kldi_plan_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(kldi_plan_info_t)])
kldi_plan_structure = _sig("kldi_plan_structure", ctypes.c_int,
                           [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_eval = _sig("kldi_eval", ctypes.c_int,
                 [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_eval_check = _sig("kldi_eval_check", ctypes.c_int,
                       [ctypes.c_void_p, ctypes.POINTER(kldi_eval_stats_t), ctypes.c_void_p])
kldi_plan_timing = _sig("kldi_plan_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32])
kldi_eval_timing = _sig("kldi_eval_timing", ctypes.c_int,
                        [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)])
kldi_eval_grid = _sig("kldi_eval_grid", ctypes.c_int,
                      [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_xc_eval = _sig("kldi_xc_eval", ctypes.c_int,
                    [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_create = _sig("kldi_mlp_create", ctypes.c_int, [ctypes.POINTER(kldi_mlp_cfg), ctypes.POINTER(ctypes.c_void_p)])
kldi_mlp_destroy = _sig("kldi_mlp_destroy", ctypes.c_int, [ctypes.c_void_p])
kldi_mlp_train = _sig("kldi_mlp_train", ctypes.c_int,
                      [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(kldi_train_cfg),
                       ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_forward = _sig("kldi_mlp_forward", ctypes.c_int,
                        [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_loss_grad = _sig("kldi_mlp_loss_grad", ctypes.c_int,
                          [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_step = _sig("kldi_mlp_step", ctypes.c_int,
                     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                      ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_step_static = _sig("kldi_mlp_step_static", ctypes.c_int,
                            [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_void_p, ctypes.c_void_p])
kldi_eval_grad = _sig("kldi_eval_grad", ctypes.c_int,
                      [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_overlap_order = _sig("kldi_overlap_order", ctypes.c_int,
                          [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p])
kldi_mlp_params = _sig("kldi_mlp_params", ctypes.c_int,
                       [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p])
kldi_plan_attach_mlp = _sig("kldi_plan_attach_mlp", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p])
kldi_last_error = _sig("kldi_last_error", ctypes.c_char_p, [])
kldi_version = _sig("kldi_version", ctypes.c_int32, [])

EXPORTS = sorted(["kldi_opts_default", "kldi_plan_create", "kldi_batch_create", "kldi_batch_layout",
                  "kldi_plan_graph", "kldi_plan_autotune", "kldi_plan_destroy", "kldi_plan_info",
                  "kldi_plan_structure", "kldi_eval", "kldi_eval_check", "kldi_plan_timing", "kldi_eval_timing",
                  "kldi_eval_grid", "kldi_xc_eval", "kldi_mlp_create", "kldi_mlp_destroy", "kldi_mlp_train",
                  "kldi_mlp_forward", "kldi_mlp_loss_grad", "kldi_mlp_step", "kldi_mlp_step_static", "kldi_mlp_params", "kldi_overlap_order", "kldi_eval_grad", "kldi_plan_attach_mlp",
                  "kldi_last_error", "kldi_version"])
STAGES = ["dprep", "basis", "xgemm", "xfunc", "vgemm", "vfinal"]


class KldiError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = kldi_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%s)" % (where, STATUS.get(status, status), msg))


def check(status, where):
    if status != KLDI_OK:
        raise KldiError(status, where)
