"""ctypes binding of libdnnmg.so: same entry-point names as include/dnnmg.h.

Argument marshalling only: each wrapper checks that the torch tensors it is
given are on the GPU, contiguous and of the expected dtype and size, then
passes raw device pointers and the current HIP stream to the library.  There
is no fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdnnmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(hipcc for gfx950). There is no CPU fallback.")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
F32, BF16, FP8_E4M3 = 0, 1, 2
N_IN, N_OUT, IN_PAD, OUT_PAD = 165, 81, 192, 96

c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p
c_f = ctypes.c_float
c_sz = ctypes.c_size_t


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("len", ctypes.c_double * 3),
                ("periodic_mask", ctypes.c_uint32), ("dirichlet_mask", ctypes.c_uint32)]

    @classmethod
    def of(cls, spec) -> "Box":
        if isinstance(spec, Box):
            return spec
        b = cls()
        for a in range(3):
            b.n[a] = int(spec.n[a])
            b.len[a] = float(spec.len[a])
        b.periodic_mask = int(spec.periodic_mask)
        b.dirichlet_mask = int(spec.dirichlet_mask)
        return b


class NS(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("dt", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("delta0", ctypes.c_double)]

    @classmethod
    def of(cls, p) -> "NS":
        if isinstance(p, NS):
            return p
        return cls(float(p.nu), float(p.dt), float(p.alpha0), float(p.delta0))


class MLP(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("W", c_vp * 3), ("b", c_vp * 3),
                ("w_scale", c_f * 3), ("a_scale", c_f * 3)]


class Feat(ctypes.Structure):
    _fields_ = [("shift", c_vp), ("inv_scale", c_vp)]


DEEP_MAX_DEPTH = 16  # DNNMG_DEEP_MAX_DEPTH of include/dnnmg.h


class DeepNetDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("dtype", ctypes.c_int32), ("W", c_vp * (DEEP_MAX_DEPTH + 1)),
                ("b", c_vp * (DEEP_MAX_DEPTH + 1))]


class CoarseOpts(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("krylov_dim", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("pre_sweeps", ctypes.c_int32), ("post_sweeps", ctypes.c_int32),
                ("coarsest_sweeps", ctypes.c_int32), ("omega", ctypes.c_double), ("fd_eta", ctypes.c_double)]


COARSE_MAX_KRYLOV = 16  # DNNMG_COARSE_MAX_KRYLOV of include/dnnmg.h


def _sig(name, argtypes, restype=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


_P = ctypes.POINTER
_sig("dnnmg_version", [])
_sig("dnnmg_last_error", [], ctypes.c_char_p)
_sig("dnnmg_box_sizes", [_P(Box), _P(c_i64), _P(c_i64), _P(c_i64)])
_sig("dnnmg_patch_dofmap", [_P(Box), c_vp, c_vp, c_vp])
_sig("dnnmg_prolong", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_residual_workspace", [_P(Box)], c_sz)
_sig("dnnmg_residual", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_residual_b", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_residual_b_noalloc", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_fallback_b", [_P(Box), _P(NS), c_vp, c_vp, c_vp, ctypes.c_double, ctypes.c_int, c_f, c_vp, c_vp, c_vp,
                          c_sz, c_vp])
_sig("dnnmg_rhs", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_residual_rhs_b", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_rhs_if", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_prolong_residual", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_prolong_residual_b", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_restrict", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_patch_gather", [_P(Box), c_vp, c_vp, _P(Feat), ctypes.c_int, c_f, c_vp, c_i64, c_vp])
_sig("dnnmg_mlp_packed_bytes", [ctypes.c_int, ctypes.c_int, ctypes.c_int], c_sz)
_sig("dnnmg_mlp_pack", [ctypes.c_int, ctypes.c_int, ctypes.c_int, c_vp, c_f, c_vp, c_vp])
_sig("dnnmg_patch_forward", [_P(MLP), c_i64, c_vp, c_i64, c_vp, c_vp, c_vp])
_sig("dnnmg_patch_forward_tiles", [_P(MLP), c_i64, c_vp, c_i64, c_vp, c_vp, ctypes.c_int, ctypes.c_int, c_vp])
_sig("dnnmg_patch_saved_bytes", [_P(MLP), c_i64], c_sz)
_sig("dnnmg_scatter_avg", [_P(Box), c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_scatter_avg_form", [_P(Box), c_vp, c_vp, c_vp, ctypes.c_int, c_vp])
_sig("dnnmg_norm2_workspace", [], c_sz)
_sig("dnnmg_norm2_f64", [c_i64, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_norm2_pair_f64", [c_i64, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_mse_grad", [c_i64, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_mse_grad_loss", [c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_patch_backward_workspace", [_P(MLP), c_i64], c_sz)
_sig("dnnmg_patch_backward", [_P(MLP), c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp * 3, c_vp * 3,
                              c_vp, c_sz, c_vp])
_sig("dnnmg_vanka_workspace", [_P(Box)], c_sz)
_sig("dnnmg_vanka_sweeps", [_P(Box), _P(NS), c_vp, c_vp, c_vp, ctypes.c_int, c_f, ctypes.c_int, c_vp, c_sz,
                            c_vp])
_sig("dnnmg_fallback_workspace", [_P(Box)], c_sz)
_sig("dnnmg_fallback", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, ctypes.c_double, ctypes.c_int, c_f, c_vp,
                        c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_patch_gather_forward", [_P(Box), _P(MLP), c_vp, c_vp, _P(Feat), c_vp, c_vp])
_sig("dnnmg_plan_workspace", [c_vp, ctypes.c_int], c_sz)
_sig("dnnmg_plan_create", [c_vp, ctypes.c_int, _P(NS), c_vp, c_sz, _P(c_vp), c_vp])
_sig("dnnmg_plan_destroy", [c_vp])
_sig("dnnmg_plan_sizes", [c_vp, _P(c_i64), _P(c_i64), _P(c_i64)])
_sig("dnnmg_plan_choice", [c_vp, _P(ctypes.c_int), _P(ctypes.c_int)])
_sig("dnnmg_plan_scatter_form", [c_vp, _P(ctypes.c_int)])
_sig("dnnmg_plan_set_scatter_form", [c_vp, ctypes.c_int])
_sig("dnnmg_batch_step", [c_vp, _P(MLP), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_batch_step_b", [c_vp, _P(MLP), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_batch_rhs", [c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_plan_autotune", [c_vp, _P(MLP), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                             ctypes.c_int, c_vp])
_sig("dnnmg_mlp_prepare", [ctypes.c_int, ctypes.c_int, c_vp * 3, c_vp * 3, c_vp * 3, c_vp, c_sz, _P(MLP), c_vp])
_sig("dnnmg_mlp_packed_bytes_io", [ctypes.c_int] * 5, c_sz)
_sig("dnnmg_mlp_pack_io", [ctypes.c_int] * 5 + [c_vp, c_f, c_vp, c_vp])
_sig("dnnmg_mlp_prepare_io", [ctypes.c_int] * 4 + [c_vp * 3, c_vp * 3, c_vp * 3, c_vp, c_sz, _P(MLP), c_vp])
_sig("dnnmg_level_sizes", [_P(Box), ctypes.c_int, _P(c_i64), _P(c_i64), _P(c_i64)])
_sig("dnnmg_patch_dofmap_levels", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_prolong_levels", [_P(Box), ctypes.c_int, ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_prolong_residual_b_levels_workspace", [_P(Box), ctypes.c_int], c_sz)
_sig("dnnmg_prolong_residual_b_levels", [_P(Box), ctypes.c_int, _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_restrict_levels", [_P(Box), ctypes.c_int, ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_patch_gather_levels", [_P(Box), ctypes.c_int, c_vp, c_vp, _P(Feat), ctypes.c_int, c_vp, c_i64, c_vp])
_sig("dnnmg_scatter_avg_levels", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp, c_vp])
_sig("dnnmg_deepnet_widths", [ctypes.c_int] * 3 + [_P(ctypes.c_int)] * 3)
_sig("dnnmg_deepnet_packed_bytes", [ctypes.c_int] * 6, c_sz)
_sig("dnnmg_deepnet_prepare", [ctypes.c_int] * 5 + [c_vp] * 8 + [c_sz, _P(DeepNetDesc), c_vp])
_sig("dnnmg_deepnet_forward", [_P(DeepNetDesc), c_i64, c_vp, c_i64, c_vp, c_vp])
_sig("dnnmg_patch_gather_paper", [_P(Box), ctypes.c_int, c_vp, c_vp, _P(Feat), ctypes.c_int, c_vp, c_i64, c_vp])
_sig("dnnmg_graph_capture_begin", [c_vp])
_sig("dnnmg_graph_capture_end", [c_vp, _P(c_vp)])
_sig("dnnmg_graph_replay", [c_vp, c_vp])
_sig("dnnmg_graph_destroy", [c_vp])
_sig("dnnmg_adamw_step", [c_i64, c_vp, c_vp, c_vp, c_vp, c_f, c_f, c_f, c_f, c_f, c_i64, c_vp])
_sig("dnnmg_coarse_levels", [_P(Box), _P(CoarseOpts)])
_sig("dnnmg_coarse_workspace", [_P(Box), _P(CoarseOpts)], c_sz)
_sig("dnnmg_coarse_solve", [_P(Box), _P(NS), c_vp, c_vp, _P(CoarseOpts), c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_coarse_jv", [_P(Box), _P(NS), c_vp, c_vp, c_vp, _P(CoarseOpts), c_vp, c_sz, c_vp])
_sig("dnnmg_coarse_vcycle", [_P(Box), _P(NS), c_vp, c_vp, c_vp, _P(CoarseOpts), c_vp, c_sz, c_vp])
_sig("dnnmg_q2_workspace", [_P(Box)], c_sz)
_sig("dnnmg_q2_residual_b", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_q2_rhs", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_q2_residual_rhs", [_P(Box), _P(NS), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("dnnmg_q2_prolong", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_q2_restrict", [_P(Box), ctypes.c_int, c_vp, c_vp, c_vp])
_sig("dnnmg_q2_patch_features", [_P(Box), c_vp, c_vp, c_vp])
_sig("dnnmg_patch_gather_geom", [_P(Box), c_vp, c_vp, c_vp, _P(Feat), ctypes.c_int, c_f, c_vp, c_i64, c_vp])
_sig("dnnmg_patch_gather_forward_geom", [_P(Box), _P(MLP), c_vp, c_vp, c_vp, _P(Feat), c_vp, c_vp])
_sig("dnnmg_q2_patch_features24", [_P(Box), c_vp, c_vp, c_vp])
_sig("dnnmg_patch_gather_paper_geom", [_P(Box), c_vp, c_vp, c_vp, _P(Feat), ctypes.c_int, c_vp, c_i64, c_vp])

EXPORTS = [
    "dnnmg_version", "dnnmg_last_error", "dnnmg_box_sizes", "dnnmg_patch_dofmap", "dnnmg_prolong",
    "dnnmg_residual_workspace", "dnnmg_residual", "dnnmg_rhs", "dnnmg_restrict",
    "dnnmg_patch_gather", "dnnmg_mlp_packed_bytes", "dnnmg_mlp_pack", "dnnmg_patch_forward",
    "dnnmg_patch_forward_tiles", "dnnmg_prolong_residual", "dnnmg_prolong_residual_b",
    "dnnmg_residual_b", "dnnmg_residual_b_noalloc", "dnnmg_fallback_b", "dnnmg_residual_rhs_b", "dnnmg_rhs_if",
    "dnnmg_patch_saved_bytes", "dnnmg_scatter_avg", "dnnmg_scatter_avg_form", "dnnmg_norm2_workspace", "dnnmg_norm2_f64",
    "dnnmg_mse_grad", "dnnmg_mse_grad_loss", "dnnmg_patch_backward_workspace", "dnnmg_patch_backward", "dnnmg_adamw_step",
    "dnnmg_vanka_workspace", "dnnmg_vanka_sweeps", "dnnmg_fallback_workspace", "dnnmg_fallback",
    "dnnmg_patch_gather_forward", "dnnmg_plan_workspace", "dnnmg_plan_create", "dnnmg_plan_destroy",
    "dnnmg_plan_sizes", "dnnmg_plan_choice", "dnnmg_plan_scatter_form", "dnnmg_plan_set_scatter_form", "dnnmg_batch_step", "dnnmg_plan_autotune",
    "dnnmg_batch_step_b", "dnnmg_batch_rhs", "dnnmg_norm2_pair_f64", "dnnmg_mlp_prepare",
    "dnnmg_graph_capture_begin", "dnnmg_graph_capture_end", "dnnmg_graph_replay", "dnnmg_graph_destroy",
    "dnnmg_mlp_packed_bytes_io", "dnnmg_mlp_pack_io", "dnnmg_mlp_prepare_io", "dnnmg_level_sizes",
    "dnnmg_patch_dofmap_levels", "dnnmg_prolong_levels", "dnnmg_prolong_residual_b_levels_workspace",
    "dnnmg_prolong_residual_b_levels", "dnnmg_restrict_levels", "dnnmg_patch_gather_levels",
    "dnnmg_scatter_avg_levels", "dnnmg_deepnet_widths", "dnnmg_deepnet_packed_bytes", "dnnmg_deepnet_prepare",
    "dnnmg_deepnet_forward", "dnnmg_patch_gather_paper", "dnnmg_coarse_levels", "dnnmg_coarse_workspace",
    "dnnmg_coarse_solve", "dnnmg_coarse_jv", "dnnmg_coarse_vcycle", "dnnmg_q2_residual_b", "dnnmg_q2_rhs", "dnnmg_q2_workspace", "dnnmg_q2_residual_rhs",
    "dnnmg_q2_prolong", "dnnmg_q2_restrict", "dnnmg_q2_patch_features", "dnnmg_patch_gather_geom",
    "dnnmg_patch_gather_forward_geom", "dnnmg_q2_patch_features24", "dnnmg_patch_gather_paper_geom",
]

# network widths per prediction depth J (levels): inputs, outputs, padded input row
LEVEL_IO = {1: (165, 81, 192), 2: (753, 375, 768)}


class DnnmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdnnmg error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise DnnmgError(rc, _lib.dnnmg_last_error().decode())


def lib():
    return _lib


def _stream(stream):
    if stream is None:
        return c_vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_vp(stream.cuda_stream)
    return c_vp(int(stream))


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return c_vp(t.data_ptr())


def box_sizes(box):
    b = Box.of(box)
    nf, nc, np_ = c_i64(), c_i64(), c_i64()
    _check(_lib.dnnmg_box_sizes(ctypes.byref(b), ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(np_)))
    return nf.value, nc.value, np_.value


def dnnmg_patch_dofmap(box, dofmap=None, mult=None, stream=None):
    b = Box.of(box)
    nf, _, npch = box_sizes(b)
    _check(_lib.dnnmg_patch_dofmap(ctypes.byref(b), _ptr(dofmap, torch.int32, npch * 27, "map"),
                                   _ptr(mult, torch.uint8, nf, "mult"), _stream(stream)))


def dnnmg_prolong(box, xc, xf, ncomp=4, stream=None):
    b = Box.of(box)
    nf, nc, _ = box_sizes(b)
    _check(_lib.dnnmg_prolong(ctypes.byref(b), ncomp, _ptr(xc, torch.float64, ncomp * nc, "xc"),
                              _ptr(xf, torch.float32, ncomp * nf, "xf"), _stream(stream)))


def residual_workspace_bytes(box) -> int:
    return int(_lib.dnnmg_residual_workspace(ctypes.byref(Box.of(box))))


def dnnmg_residual_b(box, ns, x, b, r, ws, stream=None):
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    _check(_lib.dnnmg_residual_b(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(x, torch.float32, 4 * nf, "x"),
                                 _ptr(b, torch.float32, 4 * nf, "b"), _ptr(r, torch.float32, 4 * nf, "r"),
                                 _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_residual_rhs_b(box, ns, x, b, r, ws, b_save=None, stream=None):
    """r = b - A(x) and b <- Rhs(x's velocity) in one pass; b_save (optional)
    receives b as it was."""
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    _check(_lib.dnnmg_residual_rhs_b(ctypes.byref(bx), ctypes.byref(NS.of(ns)),
                                     _ptr(x, torch.float32, 4 * nf, "x"), _ptr(b, torch.float32, 4 * nf, "b"),
                                     _ptr(r, torch.float32, 4 * nf, "r"), _ptr(b_save, torch.float32, 4 * nf, "b_save"),
                                     _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_rhs_if(box, ns, v, b_out, flag, fmid=None, stream=None):
    """dnnmg_rhs when the device int *flag is nonzero at run time."""
    b = Box.of(box)
    nf, _, _ = box_sizes(b)
    _check(_lib.dnnmg_rhs_if(ctypes.byref(b), ctypes.byref(NS.of(ns)), _ptr(v, torch.float32, 3 * nf, "v"),
                             _ptr(fmid, torch.float32, 3 * nf, "fmid"), _ptr(b_out, torch.float32, 4 * nf, "b"),
                             _ptr(flag, torch.int32, 1, "flag"), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 33 << 20  # DNNMG_NOALLOC_SCRATCH_BYTES of include/dnnmg.h


def dnnmg_residual_b_noalloc(box, ns, x, b, r, stream=None):
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    _check(_lib.dnnmg_residual_b_noalloc(ctypes.byref(bx), ctypes.byref(NS.of(ns)),
                                         _ptr(x, torch.float32, 4 * nf, "x"), _ptr(b, torch.float32, 4 * nf, "b"),
                                         _ptr(r, torch.float32, 4 * nf, "r"), _stream(stream)))


def dnnmg_residual(box, ns, x, vprev, r, ws, fmid=None, stream=None):
    b = Box.of(box)
    nf, _, _ = box_sizes(b)
    _check(_lib.dnnmg_residual(ctypes.byref(b), ctypes.byref(NS.of(ns)),
                               _ptr(x, torch.float32, 4 * nf, "x"),
                               _ptr(vprev, torch.float32, 3 * nf, "vprev"),
                               _ptr(fmid, torch.float32, 3 * nf, "fmid"),
                               _ptr(r, torch.float32, 4 * nf, "r"),
                               _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(),
                               _stream(stream)))


def dnnmg_rhs(box, ns, v, b_out, fmid=None, stream=None):
    b = Box.of(box)
    nf, _, _ = box_sizes(b)
    _check(_lib.dnnmg_rhs(ctypes.byref(b), ctypes.byref(NS.of(ns)), _ptr(v, torch.float32, 3 * nf, "v"),
                          _ptr(fmid, torch.float32, 3 * nf, "fmid"),
                          _ptr(b_out, torch.float32, 4 * nf, "b"), _stream(stream)))


def dnnmg_prolong_residual(box, ns, xc, vprev, xt, r, fmid=None, stream=None):
    b = Box.of(box)
    nf, nc, _ = box_sizes(b)
    _check(_lib.dnnmg_prolong_residual(ctypes.byref(b), ctypes.byref(NS.of(ns)), _ptr(xc, torch.float64, 4 * nc, "xc"),
                                       _ptr(vprev, torch.float32, 3 * nf, "vprev"),
                                       _ptr(fmid, torch.float32, 3 * nf, "fmid"), _ptr(xt, torch.float32, 4 * nf, "xt"),
                                       _ptr(r, torch.float32, 4 * nf, "r"), _stream(stream)))


def dnnmg_prolong_residual_b(box, ns, xc, b, xt, r, stream=None):
    bx = Box.of(box)
    nf, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_prolong_residual_b(ctypes.byref(bx), ctypes.byref(NS.of(ns)),
                                         _ptr(xc, torch.float64, 4 * nc, "xc"), _ptr(b, torch.float32, 4 * nf, "b"),
                                         _ptr(xt, torch.float32, 4 * nf, "xt"), _ptr(r, torch.float32, 4 * nf, "r"),
                                         _stream(stream)))


def dnnmg_restrict(box, bf, bc, ncomp=4, stream=None):
    b = Box.of(box)
    nf, nc, _ = box_sizes(b)
    _check(_lib.dnnmg_restrict(ctypes.byref(b), ncomp, _ptr(bf, torch.float32, ncomp * nf, "bf"),
                               _ptr(bc, torch.float64, ncomp * nc, "bc"), _stream(stream)))


_DT_TORCH = {F32: torch.float32, BF16: torch.bfloat16, FP8_E4M3: torch.uint8}


def dnnmg_patch_gather(box, x, r, X, dtype, ldx, shift=None, inv_scale=None, x_scale=1.0, stream=None):
    b = Box.of(box)
    nf, _, npch = box_sizes(b)
    feat = Feat(None if shift is None else _ptr(shift, torch.float32, 165, "shift"),
                None if inv_scale is None else _ptr(inv_scale, torch.float32, 165, "inv_scale"))
    if X.numel() * X.element_size() < npch * ldx * {F32: 4, BF16: 2, FP8_E4M3: 1}[dtype]:
        raise ValueError("X too small")
    _check(_lib.dnnmg_patch_gather(ctypes.byref(b), _ptr(x, torch.float32, 3 * nf, "x"),
                                   _ptr(r, torch.float32, 3 * nf, "r"), ctypes.byref(feat), dtype,
                                   float(x_scale), _ptr(X, None, None, "X"), ldx, _stream(stream)))


def packed_bytes(dtype, hidden, layer, n_in=N_IN, n_out=N_OUT) -> int:
    return int(_lib.dnnmg_mlp_packed_bytes_io(dtype, n_in, hidden, n_out, layer))


def dnnmg_mlp_pack(dtype, hidden, layer, W, Wp, w_scale=1.0, stream=None):
    if Wp.numel() * Wp.element_size() < packed_bytes(dtype, hidden, layer):
        raise ValueError("packed buffer too small")
    _check(_lib.dnnmg_mlp_pack(dtype, hidden, layer, _ptr(W, torch.float32, None, "W"), float(w_scale),
                               _ptr(Wp, None, None, "Wp"), _stream(stream)))


def make_mlp(dtype, hidden, Wp, bias, w_scale=(1.0, 1.0, 1.0), a_scale=(1.0, 1.0, 1.0)) -> MLP:
    net = MLP()
    net.n_in, net.hidden, net.n_out, net.dtype = N_IN, hidden, N_OUT, dtype
    for l in range(3):
        net.W[l] = Wp[l].data_ptr()
        net.b[l] = bias[l].data_ptr()
        net.w_scale[l] = float(w_scale[l])
        net.a_scale[l] = float(a_scale[l])
    return net


def level_sizes(box, levels):
    """(n_fine on level L + J, n_coarse, n_patches) of the J-level prediction."""
    b = Box.of(box)
    nf, nc, np_ = c_i64(), c_i64(), c_i64()
    _check(_lib.dnnmg_level_sizes(ctypes.byref(b), int(levels), ctypes.byref(nf), ctypes.byref(nc),
                                  ctypes.byref(np_)))
    return nf.value, nc.value, np_.value


def level_box(box, levels) -> Box:
    """The box whose own fine mesh is level L + J (n doubled J - 1 times)."""
    b = Box.of(box)
    out = Box()
    for a in range(3):
        out.n[a] = int(b.n[a]) << (int(levels) - 1)
        out.len[a] = b.len[a]
    out.periodic_mask, out.dirichlet_mask = b.periodic_mask, b.dirichlet_mask
    return out


def dnnmg_patch_dofmap_levels(box, levels, dofmap=None, mult=None, stream=None):
    b = Box.of(box)
    nf, _, npch = level_sizes(b, levels)
    nodes = ((1 << int(levels)) + 1) ** 3
    _check(_lib.dnnmg_patch_dofmap_levels(ctypes.byref(b), int(levels), _ptr(dofmap, torch.int32, npch * nodes, "map"),
                                          _ptr(mult, torch.uint8, nf, "mult"), _stream(stream)))


def dnnmg_prolong_levels(box, levels, xc, xf, ncomp=4, stream=None):
    b = Box.of(box)
    nf, nc, _ = level_sizes(b, levels)
    _check(_lib.dnnmg_prolong_levels(ctypes.byref(b), int(levels), ncomp, _ptr(xc, torch.float64, ncomp * nc, "xc"),
                                     _ptr(xf, torch.float32, ncomp * nf, "xf"), _stream(stream)))


def prolong_residual_b_levels_workspace_bytes(box, levels):
    return int(_lib.dnnmg_prolong_residual_b_levels_workspace(ctypes.byref(Box.of(box)), int(levels)))


def dnnmg_prolong_residual_b_levels(box, levels, ns, xc, b, xt, r, ws=None, stream=None):
    bx = Box.of(box)
    nf, nc, _ = level_sizes(bx, levels)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.dnnmg_prolong_residual_b_levels(ctypes.byref(bx), int(levels), ctypes.byref(NS.of(ns)),
                                                _ptr(xc, torch.float64, 4 * nc, "xc"),
                                                _ptr(b, torch.float32, 4 * nf, "b"),
                                                _ptr(xt, torch.float32, 4 * nf, "xt"),
                                                _ptr(r, torch.float32, 4 * nf, "r"),
                                                None if ws is None else _ptr(ws), nbytes, _stream(stream)))


def dnnmg_restrict_levels(box, levels, bf, bc, ncomp=4, stream=None):
    b = Box.of(box)
    nf, nc, _ = level_sizes(b, levels)
    _check(_lib.dnnmg_restrict_levels(ctypes.byref(b), int(levels), ncomp, _ptr(bf, torch.float32, ncomp * nf, "bf"),
                                      _ptr(bc, torch.float64, ncomp * nc, "bc"), _stream(stream)))


def dnnmg_patch_gather_levels(box, levels, x, r, X, dtype, ldx, shift=None, inv_scale=None, stream=None):
    b = Box.of(box)
    nf, _, npch = level_sizes(b, levels)
    nin = LEVEL_IO[int(levels)][0]
    feat = Feat(_ptr(shift, torch.float32, nin, "shift"), _ptr(inv_scale, torch.float32, nin, "inv_scale"))
    if X.numel() * X.element_size() < npch * ldx * {F32: 4, BF16: 2}[dtype]:
        raise ValueError("X too small")
    _check(_lib.dnnmg_patch_gather_levels(ctypes.byref(b), int(levels), _ptr(x, torch.float32, 3 * nf, "x"),
                                          _ptr(r, torch.float32, 3 * nf, "r"), ctypes.byref(feat), int(dtype),
                                          _ptr(X, None, None, "X"), int(ldx), _stream(stream)))


def dnnmg_scatter_avg_levels(box, levels, Y, d, vbase=None, stream=None):
    b = Box.of(box)
    nf, _, npch = level_sizes(b, levels)
    nout = 3 * ((1 << int(levels)) + 1) ** 3
    _check(_lib.dnnmg_scatter_avg_levels(ctypes.byref(b), int(levels), _ptr(Y, torch.float32, npch * nout, "Y"),
                                         _ptr(vbase, torch.float32, 4 * nf, "vbase"),
                                         _ptr(d, torch.float32, (4 if vbase is not None else 3) * nf, "d"),
                                         _stream(stream)))


def deepnet_widths(n_in, hidden, n_out):
    ip, hp, op = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.dnnmg_deepnet_widths(n_in, hidden, n_out, ctypes.byref(ip), ctypes.byref(hp), ctypes.byref(op)))
    return ip.value, hp.value, op.value


class DeepNet:
    """The paper's network packed for the kernels (dnnmg_deepnet_prepare): owns
    the FP32 parameters, the packed layers and folded biases (device)."""

    def __init__(self, dtype, Ws, gammas, betas, means, stds, device="cuda:0"):
        dev = torch.device(device)
        t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).contiguous().to(dev)
        self.dtype = int(dtype)
        self.depth = len(Ws) - 1
        self.n_in, self.hidden = np.shape(Ws[0])
        self.n_out = np.shape(Ws[-1])[1]
        self.in_pad, self.hidden_pad, self.out_pad = deepnet_widths(self.n_in, self.hidden, self.n_out)
        self.W = [t(w) for w in Ws]
        self.stats = [[t(x) for x in xs] for xs in (gammas, betas, means, stds)]
        self.Wp = [torch.zeros(int(_lib.dnnmg_deepnet_packed_bytes(self.dtype, self.n_in, self.hidden, self.n_out,
                                                                    self.depth, l)), dtype=torch.uint8, device=dev)
                   for l in range(self.depth + 1)]
        self.bias = [torch.zeros(self.hidden_pad if l < self.depth else self.out_pad, dtype=torch.float32, device=dev)
                     for l in range(self.depth + 1)]
        self._ws = torch.zeros(4 * self.hidden_pad, dtype=torch.uint8, device=dev)
        self.net = DeepNetDesc()
        arr = lambda xs: (c_vp * (self.depth + 1))(*[x.data_ptr() for x in xs])
        st = [(c_vp * self.depth)(*[x.data_ptr() for x in xs]) for xs in self.stats]
        _check(_lib.dnnmg_deepnet_prepare(self.dtype, self.n_in, self.hidden, self.n_out, self.depth, arr(self.W),
                                          st[0], st[1], st[2], st[3], arr(self.Wp), arr(self.bias), _ptr(self._ws),
                                          self._ws.numel(), ctypes.byref(self.net), _stream(None)))


def dnnmg_deepnet_forward(net: DeepNet, n, X, ldx, Y, stream=None):
    _check(_lib.dnnmg_deepnet_forward(ctypes.byref(net.net), int(n), _ptr(X, None, None, "X"), int(ldx),
                                      _ptr(Y, torch.float32, n * net.n_out, "Y"), _stream(stream)))


def dnnmg_patch_gather_paper(box, levels, x, r, X, dtype, ldx, shift=None, inv_scale=None, stream=None):
    b = Box.of(box)
    nf, _, npch = level_sizes(b, levels)
    nin = 240 if int(levels) == 1 else 1024
    feat = Feat(_ptr(shift, torch.float32, nin, "shift"), _ptr(inv_scale, torch.float32, nin, "inv_scale"))
    if X.numel() * X.element_size() < npch * ldx * {F32: 4, BF16: 2}[dtype]:
        raise ValueError("X too small")
    _check(_lib.dnnmg_patch_gather_paper(ctypes.byref(b), int(levels), _ptr(x, torch.float32, 4 * nf, "x"),
                                         _ptr(r, torch.float32, 4 * nf, "r"), ctypes.byref(feat), int(dtype),
                                         _ptr(X, None, None, "X"), int(ldx), _stream(stream)))


class PreparedMLP:
    """A network packed for the kernels by dnnmg_mlp_prepare: owns the packed
    weights and biases (device) and the filled dnnmg_mlp description."""

    def __init__(self, dtype, hidden, W32, bias, device, n_in=N_IN, n_out=N_OUT):
        self.dtype, self.hidden, self.n_in, self.n_out = int(dtype), int(hidden), int(n_in), int(n_out)
        self.W32 = [w.contiguous() for w in W32]
        self.bias = [b.contiguous() for b in bias]
        self.Wp = [torch.zeros(packed_bytes(dtype, hidden, l, n_in, n_out), dtype=torch.uint8, device=device)
                   for l in range(3)]
        self._ws = torch.zeros(256, dtype=torch.uint8, device=device)
        self.net = MLP()
        for l, (w, n) in enumerate(((n_in, hidden), (hidden, hidden), (hidden, n_out))):
            _ptr(self.W32[l], torch.float32, w * n, f"W{l + 1}")
            _ptr(self.bias[l], torch.float32, n, f"b{l + 1}")
        self.prepare()

    def prepare(self, stream=None):
        """(Re)packs from the FP32 weights (setup call: synchronises)."""
        W = (c_vp * 3)(*[w.data_ptr() for w in self.W32])
        B = (c_vp * 3)(*[b.data_ptr() for b in self.bias])
        P = (c_vp * 3)(*[w.data_ptr() for w in self.Wp])
        _check(_lib.dnnmg_mlp_prepare_io(self.dtype, self.n_in, self.hidden, self.n_out, W, B, P, _ptr(self._ws),
                                         self._ws.numel(), ctypes.byref(self.net), _stream(stream)))
        return self.net


def mlp_prepare(dtype, hidden, W32, bias, device="cuda:0", n_in=N_IN, n_out=N_OUT) -> PreparedMLP:
    return PreparedMLP(dtype, hidden, W32, bias, torch.device(device), n_in, n_out)


class Graph:
    """Executable HIP graph of the library calls made inside `capture()`
    (dnnmg_graph_capture_begin / _end); replay() launches it."""

    def __init__(self):
        self.handle = None

    def begin(self, stream):
        _check(_lib.dnnmg_graph_capture_begin(_stream(stream)))

    def end(self, stream):
        h = c_vp()
        _check(_lib.dnnmg_graph_capture_end(_stream(stream), ctypes.byref(h)))
        self.handle = h

    def replay(self, stream=None):
        if self.handle is None:
            raise RuntimeError("graph not captured")
        _check(_lib.dnnmg_graph_replay(self.handle, _stream(stream)))

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.dnnmg_graph_destroy(self.handle)
            self.handle = None


def capture_graph(fn, device="cuda:0") -> Graph:
    """Runs fn() once eagerly on a side stream (warm-up), then records the
    library calls fn() makes into a HIP graph on that stream."""
    dev = torch.device(device)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream(dev).wait_stream(s)
    torch.cuda.synchronize(dev)
    g = Graph()
    with torch.cuda.stream(s):
        g.begin(s)
        try:
            fn()
        finally:
            g.end(s)
    return g


def saved_bytes(net: MLP, n: int) -> int:
    return int(_lib.dnnmg_patch_saved_bytes(ctypes.byref(net), n))


def dnnmg_patch_forward(net: MLP, n, X, ldx, Y, saved=None, stream=None):
    _check(_lib.dnnmg_patch_forward(ctypes.byref(net), int(n), _ptr(X, None, None, "X"), int(ldx),
                                    _ptr(Y, torch.float32, n * net.n_out, "Y"),
                                    _ptr(saved, None, None, "saved"), _stream(stream)))


def dnnmg_patch_forward_tiles(net: MLP, n, X, ldx, Y, tile_patches, grid=0, saved=None, stream=None):
    _check(_lib.dnnmg_patch_forward_tiles(ctypes.byref(net), int(n), _ptr(X, None, None, "X"), int(ldx),
                                          _ptr(Y, torch.float32, n * net.n_out, "Y"),
                                          _ptr(saved, None, None, "saved"), int(tile_patches), int(grid),
                                          _stream(stream)))


def dnnmg_scatter_avg(box, Y, d, vbase=None, stream=None):
    b = Box.of(box)
    nf, _, npch = box_sizes(b)
    nd = 3 if vbase is None else 4
    _check(_lib.dnnmg_scatter_avg(ctypes.byref(b), _ptr(Y, torch.float32, npch * N_OUT, "Y"),
                                  _ptr(vbase, torch.float32, 4 * nf, "vbase"),
                                  _ptr(d, torch.float32, nd * nf, "d"), _stream(stream)))

SCATTER_AUTO, SCATTER_NODES, SCATTER_TILED = 0, 1, 2


def dnnmg_scatter_avg_form(box, Y, d, form, vbase=None, stream=None):
    b = Box.of(box)
    nf, _, npch = box_sizes(b)
    nd = 3 if vbase is None else 4
    _check(_lib.dnnmg_scatter_avg_form(ctypes.byref(b), _ptr(Y, torch.float32, npch * N_OUT, "Y"),
                                       _ptr(vbase, torch.float32, 4 * nf, "vbase"),
                                       _ptr(d, torch.float32, nd * nf, "d"), int(form), _stream(stream)))


def norm2_workspace_bytes() -> int:
    return int(_lib.dnnmg_norm2_workspace())


def dnnmg_norm2_f64(a, out, ws, b=None, n=None, stream=None):
    n = a.numel() if n is None else n
    _check(_lib.dnnmg_norm2_f64(int(n), _ptr(a, torch.float32, n, "a"), _ptr(b, torch.float32, n, "b"),
                                _ptr(out, torch.float64, 1, "out"), _ptr(ws, None, None, "ws"),
                                ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_norm2_pair_f64(a0, a1, out, ws, n=None, stream=None):
    n = a0.numel() if n is None else n
    _check(_lib.dnnmg_norm2_pair_f64(int(n), _ptr(a0, torch.float32, n, "a0"), _ptr(a1, torch.float32, n, "a1"),
                                     _ptr(out, torch.float64, 2, "out"), _ptr(ws, None, None, "ws"),
                                     ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_mse_grad(Y, T, dY, n=None, stream=None):
    n = Y.numel() // N_OUT if n is None else n
    _check(_lib.dnnmg_mse_grad(int(n), _ptr(Y, torch.float32, n * N_OUT, "Y"),
                               _ptr(T, torch.float32, n * N_OUT, "T"),
                               _ptr(dY, torch.float32, n * N_OUT, "dY"), _stream(stream)))


def dnnmg_mse_grad_loss(Y, T, dY, loss_sum, ws, n=None, stream=None):
    """dY = 2 (Y - T) / n and loss_sum = sum (Y - T)^2 (FP64) in one pass."""
    n = Y.numel() // N_OUT if n is None else n
    _check(_lib.dnnmg_mse_grad_loss(int(n), _ptr(Y, torch.float32, n * N_OUT, "Y"),
                                    _ptr(T, torch.float32, n * N_OUT, "T"),
                                    _ptr(dY, torch.float32, n * N_OUT, "dY"),
                                    _ptr(loss_sum, torch.float64, 1, "loss_sum"), _ptr(ws, None, None, "ws"),
                                    ws.numel() * ws.element_size(), _stream(stream)))


def backward_workspace_bytes(net: MLP, n: int) -> int:
    return int(_lib.dnnmg_patch_backward_workspace(ctypes.byref(net), int(n)))


def dnnmg_patch_backward(net: MLP, W2, W3, n, X, ldx, saved, dY, dW, db, ws, stream=None):
    H = net.hidden
    dw = (c_vp * 3)(*[_ptr(t, torch.float32, sz, "dW").value for t, sz in
                      zip(dW, (N_IN * H, H * H, H * N_OUT))])
    dbs = (c_vp * 3)(*[_ptr(t, torch.float32, sz, "db").value for t, sz in zip(db, (H, H, N_OUT))])
    _check(_lib.dnnmg_patch_backward(ctypes.byref(net), _ptr(W2, torch.float32, H * H, "W2"),
                                     _ptr(W3, torch.float32, H * N_OUT, "W3"), int(n),
                                     _ptr(X, None, None, "X"), int(ldx), _ptr(saved, None, None, "saved"),
                                     _ptr(dY, torch.float32, n * N_OUT, "dY"), dw, dbs,
                                     _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(),
                                     _stream(stream)))


def dnnmg_adamw_step(theta, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8, wd=1e-5, stream=None):
    n = theta.numel()
    _check(_lib.dnnmg_adamw_step(int(n), _ptr(theta, torch.float32, n, "theta"), _ptr(m, torch.float32, n, "m"),
                                 _ptr(v, torch.float32, n, "v"), _ptr(g, torch.float32, n, "g"),
                                 float(lr), float(b1), float(b2), float(eps), float(wd), int(t),
                                 _stream(stream)))


def vanka_workspace_bytes(box) -> int:
    return int(_lib.dnnmg_vanka_workspace(ctypes.byref(Box.of(box))))


def dnnmg_vanka_sweeps(box, ns, x, vprev, ws, sweeps=1, omega=1.0, coupled=False, fmid=None, stream=None):
    b = Box.of(box)
    nf, _, _ = box_sizes(b)
    _check(_lib.dnnmg_vanka_sweeps(ctypes.byref(b), ctypes.byref(NS.of(ns)), _ptr(x, torch.float32, 4 * nf, "x"),
                                   _ptr(vprev, torch.float32, 3 * nf, "vprev"),
                                   _ptr(fmid, torch.float32, 3 * nf, "fmid"), int(sweeps), float(omega),
                                   int(bool(coupled)), _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(),
                                   _stream(stream)))


def fallback_workspace_bytes(box) -> int:
    return int(_lib.dnnmg_fallback_workspace(ctypes.byref(Box.of(box))))


def dnnmg_fallback_b(box, ns, xt, b, norms, xcorr, ws, theta=1.0, sweeps=4, omega=1.0, flag_out=None,
                     stream=None):
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    _check(_lib.dnnmg_fallback_b(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(xt, torch.float32, 4 * nf, "xt"),
                                 _ptr(b, torch.float32, 4 * nf, "b"), _ptr(norms, torch.float64, 2, "norms"),
                                 float(theta), int(sweeps), float(omega), _ptr(xcorr, torch.float32, 4 * nf, "xcorr"),
                                 _ptr(flag_out, torch.int32, 1, "flag_out"), _ptr(ws, None, None, "ws"),
                                 ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_fallback(box, ns, xt, vprev, norms, xcorr, ws, theta=1.0, sweeps=4, omega=1.0, flag_out=None,
                   fmid=None, stream=None):
    b = Box.of(box)
    nf, _, _ = box_sizes(b)
    _check(_lib.dnnmg_fallback(ctypes.byref(b), ctypes.byref(NS.of(ns)), _ptr(xt, torch.float32, 4 * nf, "xt"),
                               _ptr(vprev, torch.float32, 3 * nf, "vprev"),
                               _ptr(fmid, torch.float32, 3 * nf, "fmid"), _ptr(norms, torch.float64, 2, "norms"),
                               float(theta), int(sweeps), float(omega), _ptr(xcorr, torch.float32, 4 * nf, "xcorr"),
                               _ptr(flag_out, torch.int32, 1, "flag_out"), _ptr(ws, None, None, "ws"),
                               ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_patch_gather_forward(box, net: MLP, xt, r, Y, shift=None, inv_scale=None, stream=None):
    b = Box.of(box)
    nf, _, npch = box_sizes(b)
    feat = Feat(None if shift is None else _ptr(shift, torch.float32, 165, "shift"),
                None if inv_scale is None else _ptr(inv_scale, torch.float32, 165, "inv_scale"))
    _check(_lib.dnnmg_patch_gather_forward(ctypes.byref(b), ctypes.byref(net), _ptr(xt, torch.float32, 4 * nf, "xt"),
                                           _ptr(r, torch.float32, 4 * nf, "r"), ctypes.byref(feat),
                                           _ptr(Y, torch.float32, npch * N_OUT, "Y"), _stream(stream)))


class Plan:
    """Owner of a dnnmg_plan handle and its device workspace."""

    def __init__(self, boxes, ns, device="cuda:0", stream=None):
        self.boxes = (Box * len(boxes))(*[Box.of(b) for b in boxes])
        self.nbox = len(boxes)
        nbytes = int(_lib.dnnmg_plan_workspace(self.boxes, self.nbox))
        if nbytes == 0:
            raise DnnmgError(-2, "invalid box list")
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        self.ns = NS.of(ns)
        h = c_vp()
        _check(_lib.dnnmg_plan_create(self.boxes, self.nbox, ctypes.byref(self.ns), _ptr(self.ws), nbytes,
                                      ctypes.byref(h), _stream(stream)))
        self.handle = h
        nf, nc, npch = c_i64(), c_i64(), c_i64()
        _check(_lib.dnnmg_plan_sizes(h, ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(npch)))
        self.n_fine, self.n_coarse, self.n_patches = nf.value, nc.value, npch.value

    def choice(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(_lib.dnnmg_plan_choice(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def scatter_form(self):
        f = ctypes.c_int()
        _check(_lib.dnnmg_plan_scatter_form(self.handle, ctypes.byref(f)))
        return f.value

    def set_scatter_form(self, form):
        _check(_lib.dnnmg_plan_set_scatter_form(self.handle, int(form)))

    def _args(self, net, shift, inv_scale, bufs):
        nf, nc, npch = self.n_fine, self.n_coarse, self.n_patches
        return [ctypes.byref(net), _ptr(shift, torch.float32, 165, "shift"),
                _ptr(inv_scale, torch.float32, 165, "inv_scale"),
                _ptr(bufs["xc"], torch.float64, 4 * nc, "xc"), _ptr(bufs["vprev"], torch.float32, 3 * nf, "vprev"),
                _ptr(bufs["xt"], torch.float32, 4 * nf, "xt"), _ptr(bufs["r"], torch.float32, 4 * nf, "r"),
                _ptr(bufs["Y"], torch.float32, npch * N_OUT, "Y"), _ptr(bufs["xcorr"], torch.float32, 4 * nf, "xcorr"),
                _ptr(bufs["b"], torch.float32, 4 * nf, "b"), _ptr(bufs["bc"], torch.float64, 4 * nc, "bc")]

    def step(self, net, bufs, shift=None, inv_scale=None, stream=None):
        _check(_lib.dnnmg_batch_step(self.handle, *self._args(net, shift, inv_scale, bufs), _stream(stream)))

    def step_b(self, net, bufs, shift=None, inv_scale=None, stream=None):
        nf, nc, npch = self.n_fine, self.n_coarse, self.n_patches
        _check(_lib.dnnmg_batch_step_b(self.handle, ctypes.byref(net), _ptr(shift, torch.float32, 165, "shift"),
                                       _ptr(inv_scale, torch.float32, 165, "inv_scale"),
                                       _ptr(bufs["xc"], torch.float64, 4 * nc, "xc"),
                                       _ptr(bufs["b"], torch.float32, 4 * nf, "b"),
                                       _ptr(bufs["xt"], torch.float32, 4 * nf, "xt"),
                                       _ptr(bufs["r"], torch.float32, 4 * nf, "r"),
                                       _ptr(bufs["Y"], torch.float32, npch * N_OUT, "Y"),
                                       _ptr(bufs["xcorr"], torch.float32, 4 * nf, "xcorr"),
                                       _ptr(bufs["bc"], torch.float64, 4 * nc, "bc"), _stream(stream)))

    def rhs(self, v4, b, stream=None):
        nf = self.n_fine
        _check(_lib.dnnmg_batch_rhs(self.handle, _ptr(v4, torch.float32, 4 * nf, "v"), _ptr(b, torch.float32, 4 * nf, "b"),
                                    _stream(stream)))

    def autotune(self, net, bufs, shift=None, inv_scale=None, reps=5, stream=None):
        _check(_lib.dnnmg_plan_autotune(self.handle, *self._args(net, shift, inv_scale, bufs), int(reps),
                                        _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _lib.dnnmg_plan_destroy(h)
            self.handle = None


# ---------------------------------------------------------- coarse step ----
def coarse_opts(newton_its=8, krylov_dim=16, levels=1, pre_sweeps=1, post_sweeps=0, coarsest_sweeps=1, omega=1.0,
                fd_eta=1e-3) -> CoarseOpts:
    """Defaults: the preconditioner is one coupled patch-Vanka sweep on the
    coarse mesh itself (levels=1); see dnnmg_coarse_solve for why the
    multigrid correction is off by default."""
    return CoarseOpts(int(newton_its), int(krylov_dim), int(levels), int(pre_sweeps), int(post_sweeps),
                      int(coarsest_sweeps), float(omega), float(fd_eta))


def coarse_levels(box, opts: CoarseOpts) -> int:
    n = int(_lib.dnnmg_coarse_levels(ctypes.byref(Box.of(box)), ctypes.byref(opts)))
    if n < 0:
        _check(n)
    return n


def coarse_workspace_bytes(box, opts: CoarseOpts) -> int:
    n = int(_lib.dnnmg_coarse_workspace(ctypes.byref(Box.of(box)), ctypes.byref(opts)))
    if n == 0:
        coarse_levels(box, opts)  # raises with the reason
    return n


def dnnmg_coarse_solve(box, ns, b, x, opts: CoarseOpts, ws, res_norms=None, stream=None):
    bx = Box.of(box)
    _, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_coarse_solve(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(b, torch.float64, 4 * nc, "b"),
                                   _ptr(x, torch.float64, 4 * nc, "x"), ctypes.byref(opts),
                                   _ptr(res_norms, torch.float64, opts.newton_its + 1, "res_norms"),
                                   _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_coarse_jv(box, ns, x, z, w, opts: CoarseOpts, ws, stream=None):
    bx = Box.of(box)
    _, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_coarse_jv(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(x, torch.float32, 4 * nc, "x"),
                                _ptr(z, torch.float32, 4 * nc, "z"), _ptr(w, torch.float32, 4 * nc, "w"),
                                ctypes.byref(opts), _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(),
                                _stream(stream)))


def dnnmg_coarse_vcycle(box, ns, x, s, z, opts: CoarseOpts, ws, stream=None):
    bx = Box.of(box)
    _, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_coarse_vcycle(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(x, torch.float32, 4 * nc, "x"),
                                    _ptr(s, torch.float32, 4 * nc, "s"), _ptr(z, torch.float32, 4 * nc, "z"),
                                    ctypes.byref(opts), _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(),
                                    _stream(stream)))


# ---------------------------------------- Q2/Q2 elements on curved hexahedra --

def q2_workspace_bytes(box) -> int:
    return int(_lib.dnnmg_q2_workspace(ctypes.byref(Box.of(box))))


def _q2_ws(box, ws):
    if ws is None:
        return torch.empty(q2_workspace_bytes(box), dtype=torch.uint8, device="cuda")
    return ws


def dnnmg_q2_residual_b(box, ns, coords, x, b, r, ws=None, stream=None):
    """ws: device workspace of q2_workspace_bytes(box) (allocated per call if None)."""
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    ws = _q2_ws(bx, ws)
    _check(_lib.dnnmg_q2_residual_b(ctypes.byref(bx), ctypes.byref(NS.of(ns)),
                                    _ptr(coords, torch.float64, 3 * nf, "coords"),
                                    _ptr(x, torch.float32, 4 * nf, "x"), _ptr(b, torch.float32, 4 * nf, "b"),
                                    _ptr(r, torch.float32, 4 * nf, "r"), _ptr(ws, None, None, "ws"),
                                    ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_q2_residual_rhs(box, ns, coords, x, b, r, bnext, ws=None, stream=None):
    """r = b - A(x) and bnext = Rhs(x[:3]) in one pass (bnext may be b)."""
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    ws = _q2_ws(bx, ws)
    _check(_lib.dnnmg_q2_residual_rhs(ctypes.byref(bx), ctypes.byref(NS.of(ns)),
                                      _ptr(coords, torch.float64, 3 * nf, "coords"),
                                      _ptr(x, torch.float32, 4 * nf, "x"), _ptr(b, torch.float32, 4 * nf, "b"),
                                      _ptr(r, torch.float32, 4 * nf, "r"), _ptr(bnext, torch.float32, 4 * nf, "bnext"),
                                      _ptr(ws, None, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_q2_rhs(box, ns, coords, v, b_out, fmid=None, ws=None, stream=None):
    bx = Box.of(box)
    nf, _, _ = box_sizes(bx)
    ws = _q2_ws(bx, ws)
    _check(_lib.dnnmg_q2_rhs(ctypes.byref(bx), ctypes.byref(NS.of(ns)), _ptr(coords, torch.float64, 3 * nf, "coords"),
                             _ptr(v, torch.float32, 3 * nf, "v"), _ptr(fmid, torch.float32, 3 * nf, "fmid"),
                             _ptr(b_out, torch.float32, 4 * nf, "b"), _ptr(ws, None, None, "ws"),
                             ws.numel() * ws.element_size(), _stream(stream)))


def dnnmg_q2_prolong(box, xc, xf, ncomp=4, stream=None):
    bx = Box.of(box)
    nf, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_q2_prolong(ctypes.byref(bx), ncomp, _ptr(xc, torch.float64, ncomp * nc, "xc"),
                                 _ptr(xf, torch.float32, ncomp * nf, "xf"), _stream(stream)))


def dnnmg_q2_restrict(box, bf, bc, ncomp=4, stream=None):
    bx = Box.of(box)
    nf, nc, _ = box_sizes(bx)
    _check(_lib.dnnmg_q2_restrict(ctypes.byref(bx), ncomp, _ptr(bf, torch.float32, ncomp * nf, "bf"),
                                  _ptr(bc, torch.float64, ncomp * nc, "bc"), _stream(stream)))


def dnnmg_q2_patch_features(box, coords, geom, stream=None):
    bx = Box.of(box)
    nf, _, npch = box_sizes(bx)
    _check(_lib.dnnmg_q2_patch_features(ctypes.byref(bx), _ptr(coords, torch.float64, 3 * nf, "coords"),
                                        _ptr(geom, torch.float32, 3 * npch, "geom"), _stream(stream)))


def dnnmg_patch_gather_geom(box, geom, x, r, X, dtype, ldx, shift=None, inv_scale=None, x_scale=1.0, stream=None):
    bx = Box.of(box)
    nf, _, npch = box_sizes(bx)
    feat = Feat(_ptr(shift, torch.float32, 165, "shift"), _ptr(inv_scale, torch.float32, 165, "inv_scale"))
    if X.numel() * X.element_size() < npch * ldx * {F32: 4, BF16: 2, FP8_E4M3: 1}[dtype]:
        raise ValueError("X too small")
    _check(_lib.dnnmg_patch_gather_geom(ctypes.byref(bx), _ptr(geom, torch.float32, 3 * npch, "geom"),
                                        _ptr(x, torch.float32, 3 * nf, "x"), _ptr(r, torch.float32, 3 * nf, "r"),
                                        ctypes.byref(feat), dtype, float(x_scale), _ptr(X, None, None, "X"), ldx,
                                        _stream(stream)))


def dnnmg_patch_gather_forward_geom(box, net, geom, xt, r, Y, shift=None, inv_scale=None, stream=None):
    bx = Box.of(box)
    nf, _, npch = box_sizes(bx)
    feat = Feat(_ptr(shift, torch.float32, 165, "shift"), _ptr(inv_scale, torch.float32, 165, "inv_scale"))
    _check(_lib.dnnmg_patch_gather_forward_geom(ctypes.byref(bx), ctypes.byref(net),
                                                _ptr(geom, torch.float32, 3 * npch, "geom"),
                                                _ptr(xt, torch.float32, 3 * nf, "xt"),
                                                _ptr(r, torch.float32, 3 * nf, "r"), ctypes.byref(feat),
                                                _ptr(Y, torch.float32, npch * N_OUT, "Y"), _stream(stream)))


def dnnmg_q2_patch_features24(box, coords, geo24, stream=None):
    bx = Box.of(box)
    nf, _, npch = box_sizes(bx)
    _check(_lib.dnnmg_q2_patch_features24(ctypes.byref(bx), _ptr(coords, torch.float64, 3 * nf, "coords"),
                                          _ptr(geo24, torch.float32, 24 * npch, "geo24"), _stream(stream)))


def dnnmg_patch_gather_paper_geom(box, geo24, x, r, X, dtype, ldx, shift=None, inv_scale=None, stream=None):
    bx = Box.of(box)
    nf, _, npch = box_sizes(bx)
    feat = Feat(_ptr(shift, torch.float32, 240, "shift"), _ptr(inv_scale, torch.float32, 240, "inv_scale"))
    if X.numel() * X.element_size() < npch * ldx * {F32: 4, BF16: 2}[dtype]:
        raise ValueError("X too small")
    _check(_lib.dnnmg_patch_gather_paper_geom(ctypes.byref(bx), _ptr(geo24, torch.float32, 24 * npch, "geo24"),
                                              _ptr(x, torch.float32, 4 * nf, "x"), _ptr(r, torch.float32, 4 * nf, "r"),
                                              ctypes.byref(feat), dtype, _ptr(X, None, None, "X"), ldx,
                                              _stream(stream)))
