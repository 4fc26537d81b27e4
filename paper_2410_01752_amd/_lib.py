"""ctypes binding of libsisso.so (the C ABI declared in include/sisso.h).

Argument marshalling only: torch tensors are passed as device pointers and
the current torch stream as the HIP stream.  Every computation happens in the
library's HIP kernels.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsisso.so")

OPCODE = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sq": 4, "cube": 5, "sqrt": 6,
          "inv": 7, "exp": 8, "nexp": 9, "log": 10, "sin": 11}
OPNAME = {v: k for k, v in OPCODE.items()}

MAX_UNARY, MAX_BINARY, MAX_LEVELS = 8, 4, 2
MAX_N, MAX_KEEP, MAX_SUBSPACE, MAX_D = 65536, 2048, 1024, 3
MAX_BAND = 7168
UNIT_DIMS, UNIT_SCALE = 8, 16          # SISSO_UNIT_DIMS, SISSO_UNIT_SCALE
MOMENTS_NONE, MOMENTS_WRITE, MOMENTS_READ = 0, 1, 2
MAX_BATCH = 4096
ENC, MLP_IN, MLP_HIDDEN = 64, 144, 256
MLP_PARAMS = 256 * 144 + 256 + 256 + 1
MLP_TABLES = 5 * 256 + 256 + 1
FP32, BF16 = 0, 1
PRESCREEN = {"mi": 0, "spearman": 1}


class SissoError(RuntimeError):
    pass


class Space(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("levels", ctypes.c_int32), ("rect", ctypes.c_int32),
                ("n_unary", ctypes.c_int32), ("n_binary", ctypes.c_int32),
                ("unary", ctypes.c_int32 * MAX_UNARY), ("binary", ctypes.c_int32 * MAX_BINARY),
                ("n_slots", ctypes.c_int32),
                ("slot_op", ctypes.c_int32 * (2 * MAX_BINARY)),
                ("slot_rev", ctypes.c_int32 * (2 * MAX_BINARY)),
                ("pool", ctypes.c_int64 * (MAX_LEVELS + 1)),
                ("rect_unary", ctypes.c_int64), ("rect_binary", ctypes.c_int64),
                ("total", ctypes.c_int64)]


class ScoreArgs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pool32", ctypes.c_void_p), ("ld32", ctypes.c_int64),
                ("stats", ctypes.c_void_p), ("r32", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("exclude", ctypes.c_void_p), ("n_exclude", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("list_base", ctypes.c_int32), ("w32", ctypes.c_void_p), ("units", ctypes.c_void_p),
                ("col_grid", ctypes.c_int32)]


class Problem(ctypes.Structure):
    """sisso_problem: one entry of a batched problem table (device array)."""
    _fields_ = [("n", ctypes.c_int32), ("keep", ctypes.c_int32), ("ld32", ctypes.c_int64),
                ("pool32", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("r64", ctypes.c_void_p),
                ("r32", ctypes.c_void_p), ("info", ctypes.c_void_p), ("exclude", ctypes.c_void_p),
                ("n_exclude", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class L0Problem(ctypes.Structure):
    """sisso_l0_problem: one entry of a batched SO table (device array)."""
    _fields_ = [("F", ctypes.c_void_p), ("m", ctypes.c_int32), ("ld", ctypes.c_int32), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("y", ctypes.c_void_p), ("out_tuple", ctypes.c_void_p),
                ("out_sse", ctypes.c_void_p), ("out_coef", ctypes.c_void_p), ("out_resid", ctypes.c_void_p),
                ("out_stats", ctypes.c_void_p), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_int64)]


class EvalProblem(ctypes.Structure):
    """sisso_eval_problem: one entry of a batched materialisation table."""
    _fields_ = [("n", ctypes.c_int32), ("count", ctypes.c_int32), ("pool1_64", ctypes.c_void_p),
                ("ld64", ctypes.c_int64), ("stats", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("ldo", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("valid", ctypes.c_void_p)]


class SubspaceProblem(ctypes.Structure):
    """sisso_subspace_problem: one entry of a batched subspace-update table."""
    _fields_ = [("cand", ctypes.c_void_p), ("ldc", ctypes.c_int32), ("count_max", ctypes.c_int32),
                ("cand_ids", ctypes.c_void_p), ("cand_valid", ctypes.c_void_p), ("count_dev", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("n", ctypes.c_int32), ("lds", ctypes.c_int32), ("sub", ctypes.c_void_p),
                ("sub_ids", ctypes.c_void_p), ("m_prev", ctypes.c_int32), ("k", ctypes.c_int32),
                ("n_new", ctypes.c_void_p), ("n_classes", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_int64)]


class SortProblem(ctypes.Structure):
    """sisso_sort_problem: one entry of a batched subspace-sort table."""
    _fields_ = [("src", ctypes.c_void_p), ("lds", ctypes.c_int32), ("m", ctypes.c_int32), ("ids", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("ldd", ctypes.c_int32), ("dst", ctypes.c_void_p),
                ("ids_sorted", ctypes.c_void_p), ("perm", ctypes.c_void_p)]


def device_table(recs, dev) -> torch.Tensor:
    """A ctypes record array copied to device memory (a batched call's table)."""
    return torch.frombuffer(bytearray(recs), dtype=torch.uint8).to(dev)


COLSTAT_FLOATS = 8      # sisso_colstat: 8 floats
RESID_DOUBLES = 4       # sisso_resid_info: 4 doubles

_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise SissoError(f"libsisso.so not found at {LIBPATH}; build it with "
                         "`python -m paper_2410_01752_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIBPATH)
    sp = ctypes.POINTER(Space)
    ap = ctypes.POINTER(ScoreArgs)
    sig = {
        "sisso_space_init": (_i32, [sp]),
        "sisso_decode": (_i32, [sp, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64)]),
        "sisso_materialize_pools": (_i32, [sp, _vp, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _vp]),
        "sisso_materialize_ids": (_i32, [sp, _i32, _vp, _i64, _vp, _vp, _i32, _vp, _i32, _vp, _vp]),
        "sisso_materialize_ids_stored": (_i32, [sp, _i32, _i32, _vp, _i64, _vp, _vp, _i32, _vp, _i32, _vp,
                                                _vp]),
        "sisso_prepare_residual": (_i32, [_vp, _i32, _vp, _vp, _vp]),
        "sisso_prepare_residual_weighted": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
        "sisso_pool_units": (_i32, [sp, _vp, _vp, _vp, _vp]),
        "sisso_prepare_residual_batched": (_i32, [_vp, _i32, _vp]),
        "sisso_batch_workspace_size": (_sz, [sp, _i32, _i32]),
        "sisso_batch_items": (_i32, [sp]),
        "sisso_expand_score_batched": (_i32, [sp, _vp, _i32, _i32, _i32, _vp, _sz, _vp]),
        "sisso_topk_batched": (_i32, [_vp, _i32, _vp, _sz, _vp, _vp, _vp, _vp, _vp]),
        "sisso_l0_search_batched": (_i32, [_vp, _i32, _i32, _i32, _i32, ctypes.c_double, _vp, _vp]),
        "sisso_materialize_ids_batched": (_i32, [sp, _i32, _vp, _i32, _i32, _vp, _vp]),
        "sisso_subspace_update_batched": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp]),
        "sisso_sort_subspace_batched": (_i32, [_vp, _i32, _i32, _vp, _vp]),
        "sisso_score_workspace_size": (_sz, [sp, ap]),
        "sisso_score_reset": (_i32, [_vp, _sz, _vp]),
        "sisso_expand_score": (_i32, [sp, ap, _i64, _i64, _vp, _sz, _vp]),
        "sisso_expand_score_lists": (_i32, [sp, ap, _i64, _i64]),
        "sisso_topk": (_i32, [_vp, _sz, _i32, _vp, _vp, _vp, _vp]),
        "sisso_topk_status": (_i32, [_vp, _sz, _vp, _vp]),
        "sisso_select_threshold": (_i32, [_vp, _sz, ctypes.c_float, _i32, _vp, _vp, _vp, _vp]),
        "sisso_subspace_workspace_size": (_sz, [_i32, _i32, _i32]),
        "sisso_subspace_update": (_i32, [_vp, _i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _vp,
                                         _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
        "sisso_subspace_update_weighted": (_i32, [_vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _i32,
                                                  _vp, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
        "sisso_l0_search_weighted": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _i32, ctypes.c_double, _vp, _vp,
                                            _vp, _vp, _vp, _vp, _sz, _vp]),
        "sisso_l0_workspace_size": (_sz, [_i32, _i32, _i32]),
        "sisso_l0_outcome": (_i32, [_vp]),
        "sisso_l0_scratch_capacity": (_sz, []),
        "sisso_l0_search_noalloc": (_i32, [_vp, _i32, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp,
                                           _vp, _vp, _vp]),
        "sisso_l0_search": (_i32, [_vp, _i32, _i32, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp,
                                   _vp, _vp, _vp, _sz, _vp]),
        "sisso_sort_subspace": (_i32, [_vp, _i32, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp]),
        "sisso_bf16_operands_size": (_sz, [sp, _i32]),
        "sisso_prepare_bf16": (_i32, [sp, ap, _vp, _sz, _vp]),
        "sisso_bf16_workspace_size": (_sz, [sp, ap, _i32]),
        "sisso_expand_score_bf16_lists": (_i32, [sp, ap, _i32]),
        "sisso_expand_score_bf16": (_i32, [sp, ap, _vp, _sz, _i32, _i64, _i64, _vp, _sz, _vp, _sz, _vp]),
        "sisso_bf16_residual": (_i32, [sp, ap, _i32, _vp, _sz, _vp]),
        "sisso_bf16_screen": (_i32, [sp, ap, _vp, _sz, _i32, _i64, _i64, _vp, _sz, _vp]),
        "sisso_bf16_rescore": (_i32, [sp, ap, _i32, _vp, _sz, _vp, _sz, _vp]),
        "sisso_bf16_moments_size": (_sz, [sp, _i32]),
        "sisso_bf16_screen_moments": (_i32, [sp, ap, _vp, _sz, _i32, _i64, _i64, _vp, _sz, _i32, _vp, _sz, _vp]),
        "sisso_bf16_moments_images": (_i32, [sp, ap, _vp, _sz, _i32, _i64, _i64, _vp, _sz, _vp, _sz, _vp]),
        "sisso_bf16_moments_pass": (_i32, [sp, ap, _vp, _sz, _i32, _i64, _i64, _vp, _sz, _vp, _sz, _vp]),
        "sisso_mlp_param_count": (_i32, []),
        "sisso_mlp_table_count": (_i32, []),
        "sisso_encode_operands": (_i32, [sp, ap, _i64, _i64, _vp, _vp]),
        "sisso_candidate_inputs": (_i32, [sp, _vp, _vp, _i32, _vp, _vp]),
        "sisso_score_ids": (_i32, [sp, ap, _vp, _i32, _vp, _vp]),
        "sisso_mlp_forward": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp]),
        "sisso_mlp_workspace_size": (_sz, [_i32]),
        "sisso_mlp_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
        "sisso_mlp_target": (_i32, [_vp, _i32, _vp, _vp]),
        "sisso_adam_step": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, _vp]),
        "sisso_mlp_parts": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp]),
        "sisso_mlp_tables": (_i32, [_vp, _vp, _vp]),
        "sisso_mlp_score_ids": (_i32, [sp, _vp, _vp, _vp, _vp, _i32, _vp, _vp]),
        "sisso_select_kth": (_i32, [_vp, _i32, _i32, _vp, _vp]),
        "sisso_expand_score_pruned_lists": (_i32, [sp, ap, _i64, _i64]),
        "sisso_count_pass": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
        "sisso_expand_score_pruned": (_i32, [sp, ap, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _sz, _vp, _vp]),
        "sisso_prescreen_workspace_size": (_sz, [_i32, _i32]),
        "sisso_prescreen_scores": (_i32, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _sz, _vp]),
        "sisso_prescreen_select": (_i32, [_vp, _i32, ctypes.c_double, _vp, _vp, _vp]),
        "sisso_status_string": (ctypes.c_char_p, [_i32]),
        "sisso_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ["sisso_space_init", "sisso_decode", "sisso_materialize_pools", "sisso_materialize_ids",
            "sisso_prepare_residual", "sisso_score_workspace_size", "sisso_score_reset",
            "sisso_expand_score", "sisso_expand_score_lists", "sisso_topk", "sisso_topk_status", "sisso_select_threshold",
            "sisso_subspace_workspace_size",
            "sisso_subspace_update", "sisso_l0_workspace_size", "sisso_l0_search", "sisso_l0_outcome",
            "sisso_l0_scratch_capacity", "sisso_l0_search_noalloc",
            "sisso_sort_subspace", "sisso_bf16_operands_size", "sisso_prepare_bf16",
            "sisso_bf16_workspace_size", "sisso_expand_score_bf16_lists", "sisso_expand_score_bf16",
            "sisso_bf16_residual", "sisso_bf16_screen", "sisso_bf16_rescore", "sisso_bf16_moments_size",
            "sisso_bf16_screen_moments", "sisso_bf16_moments_images", "sisso_bf16_moments_pass",
            "sisso_materialize_ids_stored", "sisso_prepare_residual_batched", "sisso_batch_workspace_size",
            "sisso_batch_items", "sisso_expand_score_batched", "sisso_topk_batched", "sisso_l0_search_batched",
            "sisso_materialize_ids_batched", "sisso_subspace_update_batched", "sisso_sort_subspace_batched",
            "sisso_mlp_param_count", "sisso_mlp_table_count", "sisso_encode_operands", "sisso_candidate_inputs",
            "sisso_score_ids", "sisso_mlp_forward", "sisso_mlp_workspace_size", "sisso_mlp_backward",
            "sisso_mlp_target", "sisso_adam_step", "sisso_mlp_parts", "sisso_mlp_tables", "sisso_mlp_score_ids", "sisso_select_kth",
            "sisso_expand_score_pruned_lists", "sisso_expand_score_pruned", "sisso_count_pass",
            "sisso_prescreen_workspace_size", "sisso_prescreen_scores", "sisso_prescreen_select",
            "sisso_prepare_residual_weighted", "sisso_subspace_update_weighted", "sisso_l0_search_weighted",
            "sisso_pool_units",
            "sisso_status_string", "sisso_version"]


def check(status: int, what: str = ""):
    if status != 0:
        msg = lib().sisso_status_string(status).decode()
        raise SissoError(f"{what}: status {status} ({msg})")


def base_units(dimensionality) -> "np.ndarray":
    """int16 rows of SISSO_UNIT_DIMS exponents (times SISSO_UNIT_SCALE) for
    the base features from their unit strings (the dimensionality option of
    Sec. 3.3): every distinct string names a base dimension, in order of first
    appearance; "" or "1" marks a dimensionless feature."""
    import numpy as np
    names = []
    for u in dimensionality:
        if u not in ("", "1") and u not in names:
            names.append(u)
    if len(names) > UNIT_DIMS:
        raise SissoError(f"at most {UNIT_DIMS} distinct units")
    M = np.zeros((len(dimensionality), UNIT_DIMS), dtype=np.int16)
    for i, u in enumerate(dimensionality):
        if u not in ("", "1"):
            M[i, names.index(u)] = UNIT_SCALE
    return M


def ptr(t) -> int:
    if t is None:
        return None
    return t.data_ptr()


def stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def make_space(d: int, unary, binary, levels: int, rect: bool) -> Space:
    s = Space()
    s.d, s.levels, s.rect = d, levels, int(rect)
    s.n_unary, s.n_binary = len(unary), len(binary)
    for i, o in enumerate(unary):
        s.unary[i] = OPCODE[o]
    for i, o in enumerate(binary):
        s.binary[i] = OPCODE[o]
    check(lib().sisso_space_init(ctypes.byref(s)), "sisso_space_init")
    return s


def decode(space: Space, fid: int):
    op = _i32(); l = _i64(); r = _i64()
    check(lib().sisso_decode(ctypes.byref(space), fid, ctypes.byref(op), ctypes.byref(l),
                             ctypes.byref(r)), "sisso_decode")
    return op.value, l.value, r.value
