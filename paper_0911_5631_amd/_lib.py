"""ctypes declarations of the C ABI in include/md.h.

Loading fails loudly: there is no fallback implementation anywhere in the
package, so without the built gfx950 library nothing runs.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmd_gfx950.so")

MD_FORCE_FP32 = 0
MD_FORCE_FP64 = 1
MD_EVEN_CELLS = 1
MD_TRACE_PROPS = 2
MD_NO_REORDER = 4
MD_NO_WINDOW = 8
AB_VARIANTS = {"full": 0, "half": 1, "cells": 2}

STATUS = {
    0: "MD_OK", -1: "MD_ERR_INVALID_ARG", -2: "MD_ERR_BOX_TOO_SMALL", -3: "MD_ERR_OOM",
    -4: "MD_ERR_HIP", -5: "MD_ERR_NEBR_OVERFLOW", -6: "MD_ERR_ATOM_ESCAPED",
    -7: "MD_ERR_NONFINITE", -8: "MD_ERR_STATE", -9: "MD_ERR_NO_SLOT",
    -10: "MD_ERR_CELL_OVERFLOW",
}

# Every function the header declares (checked by the CPU test suite).
EXPORTS = (
    "md_status_string", "md_cells_per_edge", "md_query_bytes", "md_create", "md_bin_cells",
    "md_build_nebr", "md_forces", "md_step", "md_props", "md_get_state",
    "md_get_atom_energies", "md_set_state", "md_get_cells", "md_get_bins", "md_get_pairs",
    "md_adjust_temp", "md_block_begin", "md_block_end", "md_newton3_ab",
    "md_newton3_ab_noalloc", "md_ab_pairs", "md_set_species",
    "md_profile", "md_kernel_time", "md_configure", "md_get_trace", "md_destroy", "md_batch_create", "md_batch_admit",
    "md_batch_configure", "md_batch_run", "md_batch_poll", "md_batch_props", "md_batch_get_state",
    "md_batch_release", "md_batch_usage", "md_batch_progress", "md_batch_get_trace",
    "md_batch_destroy",
)


class MDError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        name = STATUS.get(code, str(code))
        text = ""
        try:
            text = lib().md_status_string(code).decode()
        except Exception:  # noqa: BLE001 - message only
            pass
        super().__init__(f"{where}: {name} ({text})" if where else f"{name} ({text})")


class md_params(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("box", C.c_double), ("r_cut", C.c_double),
                ("shell", C.c_double), ("dt", C.c_double), ("precision", C.c_int32),
                ("nebr_cap", C.c_int32), ("cell_cap", C.c_int32), ("flags", C.c_uint32),
                ("reorder_interval", C.c_int32)]


class md_props_t(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("virial", C.c_double),
                ("ke_per_atom", C.c_double), ("pe_per_atom", C.c_double),
                ("virial_per_atom", C.c_double), ("vmax", C.c_double), ("disp", C.c_double),
                ("n_pairs", C.c_int64), ("n_rebuilds", C.c_int64), ("step", C.c_int64),
                ("max_nebr", C.c_int32), ("max_cell", C.c_int32), ("rebuild_due", C.c_int32),
                ("cells_per_edge", C.c_int32), ("n_late_bins", C.c_int64)]


class md_launch_t(C.Structure):
    _fields_ = [("steps_per_run", C.c_int32), ("grid", C.c_int32), ("sort_grid", C.c_int32),
                ("sort_split", C.c_int32), ("tile_order", C.c_int32)]


class md_trace_t(C.Structure):
    _fields_ = [("step", C.c_int64), ("ke", C.c_double), ("pe", C.c_double),
                ("virial", C.c_double), ("vmax", C.c_double)]


class md_block_t(C.Structure):
    _fields_ = [("steps", C.c_int64), ("ke_per_atom", C.c_double), ("pe_per_atom", C.c_double),
                ("etot_per_atom", C.c_double), ("virial_per_atom", C.c_double),
                ("nebr_per_atom", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class md_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    """The loaded gfx950 library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_0911_5631_amd.build` "
                "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.md_status_string.restype = C.c_char_p
        L.md_status_string.argtypes = [C.c_int]
        L.md_cells_per_edge.restype = st
        L.md_cells_per_edge.argtypes = [C.POINTER(md_params), _I32]
        L.md_query_bytes.restype = st
        L.md_query_bytes.argtypes = [C.POINTER(md_params), C.POINTER(C.c_size_t)]
        L.md_create.restype = st
        L.md_create.argtypes = [C.POINTER(md_params), _D, _D, C.POINTER(md_allocator), _P,
                                C.POINTER(_P)]
        for name in ("md_bin_cells", "md_build_nebr", "md_forces"):
            getattr(L, name).restype = st
            getattr(L, name).argtypes = [_P]
        L.md_step.restype = st
        L.md_step.argtypes = [_P, C.c_int64]
        L.md_props.restype = st
        L.md_props.argtypes = [_P, C.POINTER(md_props_t)]
        L.md_adjust_temp.restype = st
        L.md_adjust_temp.argtypes = [_P, C.c_double]
        L.md_block_begin.restype = st
        L.md_block_begin.argtypes = [_P]
        L.md_block_end.restype = st
        L.md_block_end.argtypes = [_P, C.POINTER(md_block_t)]
        L.md_set_species.restype = st
        L.md_set_species.argtypes = [_P, C.c_int32, _I32, _D, _D, _D, _D]
        L.md_newton3_ab.restype = st
        L.md_newton3_ab.argtypes = [_P, C.c_int32, C.c_int32, _D, _D, _D, _I64]
        L.md_ab_pairs.restype = st
        L.md_ab_pairs.argtypes = [_P, C.c_int32, C.c_int64, _I32, _I32, _I64]
        L.md_newton3_ab_noalloc.restype = st
        L.md_newton3_ab_noalloc.argtypes = [_P, C.c_int32, C.c_int32, _D, _D, _D, _I64]
        L.md_get_state.restype = st
        L.md_get_state.argtypes = [_P, _D, _D, _D, _I64]
        L.md_get_atom_energies.restype = st
        L.md_get_atom_energies.argtypes = [_P, _D, _D]
        L.md_set_state.restype = st
        L.md_set_state.argtypes = [_P, _D, _D]
        L.md_get_cells.restype = st
        L.md_get_cells.argtypes = [_P, _I32]
        L.md_get_bins.restype = st
        L.md_get_bins.argtypes = [_P, _I32, _I32]
        L.md_get_pairs.restype = st
        L.md_get_pairs.argtypes = [_P, C.c_int64, _I32, _I32, _I64]
        L.md_profile.restype = st
        L.md_profile.argtypes = [_P, C.c_int32]
        L.md_kernel_time.restype = st
        L.md_kernel_time.argtypes = [_P, _I64, _D]
        L.md_destroy.restype = None
        L.md_destroy.argtypes = [_P]
        L.md_batch_create.restype = st
        L.md_batch_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(md_allocator),
                                      _P, C.POINTER(_P)]
        L.md_batch_admit.restype = st
        L.md_batch_admit.argtypes = [_P, C.POINTER(md_params), _D, _D, C.c_int64, _I32]
        L.md_batch_configure.restype = st
        L.md_batch_configure.argtypes = [_P, C.POINTER(md_launch_t)]
        L.md_get_trace.restype = st
        L.md_get_trace.argtypes = [_P, C.c_int64, C.c_int64, C.POINTER(md_trace_t)]
        L.md_batch_get_trace.restype = st
        L.md_batch_get_trace.argtypes = [_P, C.c_int32, C.c_int64, C.c_int64,
                                         C.POINTER(md_trace_t)]
        L.md_configure.restype = st
        L.md_configure.argtypes = [_P, C.POINTER(md_launch_t)]
        L.md_batch_run.restype = st
        L.md_batch_run.argtypes = [_P]
        L.md_batch_poll.restype = st
        L.md_batch_poll.argtypes = [_P, _I32, C.c_int32, _I32]
        L.md_batch_props.restype = st
        L.md_batch_props.argtypes = [_P, C.c_int32, C.POINTER(md_props_t)]
        L.md_batch_get_state.restype = st
        L.md_batch_get_state.argtypes = [_P, C.c_int32, _D, _D, _I64]
        L.md_batch_release.restype = st
        L.md_batch_release.argtypes = [_P, C.c_int32]
        L.md_batch_usage.restype = st
        L.md_batch_usage.argtypes = [_P, C.POINTER(C.c_size_t), _I32]
        L.md_batch_progress.restype = st
        L.md_batch_progress.argtypes = [_P, _I64, _I32, _I64]
        L.md_batch_destroy.restype = None
        L.md_batch_destroy.argtypes = [_P]
        _lib = L
    return _lib


def check(code: int, where: str = "") -> None:
    if code != 0:
        raise MDError(code, where)
