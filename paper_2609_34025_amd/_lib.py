"""ctypes binding of libtfi.so (C ABI in include/tfi.h).

Argument marshalling only: every step of an integration runs in the HIP
library. There is no CPU fallback; if the library is missing, loading it
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfi.so")

TFI_F32 = 0
TFI_F64 = 1

POLICIES = {"adaptive": 0, "diameter": 1, "centroid": 2, "channel": 3}
TABLE_METHODS = {"auto": 0, "direct": 1, "fft": 2, "fft1d": 3, "hankel": 4}

STATUS = {0: "ok", -1: "TFI_ERR_ARG", -2: "TFI_ERR_TREE", -3: "TFI_ERR_WEIGHT",
          -4: "TFI_ERR_DTYPE", -5: "TFI_ERR_OOM", -6: "TFI_ERR_BUDGET",
          -7: "TFI_ERR_HIP", -8: "TFI_ERR_STATE"}


class TFIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class BuildOpts(C.Structure):
    _fields_ = [("policy", C.c_int32), ("leaf_max", C.c_int32), ("device", C.c_int32),
                ("table_method", C.c_int32), ("memory_budget_bytes", C.c_uint64),
                ("no_graphs", C.c_int32), ("fft_cost", C.c_float),
                ("direct_kernel", C.c_int32), ("chan_width", C.c_int32),
                ("cost_vertex", C.c_float), ("cost_direct", C.c_float),
                ("cost_fft", C.c_float), ("cost_call", C.c_float)]


class FftParams(C.Structure):
    _fields_ = [("lds_pairs", C.c_int32 * 3), ("conv1d_min_lg", C.c_int32),
                ("conv1d_pairs", C.c_int32), ("conv1d_group_mib", C.c_int32),
                ("col_lines", C.c_int32)]


_lib = None

EXPORTED = ["tfi_build", "tfi_num_vertices", "tfi_kernel_length", "tfi_integrate",
            "tfi_backward", "tfi_plan_stats", "tfi_plan_export", "tfi_profile",
            "tfi_profile_report", "tfi_autotune", "tfi_set_fft_cost", "tfi_destroy",
            "tfi_last_error", "tfi_integrate_expsum", "tfi_backward_expsum", "tfi_calibrate",
            "tfi_integrate_multi", "tfi_cell_rows", "tfi_integrate_expsum_cells",
            "tfi_backward_expsum_cells", "tfi_integrate_cells", "tfi_backward_cells",
            "tfi_integrate_noalloc", "tfi_set_scatter", "tfi_set_fft_params",
            "tfi_get_fft_params", "tfi_autotune_fft"]

# bytes of the fixed device scratch array of tfi_integrate_noalloc
# (TFI_NOALLOC_SCRATCH_BYTES in include/tfi.h)
NOALLOC_SCRATCH_BYTES = 128 << 20


def load():
    """Load libtfi.so (built by ``paper_2609_34025_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2609_34025_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64 = C.c_void_p, C.c_int64
    lib.tfi_build.argtypes = [vp, vp, i64, C.POINTER(BuildOpts), C.POINTER(vp)]
    lib.tfi_build.restype = C.c_int
    lib.tfi_num_vertices.argtypes = [vp]
    lib.tfi_num_vertices.restype = i64
    lib.tfi_kernel_length.argtypes = [vp]
    lib.tfi_kernel_length.restype = i64
    lib.tfi_integrate.argtypes = [vp, vp, vp, i64, C.c_int, vp, vp]
    lib.tfi_integrate.restype = C.c_int
    lib.tfi_integrate_noalloc.argtypes = [vp, vp, vp, i64, C.c_int, vp, vp]
    lib.tfi_integrate_noalloc.restype = C.c_int
    lib.tfi_backward.argtypes = [vp, vp, vp, vp, i64, C.c_int, vp, vp, vp]
    lib.tfi_backward.restype = C.c_int
    lib.tfi_plan_stats.argtypes = [vp, C.c_char_p, C.c_size_t]
    lib.tfi_plan_stats.restype = i64
    lib.tfi_plan_export.argtypes = [vp, C.c_char_p, vp, C.c_size_t]
    lib.tfi_plan_export.restype = i64
    lib.tfi_destroy.argtypes = [vp]
    lib.tfi_destroy.restype = None
    lib.tfi_profile.argtypes = [vp, C.c_int]
    lib.tfi_profile.restype = C.c_int
    lib.tfi_profile_report.argtypes = [vp, C.c_char_p, C.c_size_t]
    lib.tfi_profile_report.restype = i64
    lib.tfi_autotune.argtypes = [vp, vp, i64, C.c_int, C.c_int, C.POINTER(C.c_float), vp]
    lib.tfi_autotune.restype = C.c_int
    lib.tfi_set_fft_cost.argtypes = [vp, C.c_float]
    lib.tfi_set_fft_cost.restype = C.c_int
    lib.tfi_set_scatter.argtypes = [vp, C.c_int32]
    lib.tfi_set_scatter.restype = C.c_int
    lib.tfi_set_fft_params.argtypes = [vp, C.POINTER(FftParams)]
    lib.tfi_set_fft_params.restype = C.c_int
    lib.tfi_get_fft_params.argtypes = [vp, C.POINTER(FftParams)]
    lib.tfi_get_fft_params.restype = C.c_int
    lib.tfi_autotune_fft.argtypes = [vp, vp, i64, C.c_int, C.c_int, vp]
    lib.tfi_autotune_fft.restype = C.c_int
    lib.tfi_calibrate.argtypes = [vp, vp, i64, C.c_int, C.POINTER(C.c_float), vp]
    lib.tfi_calibrate.restype = C.c_int
    lib.tfi_integrate_multi.argtypes = [vp, C.c_int32, C.POINTER(vp), vp, i64, C.c_int,
                                        C.POINTER(vp), vp]
    lib.tfi_integrate_multi.restype = C.c_int
    lib.tfi_integrate_expsum.argtypes = [vp, C.c_int32, vp, vp, vp, i64, C.c_int, vp, vp]
    lib.tfi_integrate_expsum.restype = C.c_int
    lib.tfi_backward_expsum.argtypes = [vp, C.c_int32, vp, vp, vp, vp, i64, C.c_int, vp, vp, vp,
                                        vp]
    lib.tfi_backward_expsum.restype = C.c_int
    lib.tfi_integrate_cells.argtypes = [vp, vp, vp, i64, C.c_int, vp, vp, vp]
    lib.tfi_integrate_cells.restype = C.c_int
    lib.tfi_backward_cells.argtypes = [vp, vp, vp, vp, vp, i64, C.c_int, vp, vp, vp]
    lib.tfi_backward_cells.restype = C.c_int
    lib.tfi_cell_rows.argtypes = [vp]
    lib.tfi_cell_rows.restype = i64
    lib.tfi_integrate_expsum_cells.argtypes = [vp, C.c_int32, vp, vp, vp, i64, C.c_int, vp, vp,
                                               vp]
    lib.tfi_integrate_expsum_cells.restype = C.c_int
    lib.tfi_backward_expsum_cells.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, i64, C.c_int, vp,
                                              vp, vp, vp]
    lib.tfi_backward_expsum_cells.restype = C.c_int
    lib.tfi_last_error.argtypes = []
    lib.tfi_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(rc):
    if rc < 0:
        msg = load().tfi_last_error().decode(errors="replace")
        raise TFIError(int(rc), msg)
    return rc


def build_handle(parent, weight, policy="adaptive", leaf_max=0, device=0,
                 table_method="auto", memory_budget=0, graphs=True, fft_cost=0.0,
                 direct_kernel="auto", channel_width=0, cost_model=None):
    lib = load()
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    weight = np.ascontiguousarray(weight, dtype=np.int32)
    if parent.ndim != 1 or parent.shape != weight.shape:
        raise TFIError(-1, "parent and weight must be 1-D arrays of equal length")
    o = BuildOpts()
    o.policy = POLICIES[policy] if isinstance(policy, str) else int(policy)
    o.leaf_max = int(leaf_max)
    o.device = -1 if device is None else int(device)
    o.table_method = (TABLE_METHODS[table_method] if isinstance(table_method, str)
                      else int(table_method))
    o.memory_budget_bytes = int(memory_budget)
    o.no_graphs = 0 if graphs else 1
    o.fft_cost = float(fft_cost)
    o.direct_kernel = {"auto": 0, "vector": 1, "mfma": 2}[direct_kernel]
    o.chan_width = int(channel_width)
    if cost_model:
        o.cost_vertex = float(cost_model["vertex"])
        o.cost_direct = float(cost_model["direct"])
        o.cost_fft = float(cost_model["fft"])
        o.cost_call = float(cost_model.get("call", 0.0))
    h = C.c_void_p()
    check(lib.tfi_build(parent.ctypes.data, weight.ctypes.data, len(parent),
                        C.byref(o), C.byref(h)))
    return h


_EXPORT_TYPES = {"i32": np.int32, "i64": np.int64, "i8": np.int8}
