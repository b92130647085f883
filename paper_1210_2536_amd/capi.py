"""ctypes binding of ``include/spmv.h`` (argument marshalling only).

Every entry point of the C-ABI is exposed under the same name.  Loading
fails loudly when the HIP library has not been built: there is no fallback
path of any kind.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SMAT_SPMV_LIB") or os.path.join(HERE, "libsmat_spmv.so")

SPMV_F32, SPMV_F64 = 0, 1
SPMV_OK, SPMV_EINVAL, SPMV_ENOMEM, SPMV_EDEVICE, SPMV_EUNSUPPORTED = 0, -1, -2, -3, -4
KERNELS = ("csr_scalar", "csr_vector", "csr_adaptive", "ell", "dia", "dia_direct", "coo",
           "csr_panel", "bcsr")
(K_CSR_SCALAR, K_CSR_VECTOR, K_CSR_ADAPTIVE, K_ELL, K_DIA, K_DIA_DIRECT, K_COO, K_CSR_PANEL,
 K_BCSR) = range(9)
K_COUNT = 9
FORMATS = ("csr", "coo", "ell", "dia", "bcsr")
# storage format each kernel runs on (index into FORMATS); column panels are CSR
FORMAT_OF = (0, 0, 0, 2, 3, 3, 1, 0, 4)
SELECT_RULES, SELECT_MLP, SELECT_EXHAUSTIVE, SELECT_FORCED = range(4)

i32, i64, u32, u64, f32, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_float, ctypes.c_double)
vp = ctypes.c_void_p


class spmv_csr(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("nnz", i64), ("row_ptr_dev", vp), ("col_dev", vp),
                ("val_dev", vp), ("dtype", i32)]


class spmv_params(ctypes.Structure):
    _fields_ = [("block", i32), ("vector_lanes", i32), ("adaptive_rows_per_lane", i32),
                ("adaptive_wg_min", i32), ("dia_rows_per_thread", i32), ("dia_span", i32),
                ("coo_chunk", i32), ("ell_unroll", i32), ("stream_nt", i32),
                ("panel_kib", i32), ("panel_xcd", i32), ("wide_loads", i32), ("bcsr_lanes", i32), ("long_lds", i32),
                ("tile_row_min", i32), ("panel_direct_max", i32)]


ALLOC_FN = ctypes.CFUNCTYPE(vp, ctypes.c_size_t, vp)
FREE_FN = ctypes.CFUNCTYPE(None, vp, ctypes.c_size_t, vp)


class spmv_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", vp)]


class spmv_plan_opts(ctypes.Structure):
    _fields_ = [("selector", i32), ("force_kernel", i32), ("confidence_tau", f32),
                ("measure_topk", i32), ("timing_reps", i32), ("disable_mask", u32),
                ("mem_cap_bytes", u64), ("model", vp), ("autotune", i32), ("use_params", i32),
                ("params", spmv_params), ("segments", i32), ("staged", i32),
                ("stage_conf", f32), ("allocator", spmv_allocator), ("time_baseline", i32),
                ("log", i32)]


class spmv_features(ctypes.Structure):
    _fields_ = [(k, i64) for k in ("m", "n", "nnz", "sum_rd", "sum_rd2", "max_rd", "min_rd",
                                   "ndiags", "ntdiags", "bandwidth", "blocks4")] + \
               [(k, f64) for k in ("aver_rd", "var_rd", "std_rd", "er_dia", "er_ell",
                                   "ntdiags_ratio", "R", "block_fill")] + \
               [("dia_feasible", i32), ("ell_feasible", i32)]


class spmv_plan_info(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("nnz", i64), ("dtype", i32), ("kernel", i32),
                ("format", i32), ("selector_used", i32), ("confidence", f32),
                ("mlp_scores", f32 * K_COUNT), ("n_measured", i32),
                ("measured_kernel", i32 * K_COUNT), ("measured_ms", f64 * K_COUNT),
                ("feasible_mask", u32), ("features", spmv_features), ("params", spmv_params),
                ("ell_width", i32), ("dia_ndiags", i32), ("dia_windows", i32), ("m_pad", i64),
                ("device_bytes", u64), ("t_validate_ms", f64), ("t_features_ms", f64),
                ("t_select_ms", f64), ("t_convert_ms", f64), ("t_plan_ms", f64),
                ("mlp_input", f32 * 12), ("rules_kernel", i32),
                ("out_of_domain", i32), ("t_tune_ms", f64), ("bcsr_blocks", i64),
                ("n_segments", i32), ("feature_stage", i32), ("stage_confidence", f32),
                ("tune_rejected", i32), ("long_lanes", i32), ("long_rows", i64),
                ("t_run_ms", f64), ("t_plain_ms", f64), ("break_even_calls", f64)]


_SIGS = {
    "spmv_plan_opts_default": (i32, [vp]),
    "spmv_plan_opts_apply_env": (i32, [vp]),
    "spmv_plan_create": (i32, [vp, vp, vp, vp]),
    "spmv_run": (i32, [vp, vp, vp, vp]),
    "spmv_plan_info_get": (i32, [vp, vp]),
    "spmv_plan_segment": (i32, [vp, i32, vp, vp]),
    "spmv_plan_destroy": (i32, [vp]),
    "spmv_features_compute": (i32, [vp, vp, vp]),
    "spmv_features_compute_noalloc": (i32, [vp, vp, vp]),
    "spmv_convert_roundtrip": (i32, [vp, vp, vp, vp, vp]),
    "spmv_plan_export": (i32, [vp, i32, vp, ctypes.c_size_t, vp, vp]),
    "spmv_selector_create": (i32, [vp, i64, vp, vp, vp]),
    "spmv_selector_destroy": (i32, [vp]),
    "spmv_selector_set_domain": (i32, [vp, vp, vp]),
    "spmv_selector_set_stage": (i32, [vp, vp, vp, vp, vp, vp, vp, i32]),
    "spmv_selector_score": (i32, [vp, vp, i64, vp, vp]),
    "spmv_mlp_param_count": (i64, [i32]),
    "spmv_mlp_workspace_floats": (i64, [i64]),
    "spmv_mlp_forward": (i32, [vp, i32, vp, i64, vp, vp, vp]),
    "spmv_mlp_backward": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp, vp]),
    "spmv_mlp_adam": (i32, [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]),
    "spmv_batch_create": (i32, [vp, i32, i32, vp]),
    "spmv_batch_run": (i32, [vp, vp, vp, vp]),
    "spmv_batch_destroy": (i32, [vp]),
    "spmv_batch_tune": (i32, [vp, vp, vp, i32, vp, vp]),
    "spmv_batch_shape": (i32, [vp, vp, vp]),
    "spmv_stream_copy": (i32, [vp, vp, ctypes.c_size_t, vp]),
    "spmv_stream_read": (i32, [vp, ctypes.c_size_t, vp, vp]),
    "spmv_stream_read_out_bytes": (ctypes.c_size_t, []),
    "spmv_gather_probe": (i32, [vp, i64, vp, vp, i64, i32, vp, vp]),
    "spmv_gather_probe_threads": (i64, []),
    "spmv_status_string": (ctypes.c_char_p, [i32]),
    "spmv_last_error": (ctypes.c_char_p, []),
    "spmv_kernel_name": (ctypes.c_char_p, [i32]),
}

_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1210_2536_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


class SpmvError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        self.status = status
        msg = L.spmv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.spmv_status_string(status).decode()} ({msg})")


def check(status, where):
    if status != SPMV_OK:
        raise SpmvError(status, where)
    return status


def __getattr__(name):  # module-level access to raw entry points: capi.spmv_run(...)
    if name.startswith("spmv_"):
        return getattr(lib(), name)
    raise AttributeError(name)
