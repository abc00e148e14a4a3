"""ctypes declarations of the C ABI in include/xengine.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libxengine.so")

c_i32, c_i64, c_f64, c_vp, c_char_p, c_size_t = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t)

# enums (xengine.h)
XC_OK = 0
STATUS_NAMES = {0: "XC_OK", 1: "XC_ERR_INVALID_ARG", 2: "XC_ERR_UNSUPPORTED", 3: "XC_ERR_OUT_OF_MEMORY",
                4: "XC_ERR_OVERFLOW_RISK", 5: "XC_ERR_ADMISSION", 6: "XC_ERR_BACKPRESSURE", 7: "XC_ERR_HIP",
                8: "XC_ERR_STATE"}
XC_IN_CF32, XC_IN_CI8, XC_IN_CF16, XC_IN_CBF16 = 0, 1, 2, 3
XC_OUT_CF32, XC_OUT_CI32 = 0, 1
XC_KERNEL_AUTO, XC_KERNEL_VALU, XC_KERNEL_MFMA = 0, 1, 2
XC_CI32_MAX_TIMES = 66572
XC_SPLIT_STATIC_SCRATCH_BYTES = 64 << 20
XC_PEAK_F32_MFMA16, XC_PEAK_F32_MFMA32, XC_PEAK_I8_MFMA, XC_PEAK_F16_MFMA, XC_PEAK_BF16_MFMA, XC_PEAK_F32_FMA, \
    XC_PEAK_HBM_COPY = range(7)


XC_STAGING_AUTO, XC_STAGING_REGISTERS, XC_STAGING_LDS = 0, 1, 2
XC_PRODUCT_AUTO, XC_PRODUCT_FOUR, XC_PRODUCT_THREE = 0, 1, 2
XC_LAYOUT_TIME_MAJOR, XC_LAYOUT_STATION_MAJOR = 0, 1


class XcConfig(ctypes.Structure):
    _fields_ = [("kernel", c_i32), ("block", c_i32), ("time_chunk", c_i32), ("time_split", c_i32),
                ("staging", c_i32), ("product", c_i32), ("tile_w", c_i32), ("tile_h", c_i32)]


class XcSubarray(ctypes.Structure):
    _fields_ = [("samples", c_vp), ("vis", c_vp), ("n_stations", c_i32), ("n_channels", c_i32),
                ("n_times", c_i32)]


class XcStreamDesc(ctypes.Structure):
    _fields_ = [("n_stations", c_i32), ("n_pol", c_i32), ("n_channels", c_i32), ("block_times", c_i32),
                ("blocks_per_integration", c_i32), ("blocks_per_fold", c_i32), ("ring_blocks", c_i32),
                ("in_type", c_i32), ("acc_type", c_i32), ("staggered", c_i32), ("block_period_s", c_f64)]


class XcLatencyStats(ctypes.Structure):
    _fields_ = [("p50_ms", c_f64), ("p99_ms", c_f64), ("max_ms", c_f64), ("deadline_ms", c_f64), ("tflops", c_f64),
                ("blocks", c_i64), ("misses", c_i64), ("pending", c_i64), ("fold_p50_ms", c_f64),
                ("fold_p99_ms", c_f64), ("fold_max_ms", c_f64), ("fold_deadline_ms", c_f64), ("folds", c_i64),
                ("fold_misses", c_i64), ("integrations", c_i64)]


# name -> (restype, argtypes): every symbol include/xengine.h declares
SIGNATURES = {
    "xc_n_baselines": (c_i64, [c_i32]),
    "xc_baseline_index": (c_i64, [c_i32, c_i32]),
    "xc_vis_elems": (c_i64, [c_i32, c_i32, c_i32]),
    "xc_sample_bytes": (c_i64, [c_i32, c_i32, c_i32, c_i32, c_i32]),
    "xc_vis_bytes": (c_i64, [c_i32, c_i32, c_i32, c_i32]),
    "xc_correlate": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_i32, c_i32, c_vp]),
    "xc_resolve_config": (c_i32, [ctypes.POINTER(XcConfig), c_i32, c_i32, c_i32, c_i32, c_i32, c_i32,
                                  ctypes.POINTER(XcConfig)]),
    "xc_correlate_config": (c_i32, [ctypes.POINTER(XcConfig), c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp,
                                    c_i32, c_i32, c_vp]),
    "xc_correlate_split_bytes": (c_i64, [c_i32, c_i32, c_i32, c_i32, c_i32]),
    "xc_correlate_split": (c_i32, [ctypes.POINTER(XcConfig), c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_i32,
                                   c_i32, c_i32, c_vp, c_i64, c_vp]),
    "xc_correlate_split_static": (c_i32, [ctypes.POINTER(XcConfig), c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp,
                                          c_i32, c_i32, c_i32, c_vp]),
    "xc_correlate_station_major": (c_i32, [ctypes.POINTER(XcConfig), c_vp, c_i32, c_i32, c_i32, c_i32, c_i32,
                                           c_vp, c_i32, c_i32, c_vp]),
    "xc_tile_cost": (c_i32, [c_i32, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                             ctypes.POINTER(c_i64)]),
    "xc_perf_max": (c_f64, [c_f64, c_f64, c_f64]),
    "xc_ai_global": (c_f64, [c_i32]),
    "xc_flops": (c_f64, [c_i32, c_i32, c_i32]),
    "xc_batch_plan_create": (c_i32, [ctypes.POINTER(XcSubarray), c_i32, c_i32, c_i32, c_i32, c_i32,
                                     ctypes.POINTER(XcConfig), c_char_p, c_i32, c_vp, ctypes.POINTER(c_vp)]),
    "xc_batch_plan_run": (c_i32, [c_vp, c_vp]),
    "xc_batch_plan_destroy": (None, [c_vp]),
    "xc_batch_plan_units": (c_i64, [c_vp]),
    "xc_batch_worklist": (c_i64, [ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), c_i32,
                                  c_i32, ctypes.POINTER(c_i32), c_i64, ctypes.POINTER(c_i32)]),
    "xc_autotune": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_i32, c_char_p, c_vp,
                            ctypes.POINTER(XcConfig), ctypes.POINTER(c_f64)]),
    "xc_tune_cache_load": (c_i64, [c_char_p]),
    "xc_tune_candidates": (c_i64, [c_i32, ctypes.POINTER(XcConfig), c_i64]),
    "xc_tune_bucket": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_i32)]),
    "xc_server_create": (c_i32, [c_size_t, ctypes.POINTER(c_vp)]),
    "xc_server_destroy": (None, [c_vp]),
    "xc_stream_footprint": (c_size_t, [ctypes.POINTER(XcStreamDesc)]),
    "xc_stream_open": (c_i32, [c_vp, ctypes.POINTER(XcStreamDesc), ctypes.POINTER(c_i32)]),
    "xc_stream_acquire": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp)]),
    "xc_stream_commit": (c_i32, [c_vp, c_i32, ctypes.c_uint64]),
    "xc_stream_commit_after": (c_i32, [c_vp, c_i32, ctypes.c_uint64, c_vp]),
    "xc_stream_integration": (c_i32, [c_vp, c_i32, c_i64, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp)]),
    "xc_stream_release": (c_i32, [c_vp, c_i32, c_i64, c_vp]),
    "xc_wait_event": (c_i32, [c_vp, c_vp]),
    "xc_stream_hold": (c_i32, [c_vp, c_i32, c_f64]),
    "xc_stream_resume": (c_i32, [c_vp, c_i32]),
    "xc_stream_latest": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_i64)]),
    "xc_stream_stats": (c_i32, [c_vp, c_i32, ctypes.POINTER(XcLatencyStats)]),
    "xc_stream_close": (c_i32, [c_vp, c_i32]),
    "xc_stream_flush": (c_i32, [c_vp, c_i32]),
    "xc_server_set_fold_order": (c_i32, [c_vp, c_i32]),
    "xc_stream_reset_stats": (c_i32, [c_vp, c_i32]),
    "xc_quantile": (c_f64, [ctypes.POINTER(c_f64), c_i64, c_f64]),
    "xc_stream_schedule": (c_i32, [ctypes.POINTER(XcStreamDesc), c_i64, c_i32, ctypes.POINTER(c_i64), c_i64,
                                   ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_i64]),
    "xc_transpose_to_time_major": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp]),
    "xc_ingest_create": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_vp)]),
    "xc_ingest_info": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64)]),
    "xc_ingest_run": (c_i32, [c_vp, ctypes.POINTER(XcConfig), c_vp, c_vp, c_i32, c_i32, c_i32, c_vp]),
    "xc_ingest_destroy": (None, [c_vp]),
    "xc_pfb_create": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i64, ctypes.POINTER(c_vp)]),
    "xc_pfb_info": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64)]),
    "xc_pfb_run": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "xc_pfb_run_station_major": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "xc_pfb_destroy": (None, [c_vp]),
    "xc_measure_peak": (c_i32, [c_i32, ctypes.POINTER(c_f64)]),
    "xc_status_string": (c_char_p, [c_i32]),
    "xc_last_error": (c_char_p, []),
    "xc_version": (c_char_p, []),
}

_lock = threading.Lock()
_lib = None


class XengineError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


def load() -> ctypes.CDLL:
    """Load libxengine.so.  There is no fallback: if the library has not been
    built (``python -c 'import __graft_entry__ as g; g.build()'``) this raises."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is missing: build the HIP library first (__graft_entry__.build())")
        lib = ctypes.CDLL(LIBRARY)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(status: int) -> None:
    if status != XC_OK:
        msg = load().xc_last_error()
        raise XengineError(status, msg.decode() if msg else "")
