"""MI355X (gfx950) correlator X-engine.

Computes, per frequency channel c, the visibilities of Section 2 of
van Nieuwpoort & Romein, "Correlating Radio Astronomy Signals with Many-Core
Hardware":

    V[c][b(i,j)][p][q] = sum_t x[c][t][i][p] * conj(x[c][t][j][q]),
    0 <= i <= j < S,  b(i,j) = j(j+1)/2 + i,  p, q in {X, Y}.

Every step runs in the HIP library ``libxengine.so`` (include/xengine.h);
this package only marshals torch tensors (device memory and streams) into the
C ABI.  There is no CPU path: tensors must live on the GPU and the library
must be built.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (XC_CI32_MAX_TIMES, XC_IN_CBF16, XC_IN_CF16, XC_IN_CF32, XC_IN_CI8, XC_KERNEL_AUTO,
                   XC_KERNEL_MFMA, XC_KERNEL_VALU, XC_OUT_CF32, XC_OUT_CI32, XC_STAGING_AUTO, XC_STAGING_LDS,
                   XC_STAGING_REGISTERS, XC_PRODUCT_AUTO, XC_PRODUCT_FOUR, XC_PRODUCT_THREE, XC_LAYOUT_TIME_MAJOR,
                   XC_LAYOUT_STATION_MAJOR, XengineError)

__all__ = ["correlate", "correlate_into", "n_baselines", "baseline_index", "tile_cost", "perf_max", "ai_global",
           "flops", "resolve_config", "BatchPlan", "batch_worklist", "autotune", "tune_cache_load", "Server",
           "quantile", "XengineError", "in_type_of", "vis_shape", "Ingest", "transpose_to_time_major", "Pfb",
           "tune_candidates", "tune_bucket"]


def lib():
    return _lib.load()


def n_baselines(n_stations: int) -> int:
    return int(lib().xc_n_baselines(n_stations))


def baseline_index(i: int, j: int) -> int:
    return int(lib().xc_baseline_index(i, j))


def tile_cost(w: int, h: int):
    """(flops, bytes, min_registers) of a w x h tile (Table 1)."""
    f, b, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _lib.check(lib().xc_tile_cost(w, h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(r)))
    return f.value, b.value, r.value


def perf_max(perf_peak: float, arithmetic_intensity: float, bandwidth: float) -> float:
    return float(lib().xc_perf_max(perf_peak, arithmetic_intensity, bandwidth))


def ai_global(n_stations: int) -> float:
    return float(lib().xc_ai_global(n_stations))


def flops(n_stations: int, n_channels: int, n_times: int) -> float:
    return float(lib().xc_flops(n_stations, n_channels, n_times))


PEAK_NAMES = {"f32_mfma16": _lib.XC_PEAK_F32_MFMA16, "f32_mfma32": _lib.XC_PEAK_F32_MFMA32,
              "i8_mfma": _lib.XC_PEAK_I8_MFMA, "f16_mfma": _lib.XC_PEAK_F16_MFMA, "bf16_mfma": _lib.XC_PEAK_BF16_MFMA,
              "f32_fma": _lib.XC_PEAK_F32_FMA, "hbm_copy": _lib.XC_PEAK_HBM_COPY}


def measure_peak(name: str) -> float:
    """Achievable rate of one instruction (TFLOP/s or TOP/s) or of a device
    copy (GB/s) on the current GPU."""
    v = ctypes.c_double()
    _lib.check(lib().xc_measure_peak(PEAK_NAMES[name], ctypes.byref(v)))
    return v.value


def quantile(values, q: float) -> float:
    arr = (ctypes.c_double * len(values))(*values)
    return float(lib().xc_quantile(arr, len(values), q))


def in_type_of(x: torch.Tensor):
    """(xc_in_type, C, T, S, P) of a sample tensor."""
    if x.dtype == torch.complex64:
        if x.dim() != 4:
            raise ValueError("complex64 samples must have shape [C, T, S, P]")
        C, T, S, P = x.shape
        return XC_IN_CF32, C, T, S, P
    kinds = {torch.int8: XC_IN_CI8, torch.float16: XC_IN_CF16, torch.bfloat16: XC_IN_CBF16}
    if x.dtype not in kinds:
        raise TypeError(f"unsupported sample dtype {x.dtype}")
    if x.dim() != 5 or x.shape[-1] != 2:
        raise ValueError(f"{x.dtype} samples must have shape [C, T, S, P, 2] (re, im)")
    C, T, S, P, _ = x.shape
    return kinds[x.dtype], C, T, S, P


def vis_shape(n_channels: int, n_stations: int, out_type: int, n_pol: int = 2):
    B = n_stations * (n_stations + 1) // 2
    return (n_channels, B, n_pol, n_pol) if out_type == XC_OUT_CF32 else (n_channels, B, n_pol, n_pol, 2)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_device(*tensors):
    for t in tensors:
        if not t.is_cuda:
            raise ValueError("the correlator runs on the GPU only: pass device tensors")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _config(config):
    if config is None:
        return None
    if isinstance(config, _lib.XcConfig):
        return config
    return _lib.XcConfig(int(config.get("kernel", 0)), int(config.get("block", 0)),
                         int(config.get("time_chunk", 0)), int(config.get("time_split", 0)),
                         int(config.get("staging", 0)), int(config.get("product", 0)),
                         int(config.get("tile_w", 0)), int(config.get("tile_h", 0)))


def _config_dict(c) -> dict:
    return {"kernel": c.kernel, "block": c.block, "time_chunk": c.time_chunk, "time_split": c.time_split,
            "staging": c.staging, "product": c.product, "tile_w": c.tile_w, "tile_h": c.tile_h}


def resolve_config(x_shape_type, out_type=XC_OUT_CF32, config=None) -> dict:
    """Resolved configuration for (in_type, C, T, S, P) without touching the GPU."""
    in_type, C, T, S, P = x_shape_type
    cfg = _config(config)
    res = _lib.XcConfig()
    _lib.check(lib().xc_resolve_config(ctypes.byref(cfg) if cfg else None, in_type, out_type, S, P, C, T,
                                       ctypes.byref(res)))
    return _config_dict(res)


def correlate_into(x: torch.Tensor, out: torch.Tensor, accumulate: bool = False, stream=None,
                   config=None, split: int = 1, layout: int = XC_LAYOUT_TIME_MAJOR,
                   static_scratch: bool = False) -> torch.Tensor:
    """out (+)= correlation of x; out dtype complex64 (XC_OUT_CF32) or int32 (XC_OUT_CI32).
    split > 1 cuts the integration into that many pieces, one set of
    workgroups each, and adds their partial sums in a fixed order (for
    workloads with few channels and stations); the workspace is a torch
    allocation on the device.  layout = XC_LAYOUT_STATION_MAJOR takes
    complex64 x[C, S, T, 2] (each station's series contiguous) and corner-turns
    it in the kernel's copies into LDS (64-station matrix-core kernel).
    static_scratch = True runs the split through xc_correlate_split_static,
    which allocates nothing: the partial sums go to the library's fixed
    per-device scratch (calls on one device must not overlap)."""
    if layout == XC_LAYOUT_STATION_MAJOR:
        in_type, C, S, T, P = in_type_of(x)      # dims 1 and 2 are (S, T) here
        if split > 1:
            raise ValueError("station-major input is not combined with a split integration")
        out_type = XC_OUT_CI32 if out.dtype == torch.int32 else XC_OUT_CF32
        if tuple(out.shape) != vis_shape(C, S, out_type, P):
            raise ValueError(f"out has shape {tuple(out.shape)}, expected {vis_shape(C, S, out_type, P)}")
        _require_device(x, out)
        cfg = _config(config)
        st = lib().xc_correlate_station_major(ctypes.byref(cfg) if cfg else None, ctypes.c_void_p(x.data_ptr()),
                                              in_type, S, P, C, T, ctypes.c_void_p(out.data_ptr()), out_type,
                                              1 if accumulate else 0, _stream_ptr(stream))
        _lib.check(st)
        return out
    if layout != XC_LAYOUT_TIME_MAJOR:
        raise ValueError(f"unknown layout {layout}")
    in_type, C, T, S, P = in_type_of(x)
    out_type = XC_OUT_CI32 if out.dtype == torch.int32 else XC_OUT_CF32
    if out.dtype not in (torch.int32, torch.complex64):
        raise TypeError("out must be complex64 or int32")
    if tuple(out.shape) != vis_shape(C, S, out_type, P):
        raise ValueError(f"out has shape {tuple(out.shape)}, expected {vis_shape(C, S, out_type, P)}")
    _require_device(x, out)
    cfg = _config(config)
    if static_scratch:
        st = lib().xc_correlate_split_static(ctypes.byref(cfg) if cfg else None, ctypes.c_void_p(x.data_ptr()),
                                             in_type, S, P, C, T, ctypes.c_void_p(out.data_ptr()), out_type,
                                             1 if accumulate else 0, int(split), _stream_ptr(stream))
        _lib.check(st)
        return out
    if split > 1:
        nbytes = lib().xc_correlate_split_bytes(S, P, C, T, split)
        if nbytes < 0:
            raise ValueError("invalid split correlation shape")
        work = torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=x.device)
        if stream is not None:
            work.record_stream(stream)
        st = lib().xc_correlate_split(ctypes.byref(cfg) if cfg else None, ctypes.c_void_p(x.data_ptr()), in_type, S,
                                      P, C, T, ctypes.c_void_p(out.data_ptr()), out_type, 1 if accumulate else 0,
                                      int(split), ctypes.c_void_p(work.data_ptr()), work.numel(), _stream_ptr(stream))
        _lib.check(st)
        return out
    st = lib().xc_correlate_config(ctypes.byref(cfg) if cfg else None, ctypes.c_void_p(x.data_ptr()), in_type, S, P,
                                   C, T, ctypes.c_void_p(out.data_ptr()), out_type, 1 if accumulate else 0,
                                   _stream_ptr(stream))
    _lib.check(st)
    return out


def correlate(x: torch.Tensor, out: torch.Tensor | None = None, accumulate: bool = False, stream=None,
              config=None, out_type: int | None = None, split: int = 1,
              layout: int = XC_LAYOUT_TIME_MAJOR) -> torch.Tensor:
    """Visibilities of samples x.

    x: complex64 [C, T, S, 2], or int8 / float16 / bfloat16 [C, T, S, 2, 2]
    (layout = XC_LAYOUT_STATION_MAJOR: complex64 [C, S, T, 2])
    returns complex64 [C, B, 2, 2] (int8 input: int32 [C, B, 2, 2, 2] unless
    out_type = XC_OUT_CF32).  The paper's correlation[b][c][p][q] order is
    ``out.permute(1, 0, 2, 3)``.
    """
    in_type, C, T, S, P = in_type_of(x)
    if layout == XC_LAYOUT_STATION_MAJOR:
        S, T = T, S
    if out is None:
        if out_type is None:
            out_type = XC_OUT_CI32 if in_type == XC_IN_CI8 else XC_OUT_CF32
        dtype = torch.int32 if out_type == XC_OUT_CI32 else torch.complex64
        alloc = torch.zeros if accumulate else torch.empty
        out = alloc(vis_shape(C, S, out_type, P), dtype=dtype, device=x.device)
    return correlate_into(x, out, accumulate=accumulate, stream=stream, config=config, split=split, layout=layout)


def transpose_to_time_major(x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Station-major device samples x[C][S][T][P] (complex64 [C, S, T, 2], or
    int8 / float16 / bfloat16 [C, S, T, 2, 2]) -> time-major [C, T, S, P] on the
    GPU (Section 4.4's memory-layout transpose)."""
    in_type, C, S, T, P = in_type_of(x)      # dims 1 and 2 are (S, T) here
    shape = (C, T, S) + tuple(x.shape[3:])
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    if tuple(out.shape) != shape or out.dtype != x.dtype:
        raise ValueError(f"out must be {x.dtype} of shape {shape}")
    _require_device(x, out)
    _lib.check(lib().xc_transpose_to_time_major(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                in_type, S, P, C, T, _stream_ptr(stream)))
    return out


class Ingest:
    """Correlation of samples held in host memory: channel groups are copied to
    the device (pinned host memory: asynchronous DMA on a copy stream,
    overlapping the previous group's correlation), transposed on the GPU when
    the host layout is station-major, and correlated into their channels of V
    by the same kernels as device-resident input (Sections 3.6 and 4.4)."""

    def __init__(self, in_type: int, n_stations: int, n_channels: int, n_times: int,
                 layout: int = XC_LAYOUT_TIME_MAJOR, channels_per_group: int = 0):
        h = ctypes.c_void_p()
        _lib.check(lib().xc_ingest_create(in_type, n_stations, 2, n_channels, n_times, layout, channels_per_group,
                                          ctypes.byref(h)))
        self._h = h
        self.in_type, self.layout = in_type, layout
        self.S, self.C, self.T = n_stations, n_channels, n_times
        g, b = ctypes.c_int32(), ctypes.c_int64()
        _lib.check(lib().xc_ingest_info(h, ctypes.byref(g), ctypes.byref(b)))
        self.channels_per_group, self.device_bytes = g.value, b.value

    def host_shape(self):
        mid = (self.T, self.S) if self.layout == XC_LAYOUT_TIME_MAJOR else (self.S, self.T)
        return (self.C,) + mid + ((2,) if self.in_type == XC_IN_CF32 else (2, 2))

    def run(self, x_host: torch.Tensor, out: torch.Tensor | None = None, accumulate: bool = False,
            overlap: bool = True, config=None, stream=None, out_type: int | None = None) -> torch.Tensor:
        """out (+)= correlation of the host samples; enqueued on `stream`.  x_host
        must stay alive and unchanged until the stream has finished the work."""
        dtypes = {XC_IN_CF32: torch.complex64, XC_IN_CI8: torch.int8, XC_IN_CF16: torch.float16,
                  XC_IN_CBF16: torch.bfloat16}
        if x_host.is_cuda or x_host.dtype != dtypes[self.in_type] or tuple(x_host.shape) != self.host_shape():
            raise ValueError(f"x_host must be a host tensor of {dtypes[self.in_type]} {self.host_shape()}")
        if not x_host.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if out is None:
            if out_type is None:
                out_type = XC_OUT_CI32 if self.in_type == XC_IN_CI8 else XC_OUT_CF32
            alloc = torch.zeros if accumulate else torch.empty
            out = alloc(vis_shape(self.C, self.S, out_type), dtype=torch.int32 if out_type == XC_OUT_CI32
                        else torch.complex64, device="cuda")
        out_type = XC_OUT_CI32 if out.dtype == torch.int32 else XC_OUT_CF32
        if tuple(out.shape) != vis_shape(self.C, self.S, out_type):
            raise ValueError(f"out has shape {tuple(out.shape)}, expected {vis_shape(self.C, self.S, out_type)}")
        _require_device(out)
        cfg = _config(config)
        _lib.check(lib().xc_ingest_run(self._h, ctypes.byref(cfg) if cfg else None, ctypes.c_void_p(x_host.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), out_type, 1 if accumulate else 0,
                                       1 if overlap else 0, _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().xc_ingest_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pfb:
    """F-engine: polyphase filter bank of N channels and M taps over each
    station's and polarisation's sample stream z[S][2][n_in] (complex64),
    producing the correlator's input x[N][T][S][2] (complex64), optionally
    weighted per (station, polarisation, channel) for delay or gain
    correction.  ``run`` returns x, which ``correlate`` takes as it is."""

    def __init__(self, n_stations: int, n_channels: int, n_taps: int, n_in: int):
        h = ctypes.c_void_p()
        _lib.check(lib().xc_pfb_create(n_stations, 2, n_channels, n_taps, n_in, ctypes.byref(h)))
        self._h = h
        self.S, self.N, self.M, self.n_in = n_stations, n_channels, n_taps, n_in
        t, b = ctypes.c_int32(), ctypes.c_int64()
        _lib.check(lib().xc_pfb_info(h, ctypes.byref(t), ctypes.byref(b)))
        self.n_frames, self.device_bytes = t.value, b.value

    def out_shape(self, layout: int = XC_LAYOUT_TIME_MAJOR):
        if layout == XC_LAYOUT_STATION_MAJOR:
            return (self.N, self.S, self.n_frames, 2)
        return (self.N, self.n_frames, self.S, 2)

    def run(self, z: torch.Tensor, taps: torch.Tensor, weights: torch.Tensor | None = None,
            out: torch.Tensor | None = None, stream=None, layout: int = XC_LAYOUT_TIME_MAJOR) -> torch.Tensor:
        """layout = XC_LAYOUT_STATION_MAJOR writes x[N][S][T][2] in one kernel,
        for ``correlate(..., layout=XC_LAYOUT_STATION_MAJOR)``."""
        if z.dtype != torch.complex64 or tuple(z.shape) != (self.S, 2, self.n_in):
            raise ValueError(f"z must be complex64 of shape {(self.S, 2, self.n_in)}")
        if taps.dtype != torch.float32 or taps.numel() != self.M * self.N:
            raise ValueError(f"taps must be float32 with {self.M * self.N} values")
        if weights is not None and (weights.dtype != torch.complex64 or tuple(weights.shape) != (self.S, 2, self.N)):
            raise ValueError(f"weights must be complex64 of shape {(self.S, 2, self.N)}")
        if layout not in (XC_LAYOUT_TIME_MAJOR, XC_LAYOUT_STATION_MAJOR):
            raise ValueError(f"unknown layout {layout}")
        shape = self.out_shape(layout)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=z.device)
        if out.dtype != torch.complex64 or tuple(out.shape) != shape:
            raise ValueError(f"out must be complex64 of shape {shape}")
        tensors = [z, taps, out] + ([weights] if weights is not None else [])
        _require_device(*tensors)
        for t in tensors:
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous")
        fn = lib().xc_pfb_run_station_major if layout == XC_LAYOUT_STATION_MAJOR else lib().xc_pfb_run
        _lib.check(fn(self._h, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(taps.data_ptr()),
                      ctypes.c_void_p(weights.data_ptr()) if weights is not None else None,
                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().xc_pfb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_worklist(shapes, block: int, with_bounds: bool = False):
    """Host-side work list [(item, channel, bi, bj), ...] of a launch over a
    batch of (n_stations, n_channels, n_times) shapes; with_bounds also returns
    the start of each XCD's range and the end of the last (9 entries)."""
    n = len(shapes)
    S = (ctypes.c_int32 * n)(*[s[0] for s in shapes])
    C = (ctypes.c_int32 * n)(*[s[1] for s in shapes])
    T = (ctypes.c_int32 * n)(*[s[2] for s in shapes])
    count = lib().xc_batch_worklist(S, C, T, n, block, None, 0, None)
    if count < 0:
        raise ValueError("invalid batch shapes")
    buf = (ctypes.c_int32 * (4 * count))()
    bounds = (ctypes.c_int32 * 9)()
    lib().xc_batch_worklist(S, C, T, n, block, buf, count, bounds)
    units = [tuple(buf[4 * k:4 * k + 4]) for k in range(count)]
    return (units, list(bounds)) if with_bounds else units


class BatchPlan:
    """Many sub-arrays of uneven shape correlated by one launch per kernel
    configuration (one workgroup per unit), replayed from a hipGraph when
    use_graph is true."""

    def __init__(self, samples, outs, accumulate=False, config=None, use_graph=True, stream=None,
                 tune_cache: str | None = None):
        if len(samples) != len(outs) or not samples:
            raise ValueError("need one output per sample block")
        kinds = {in_type_of(x)[0] for x in samples}
        if len(kinds) != 1:
            raise ValueError("all items of a batch share one sample type")
        self.in_type = kinds.pop()
        self.out_type = XC_OUT_CI32 if outs[0].dtype == torch.int32 else XC_OUT_CF32
        items = (_lib.XcSubarray * len(samples))()
        for k, (x, o) in enumerate(zip(samples, outs)):
            _, C, T, S, P = in_type_of(x)
            if tuple(o.shape) != vis_shape(C, S, self.out_type, P):
                raise ValueError(f"item {k}: output shape {tuple(o.shape)} does not match")
            _require_device(x, o)
            items[k] = _lib.XcSubarray(x.data_ptr(), o.data_ptr(), S, C, T)
        self._keep = (list(samples), list(outs))
        cfg = _config(config)
        handle = ctypes.c_void_p()
        _lib.check(lib().xc_batch_plan_create(items, len(samples), 2, self.in_type, self.out_type,
                                              1 if accumulate else 0, ctypes.byref(cfg) if cfg else None,
                                              tune_cache.encode() if tune_cache else None, 1 if use_graph else 0,
                                              _stream_ptr(stream), ctypes.byref(handle)))
        self._h = handle

    @property
    def units(self) -> int:
        return int(lib().xc_batch_plan_units(self._h))

    def run(self, stream=None):
        _lib.check(lib().xc_batch_plan_run(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().xc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(x: torch.Tensor, out: torch.Tensor, cache_path: str | None = None, stream=None):
    """Time every valid configuration for x's shape; returns (config dict, ms).
    Later AUTO calls for the same shape use the winner."""
    in_type, C, T, S, P = in_type_of(x)
    out_type = XC_OUT_CI32 if out.dtype == torch.int32 else XC_OUT_CF32
    _require_device(x, out)
    best = _lib.XcConfig()
    ms = ctypes.c_double()
    _lib.check(lib().xc_autotune(ctypes.c_void_p(x.data_ptr()), in_type, S, P, C, T, ctypes.c_void_p(out.data_ptr()),
                                 out_type, cache_path.encode() if cache_path else None, _stream_ptr(stream),
                                 ctypes.byref(best), ctypes.byref(ms)))
    return _config_dict(best), ms.value


def tune_cache_load(path: str) -> int:
    return int(lib().xc_tune_cache_load(path.encode()))


def tune_candidates(in_type: int) -> list:
    """The auto-tuner's candidate configurations for a sample type, after the
    Table 1 register pruning of the vector-ALU tiles."""
    n = lib().xc_tune_candidates(in_type, None, 0)
    if n < 0:
        raise ValueError(f"invalid in_type {in_type}")
    buf = (_lib.XcConfig * n)()
    lib().xc_tune_candidates(in_type, buf, n)
    return [_config_dict(c) for c in buf]


def tune_bucket(in_type: int, out_type: int, n_stations: int, n_channels: int, n_times: int) -> tuple:
    """The tuning bucket of a shape (shapes with equal buckets share a tuned configuration)."""
    key = (ctypes.c_int32 * 6)()
    _lib.check(lib().xc_tune_bucket(in_type, out_type, n_stations, n_channels, n_times, key))
    return tuple(key)


class _DevicePointer:
    """Exposes a raw device allocation of the library to torch (no copy)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


def device_tensor(ptr: int, shape, dtype: torch.dtype, device="cuda") -> torch.Tensor:
    """A torch view of library-owned device memory (stream ring slots, resident
    integrations); the memory stays owned by the library."""
    typestr = {torch.int8: "|i1", torch.int16: "<i2", torch.int32: "<i4", torch.float32: "<f4", torch.float16: "<f2",
               torch.complex64: "<c8"}[dtype]
    return torch.as_tensor(_DevicePointer(ptr, shape, typestr), device=device)


class Server:
    """Streaming correlator: blocks arrive into a device ring, partial
    integrations stay resident, streams are admitted by device-memory footprint."""

    def __init__(self, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _lib.check(lib().xc_server_create(hbm_budget_bytes, ctypes.byref(h)))
        self._h = h

    @staticmethod
    def desc(n_stations, n_channels, block_times, blocks_per_integration, blocks_per_fold=1, ring_blocks=0,
             in_type=XC_IN_CI8, acc_type=XC_OUT_CI32, block_period_s=0.0, staggered=True, spread_ends=False):
        """Stream descriptor; staggered folds one of k channel groups per block
        (every channel still every k blocks), otherwise all channels every k
        blocks.  spread_ends (staggered only): each group folds what it has
        left of an integration at its next turn instead of all groups at the
        integration's last block."""
        if ring_blocks == 0:
            ring_blocks = 2 * blocks_per_fold
        mode = (2 if spread_ends else 1) if staggered else 0
        return _lib.XcStreamDesc(n_stations, 2, n_channels, block_times, blocks_per_integration, blocks_per_fold,
                                 ring_blocks, in_type, acc_type, mode, block_period_s)

    def set_fold_order(self, one_at_a_time: bool):
        """True: the folds of all streams run one at a time, in enqueue order."""
        _lib.check(lib().xc_server_set_fold_order(self._h, 1 if one_at_a_time else 0))

    def flush(self, sid: int):
        """Folds and publishes what is left of complete integrations (spread ends)."""
        _lib.check(lib().xc_stream_flush(self._h, sid))

    @staticmethod
    def footprint(desc) -> int:
        return int(lib().xc_stream_footprint(ctypes.byref(desc)))

    @staticmethod
    def schedule(desc, n_blocks: int, flush: bool = False):
        """The folds the server enqueues for n_blocks commits (and a flush),
        computed on the host: (folds, published_after), folds as rows
        (trigger block, group, first channel, end channel, first block,
        last block), published_after[j] the block whose commit publishes
        integration j (n_blocks: the flush; -1: not published)."""
        n = ctypes.c_int64()
        n_int = n_blocks // desc.blocks_per_integration + 1
        pub = (ctypes.c_int64 * n_int)()
        _lib.check(lib().xc_stream_schedule(ctypes.byref(desc), n_blocks, 1 if flush else 0, None, 0,
                                            ctypes.byref(n), pub, n_int))
        rows = (ctypes.c_int64 * (6 * max(n.value, 1)))()
        _lib.check(lib().xc_stream_schedule(ctypes.byref(desc), n_blocks, 1 if flush else 0, rows, n.value,
                                            ctypes.byref(n), pub, n_int))
        folds = [tuple(rows[6 * r:6 * r + 6]) for r in range(n.value)]
        return folds, list(pub)

    def open(self, desc) -> int:
        sid = ctypes.c_int32()
        _lib.check(lib().xc_stream_open(self._h, ctypes.byref(desc), ctypes.byref(sid)))
        return sid.value

    def acquire(self, sid: int) -> int:
        p = ctypes.c_void_p()
        _lib.check(lib().xc_stream_acquire(self._h, sid, ctypes.byref(p)))
        return p.value

    def commit(self, sid: int, arrival_ns: int, producer_stream=None):
        """Marks the acquired slot filled.  With producer_stream (a torch
        stream), the folds wait for the work enqueued on it so far instead of
        the slot having to be complete already."""
        if producer_stream is None:
            _lib.check(lib().xc_stream_commit(self._h, sid, arrival_ns))
        else:
            _lib.check(lib().xc_stream_commit_after(self._h, sid, arrival_ns, _stream_ptr(producer_stream)))

    def integration(self, sid: int, k: int):
        """(device pointer, ready event handle) of integration k."""
        p, ev = ctypes.c_void_p(), ctypes.c_void_p()
        _lib.check(lib().xc_stream_integration(self._h, sid, k, ctypes.byref(p), ctypes.byref(ev)))
        return p.value, ev.value

    def wait_integration(self, sid: int, k: int, stream=None) -> int:
        """Makes `stream` (default: the current torch stream) wait for
        integration k without blocking the host; returns its device pointer."""
        p, ev = self.integration(sid, k)
        _lib.check(lib().xc_wait_event(ctypes.c_void_p(ev), _stream_ptr(stream)))
        return p

    def release(self, sid: int, k: int, stream=None):
        """The work enqueued on `stream` so far is the last that reads
        integration k: the fold that overwrites it waits for that work."""
        _lib.check(lib().xc_stream_release(self._h, sid, k, _stream_ptr(stream)))

    def hold(self, sid: int, max_wait_s: float):
        _lib.check(lib().xc_stream_hold(self._h, sid, max_wait_s))

    def resume(self, sid: int):
        _lib.check(lib().xc_stream_resume(self._h, sid))

    def latest(self, sid: int):
        p = ctypes.c_void_p()
        seq = ctypes.c_int64()
        _lib.check(lib().xc_stream_latest(self._h, sid, ctypes.byref(p), ctypes.byref(seq)))
        return p.value, seq.value

    def stats(self, sid: int) -> dict:
        s = _lib.XcLatencyStats()
        _lib.check(lib().xc_stream_stats(self._h, sid, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _lib.XcLatencyStats._fields_}

    def reset_stats(self, sid: int):
        _lib.check(lib().xc_stream_reset_stats(self._h, sid))

    def close_stream(self, sid: int):
        _lib.check(lib().xc_stream_close(self._h, sid))

    def close(self):
        if getattr(self, "_h", None):
            lib().xc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
