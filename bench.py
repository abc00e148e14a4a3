"""Benchmark of the correlator X-engine on one MI355X.

Default workload: the LOFAR-scale correlation of Section 2 -- 64 dual-polarised
stations, 256 channels, integrations of 768 complex-float32 samples (noise plus
three point sources).  One step = one correlation of the whole block (every
channel, every station pair, all four polarisation pairs) with the samples
already resident in device memory.  Throughput is counted as 8 flops per
complex multiply-accumulate, 32 per baseline per sample.  Before the W warm-up
steps an untimed settle phase repeats the step for 0.2 s so that the GPU runs at
its steady clock (a correlator runs continuously); the timed region is exactly K
steps.

Prints one JSON line with the headline value, the roofline position of the
kernel, a CPU baseline (the oracle on the host cores, on a bounded sample of
the same workload) and the other kernel paths on the 256-station int8
workload for comparison (MFMA int8 / f16 / bf16 / f32 against the FP32
vector-ALU form on the same values).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp32_mfma_TF": 157.3,
    "fp16_mfma_TF": 2500.0,
    "bf16_mfma_TF": 2500.0,
    "int8_mfma_TOPS": 5000.0,
    "fp32_valu_TF": 157.3,
}
_CSRC = "paper_1702_00844_amd/csrc/"
# the sources each kernel family is compiled from
KERNEL_SOURCES = {
    "valu": [_CSRC + "valu.hip", _CSRC + "common.h"],
    "mfma": [_CSRC + "mfma.hip", _CSRC + "mfma_parts.h", _CSRC + "common.h"],
    "mfma16": [_CSRC + "mfma16.hip", _CSRC + "lds_dma.h", _CSRC + "common.h"],
    "dma": [_CSRC + "mfma_dma.hip", _CSRC + "lds_dma.h", _CSRC + "mfma_parts.h", _CSRC + "common.h"],
    "pfb": [_CSRC + "pfb.hip", _CSRC + "transpose.h", _CSRC + "common.h"],
}


def code_text(src: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed to one
    space: what a change must touch to change the compiled kernel."""
    out, i, n = [], 0, len(src)
    while i < n:
        ch = src[i]
        if ch in "\"'":                       # string or character literal, kept whole
            j = i + 1
            while j < n and src[j] != ch:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def source_sha(kind: str) -> str:
    """Hash of a kernel's sources, comments and layout aside."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, path), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(key: str, kind: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, or None if
    absent or taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    ent = table.get(key)
    if not ent or ent.get("source_sha") != source_sha(kind):
        return None
    return ent.get("bytes_per_launch")


def executed_flops_mfma16(S, C, T, time_split, product):
    """Matrix-core flops the 16 x 16 FP32 kernel issues for one launch: per
    channel, each diagonal 64-station block pair runs 36 of its 8 x 8 tiles of
    16 x 16 (row, column) pairs and each off-diagonal pair all 64, over the
    time steps rounded up to whole chunks (32 or 16 off the diagonal, twice
    that on it, for two or one time groups); a tile costs 2048 flops per time
    step with four real products (four 16x16x4 MFMAs per four time steps) and
    1536 with three."""
    nb = (S + 63) // 64
    kt_off = 32 if time_split == 2 else 16
    kt_diag = 2 * kt_off
    pad = lambda kt: (T + kt - 1) // kt * kt
    per_t = 1536 if product == 2 else 2048
    tiles_t = nb * 36 * pad(kt_diag) + nb * (nb - 1) // 2 * 64 * pad(kt_off)
    return float(C) * tiles_t * per_t


def executed_flops_mfma32_b64(S, C, T, chunk):
    """Matrix-core flops the int8 / 16-bit kernels on 64-station blocks issue
    for one launch: a block pair is a 128 x 128 square of (station, pol) rows
    held by four waves as 2 x 2 tiles of 32 x 32; a wave with any tile on or
    above the diagonal computes all four (on a diagonal pair three of the four
    waves run: 12 tiles), an off-diagonal pair runs 16; a tile costs two MFMAs
    (real and imaginary parts) over K = 2 values per time step, 8192 flops per
    time step (the same 8 flops per complex multiply-accumulate as the
    algorithmic count), over the time steps rounded up to whole chunks."""
    nb = (S + 63) // 64
    tiles = nb * 12 + nb * (nb - 1) // 2 * 16
    return float(C) * tiles * 8192 * ((T + chunk - 1) // chunk * chunk)


def executed_flops_valu(S, C, T, tile_w, tile_h, chunk):
    """Vector-ALU flops for one launch: 32-station block pairs, one lane per
    tile_w x tile_h tile of station pairs; on a diagonal pair the tiles wholly
    below the diagonal are idle, the others compute every pair of their tile;
    32 flops per station pair and time step, time rounded up to whole chunks."""
    nb = (S + 31) // 32
    ti, tj = 32 // tile_w, 32 // tile_h
    diag_tiles = sum(1 for a in range(ti) for b in range(tj) if not (a * tile_w > b * tile_h + tile_h - 1))
    pairs = nb * diag_tiles * tile_w * tile_h + nb * (nb - 1) // 2 * 1024
    return float(C) * pairs * 32 * ((T + chunk - 1) // chunk * chunk)


def cpu_info():
    """Model, sockets and logical CPUs of the host (from /proc/cpuinfo)."""
    model, phys = None, set()
    n = 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and model is None:
                    model = v.strip()
                elif k == "physical id":
                    phys.add(v.strip())
                elif k == "processor":
                    n += 1
    except OSError:
        pass
    return {"cpu_model": model, "sockets": len(phys) or None, "logical_cpus": n or os.cpu_count()}


def time_launches(fn, steps: int, warmup: int, stream, settle_s: float = 0.2):
    """ms per launch of fn over `steps` launches, after `settle_s` seconds of
    untimed launches (the GPU's clock ramps up over the first few hundred
    microseconds of a busy period: a 0.73 ms int8 launch timed from idle
    measures 0.8-0.9 ms) and `warmup` more."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle_s:
        fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per launch, measured on the launch stream


def cpu_baseline(x_host_fn, n_channels_total: int, flops_per_channel: float, budget_s: float = 12.0,
                 in_kind: str = "cf32"):
    """Time the oracle on a bounded sample of the workload: channels are
    independent, so the sample is the first n channels, repeated until about
    budget_s seconds of CPU work have been timed."""
    import numpy as np
    import oracle
    lib = oracle.load()

    def run(xs):
        if in_kind == "ci8":
            return oracle.correlate_i64(xs, lib)
        if np.iscomplexobj(xs):
            return oracle.correlate_f64(xs, lib)
        return oracle.correlate_f64(xs[..., 0] + 1j * xs[..., 1], lib)

    threads = oracle.threads()
    n = min(n_channels_total, max(1, threads))
    xs = x_host_fn(n)
    t0 = time.perf_counter()
    run(xs)
    t1 = time.perf_counter() - t0
    # grow the channel count (up to the whole workload), then repeat passes
    if t1 < budget_s:
        n = min(n_channels_total, max(n, int(n * budget_s / max(t1, 1e-3))))
        xs = x_host_fn(n)
    passes, dt = 0, 0.0
    while dt < budget_s or passes == 0:
        t0 = time.perf_counter()
        run(xs)
        dt += time.perf_counter() - t0
        passes += 1
        if dt > budget_s / 2 and passes >= 1 and dt + dt / passes > 2.5 * budget_s:
            break
    info = cpu_info()
    return {"value": flops_per_channel * n * passes / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} of {n_channels_total} channels of the same workload x {passes} passes "
                      f"({dt:.1f} s of wall time on {threads} OpenMP threads, FP64/int64 oracle, OpenMP over "
                      f"channels)",
            "cpu_model": info["cpu_model"], "sockets": info["sockets"], "logical_cpus": info["logical_cpus"]}


def oracle_timing(xe, inputs, torch, budget_full_s=12.0):
    """The oracle on the host cores (all OpenMP threads) for every workload,
    best of three wall-time passes, excluding data generation, counted with the
    same 8 flops per complex multiply-accumulate.  The 8-, 64- and 256-station
    workloads run in full (the 256-station one once only if a pass takes longer
    than budget_full_s); the batch and streaming workloads run on a seeded
    subset of 8 channels per sub-array / stream, scaled by channel count
    (channels are independent) and labelled extrapolated."""
    import numpy as np
    import oracle
    lib = oracle.load()

    def best(fn, reps=3, cap=None):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
            if cap is not None and ts[-1] > cap:
                break
        return min(ts), len(ts)

    out = dict(cpu_info(), threads=oracle.threads())
    rows = {}
    x1 = inputs.cn_gaussian(16, 256, 8, seed=1).numpy()
    t, n = best(lambda: oracle.correlate_f64(x1, lib))
    rows["small_8st"] = {"seconds": t, "passes": n, "GFLOP/s": xe.flops(8, 16, 256) / t / 1e9, "extent": "full"}
    x2, _ = inputs.point_sources(256, 768, 64, seed=2)
    x2 = x2.numpy()
    t, n = best(lambda: oracle.correlate_f64(x2, lib))
    rows["lofar64"] = {"seconds": t, "passes": n, "GFLOP/s": xe.flops(64, 256, 768) / t / 1e9, "extent": "full"}
    del x2
    x3 = inputs.ci8_gaussian(1024, 1024, 256, seed=3).numpy()
    t, n = best(lambda: oracle.correlate_i64(x3, lib), cap=budget_full_s)
    rows["p256_int8"] = {"seconds": t, "passes": n, "GFLOP/s": xe.flops(256, 1024, 1024) / t / 1e9, "extent": "full"}
    del x3
    # batch draw: 8 channels of each sub-array, scaled to the draw's channel counts
    shapes = inputs.subarray_shapes(32, seed=4)
    tot_t, tot_f = 0.0, 0.0
    for k, (S, C, T) in enumerate(shapes):
        xs = inputs.ci8_gaussian(8, T, S, seed=1000 + k).numpy()
        t, _ = best(lambda: oracle.correlate_i64(xs, lib), reps=1)
        tot_t += t * C / 8
        tot_f += xe.flops(S, C, T)
    rows["batch32_int8"] = {"seconds": tot_t, "GFLOP/s": tot_f / tot_t / 1e9,
                            "extent": "extrapolated from 8 channels per sub-array"}
    # streaming: one 256-sample block of 512 stations, 8 of 4096 channels
    x5 = inputs.ci8_gaussian(8, 256, 512, seed=5).numpy()
    t, n = best(lambda: oracle.correlate_i64(x5, lib))
    per_block = t * 4096 / 8
    rows["stream512_int8_per_block"] = {"seconds": per_block, "GFLOP/s": xe.flops(512, 4096, 256) / per_block / 1e9,
                                        "realtime_fraction": round((256 / 49152.0) / per_block, 6),
                                        "extent": "extrapolated from 8 of 4096 channels"}
    for r in rows.values():
        r["seconds"] = round(r["seconds"], 4)
        r["GFLOP/s"] = round(r["GFLOP/s"], 2)
    out["workloads"] = rows
    out["timing"] = "wall time, best of up to 3 passes, data generation excluded"
    return out


def precision_bench(xe, inputs, torch, dev):
    """16-bit samples on Gaussian float data, per (workload, type): total error
    (against the oracle on the unrounded complex64 samples: input rounding plus
    accumulation) and accumulation-only error (against the oracle on the
    rounded samples), normwise and as the largest Cauchy-Schwarz-normalised
    element error.  Channel subsets are labelled."""
    import numpy as np
    import oracle
    lib = oracle.load()

    def errs(got, ref, S):
        nw = float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
        idx = [s * (s + 1) // 2 + s for s in range(S)]
        pw = np.stack([ref[:, idx, 0, 0].real, ref[:, idx, 1, 1].real], axis=-1)      # [C, S, 2]
        jj = np.concatenate([np.full(j + 1, j) for j in range(S)])
        ii = np.concatenate([np.arange(j + 1) for j in range(S)])
        scale = np.sqrt(pw[:, ii][:, :, :, None] * pw[:, jj][:, :, None, :])           # [C, B, 2, 2]
        return nw, float(np.max(np.abs(got - ref) / scale))

    res = {}
    for name, (S, C, T, Csub) in {"lofar64": (64, 256, 768, 256), "p256": (256, 1024, 1024, 16),
                                  "stream512_block": (512, 4096, 256, 4)}.items():
        x = inputs.cn_gaussian(Csub, T, S, seed=30 + S, device=dev)
        ref_total = oracle.correlate_f64(x.cpu().numpy(), lib)
        row = {"channels": f"{Csub} of {C}" if Csub < C else "all", "S": S, "T": T}
        for dt, tname in ((torch.float16, "f16"), (torch.bfloat16, "bf16")):
            xr = torch.view_as_real(x).to(dt).contiguous()                                  # [C, T, S, 2, 2]
            v = xe.correlate(xr)
            torch.cuda.synchronize()
            got = v.cpu().numpy().astype(np.complex128)
            f = xr.cpu().to(torch.float64).numpy()
            ref_acc = oracle.correlate_f64(f[..., 0] + 1j * f[..., 1], lib)
            tot = errs(got, ref_total, S)
            acc = errs(got, ref_acc, S)
            row[tname] = {"total_normwise": float(f"{tot[0]:.3e}"), "total_worst_cs": float(f"{tot[1]:.3e}"),
                          "accumulation_normwise": float(f"{acc[0]:.3e}"),
                          "accumulation_worst_cs": float(f"{acc[1]:.3e}")}
        res[name] = row
    return res


WORKLOADS = {
    # name: (S, C, T, sample type, kernel config or None)
    "lofar64": (64, 256, 768, "cf32", None),
    "p256_ci8": (256, 1024, 1024, "ci8", None),
    "p256_cf16": (256, 1024, 1024, "cf16", None),
    "p256_cbf16": (256, 1024, 1024, "cbf16", None),
    "p256_cf32_mfma": (256, 1024, 1024, "cf32", {"kernel": 2}),
    "p256_cf32_valu": (256, 1024, 1024, "cf32", {"kernel": 1}),
}
DESCRIPTIONS = {
    "lofar64": "lofar64: 64 stations x 2 pol, 256 channels, 768 samples, complex64 CN(0,1) noise + 3 point sources",
    "p256": "p256: 256 stations x 2 pol, 1024 channels, 1024 samples, complex int8 clamp(rint(N(0,32^2)))",
}


def make_input(xe, inputs, torch, dev, name):
    S, C, T, kind, cfg = WORKLOADS[name]
    if name == "lofar64":
        x, _ = inputs.point_sources(C, T, S, seed=2, device=dev)
    else:
        xi = inputs.ci8_gaussian(C, T, S, seed=3, device=dev)
        x = {"ci8": lambda: xi, "cf16": lambda: xi.to(torch.float16), "cbf16": lambda: xi.to(torch.bfloat16),
             "cf32": lambda: torch.view_as_complex(xi.to(torch.float32))}[kind]()
    ot = xe.XC_OUT_CI32 if kind == "ci8" else xe.XC_OUT_CF32
    out = torch.empty(xe.vis_shape(C, S, ot), dtype=torch.int32 if kind == "ci8" else torch.complex64, device=dev)
    return x, out, ot


def copy_calibration(steps):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="lofar64")
    ap.add_argument("--kernel", choices=["auto", "mfma", "valu"], default="auto",
                    help="kernel family for the lofar64 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the other kernel paths")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--batch", choices=["none", "ci8", "cf32", "both"], default="both",
                    help="also time the 32-sub-array batch plan")
    ap.add_argument("--stream-ks", default="1,2,4,8",
                    help="fold lengths k of the one-stream runs (deadline k x period; '' to skip)")
    ap.add_argument("--stream-blocks", type=int, default=1000,
                    help="blocks per stream after one warm-up integration")
    ap.add_argument("--stream-fold", type=int, default=8, help="k of the all-channel and multi-stream runs")
    ap.add_argument("--stream-ref-blocks", type=int, default=384,
                    help="blocks of the all-channels-at-once run at --stream-fold (0: skip)")
    ap.add_argument("--stream-multi", type=int, default=5,
                    help="streams requested for the admission/multi-stream run at --stream-fold (0: skip)")
    ap.add_argument("--stream-multi-blocks", type=int, default=384)
    ap.add_argument("--stream-two-k", type=int, default=16,
                    help="k of the two-stream real-time run (spread ends, folds in order; 0: skip)")
    ap.add_argument("--no-oracle-timing", action="store_true", help="skip the oracle timing on every workload")
    ap.add_argument("--no-precision", action="store_true", help="skip the 16-bit error measurement")
    ap.add_argument("--no-fengine", action="store_true", help="skip the filter-bank measurement")
    ap.add_argument("--no-small-launch", action="store_true", help="skip the 8-station launch-latency measurement")
    ap.add_argument("--paths-steps", type=int, default=10, help="timed launches per 256-station kernel path")
    ap.add_argument("--stream-only", action="store_true", help="run only the streaming measurements")
    ap.add_argument("--batch-only", action="store_true", help="run only the batch measurement")
    ap.add_argument("--no-ingest", action="store_true", help="skip the host-ingest measurement")
    ap.add_argument("--ingest-only", action="store_true", help="run only the host-ingest measurement")
    ap.add_argument("--fengine-only", action="store_true", help="run only the filter-bank measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this correlator runs on one GPU: channels would shard across GPUs, "
                                   "but no multi-GPU path exists"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.steps)
        return

    import torch
    import paper_1702_00844_amd as xe
    from paper_1702_00844_amd import inputs

    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    if args.stream_only:
        print(json.dumps(stream_all(xe, inputs, torch, args)), flush=True)
        return
    if args.fengine_only:
        print(json.dumps({"fengine": fengine_bench(xe, inputs, torch, dev, stream),
                          "small_launch": small_launch_bench(xe, inputs, torch, dev, stream)}), flush=True)
        return
    if args.ingest_only:
        print(json.dumps({"ingest": ingest_bench(xe, inputs, torch, dev, stream)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({k: batch_bench(xe, inputs, torch, dev, stream, k)
                          for k in (["ci8", "cf32"] if args.batch == "both" else [args.batch])}), flush=True)
        return
    S, C, T, kind_in, cfg = WORKLOADS[args.workload]
    if args.workload == "lofar64" and args.kernel != "auto":
        cfg = {"mfma": {"kernel": xe.XC_KERNEL_MFMA}, "valu": {"kernel": xe.XC_KERNEL_VALU}}[args.kernel]
    x, out, out_type = make_input(xe, inputs, torch, dev, args.workload)
    in_type = xe.in_type_of(x)[0]
    resolved = xe.resolve_config((in_type, C, T, S, 2), out_type, config=cfg)
    kind = "mfma" if resolved["kernel"] == xe.XC_KERNEL_MFMA else "valu"
    src_kind = kind
    if kind == "mfma" and resolved["block"] == 64:
        src_kind = "mfma16" if kind_in == "cf32" else ("dma" if resolved["staging"] == xe.XC_STAGING_LDS else "mfma")

    def step():
        xe.correlate_into(x, out, config=cfg, stream=stream)

    # untimed settle phase (steady clock), then the W warm-up steps
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < 0.2:
        for _ in range(16):
            step()
        torch.cuda.synchronize()
    # timed region: synchronise, K steps, synchronise (one GPU: no barrier partner)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms_launch = e0.elapsed_time(e1) / args.steps
    flops = xe.flops(S, C, T)
    value = flops * args.steps / t_wall / 1e12
    achieved = flops / (ms_launch * 1e-3) / 1e12
    peak_key = {"cf32": "fp32_mfma_TF" if kind == "mfma" else "fp32_valu_TF", "ci8": "int8_mfma_TOPS",
                "cf16": "fp16_mfma_TF", "cbf16": "bf16_mfma_TF"}[kind_in]
    peak = PEAKS[peak_key]
    traffic_key = f"{args.workload}_{src_kind}_b{resolved['block']}"
    peak_probe = {"cf32": "f32_mfma16" if src_kind == "mfma16" else ("f32_mfma32" if kind == "mfma" else "f32_fma"),
                  "ci8": "i8_mfma", "cf16": "f16_mfma", "cbf16": "bf16_mfma"}[kind_in]
    achievable = xe.measure_peak(peak_probe)
    roofline = {"bound": "mfma" if kind == "mfma" else "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": load_traffic(traffic_key, src_kind),
                "kernel": src_kind, "ms_per_launch": round(ms_launch, 5),
                "algorithmic_flops_per_launch": flops,
                "peak_achievable": round(achievable, 1), "frac_of_achievable": round(achieved / achievable, 4),
                "achievable_probe": peak_probe}
    if src_kind == "mfma16":
        # what the matrix cores actually execute (tiles below the diagonal of
        # diagonal block pairs included; three or four real products)
        ex = executed_flops_mfma16(S, C, T, resolved["time_split"], resolved["product"])
        roofline.update({"products": 3 if resolved["product"] == xe.XC_PRODUCT_THREE else 4,
                         "executed_flops_per_launch": ex,
                         "executed_TFLOP/s": round(ex / (ms_launch * 1e-3) / 1e12, 2),
                         "executed_frac": round(ex / (ms_launch * 1e-3) / 1e12 / peak, 4),
                         "executed_frac_of_achievable": round(ex / (ms_launch * 1e-3) / 1e12 / achievable, 4)})
    dtype = {"cf32": "f32", "ci8": "i8->i32", "cf16": "f16->f32", "cbf16": "bf16->f32"}[kind_in]
    desc = DESCRIPTIONS["lofar64" if args.workload == "lofar64" else "p256"]
    res = {"metric": "visibility TFLOP/s (8 flop/CMAC) + % roofline, FP32 vs MFMA; stream p99",
           "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_wall / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": desc, "n_stations": S, "n_channels": C, "n_times": T, "kernel": resolved},
           "roofline": roofline}

    if not args.no_compare and args.workload == "lofar64":
        del x, out
        torch.cuda.empty_cache()
        res["paths"] = compare_paths(xe, inputs, torch, dev, stream, steps=args.paths_steps)

    if not args.no_compare and args.workload == "lofar64":
        if args.batch != "none":
            res["batch"] = {k: batch_bench(xe, inputs, torch, dev, stream, k)
                            for k in (["ci8", "cf32"] if args.batch == "both" else [args.batch])}
        res.update(stream_all(xe, inputs, torch, args))
        if not args.no_ingest:
            res["ingest"] = ingest_bench(xe, inputs, torch, dev, stream)
        if not args.no_fengine:
            res["fengine"] = fengine_bench(xe, inputs, torch, dev, stream)
        if not args.no_small_launch:
            res["small_launch"] = small_launch_bench(xe, inputs, torch, dev, stream)
        if not args.no_precision:
            res["precision"] = precision_bench(xe, inputs, torch, dev)
        if not args.no_oracle_timing:
            res["oracle_timing"] = oracle_timing(xe, inputs, torch)

    if not args.no_cpu_baseline:
        xh = None

        def host_sample(n):
            nonlocal xh
            if xh is None:
                xh = make_input(xe, inputs, torch, "cpu", args.workload)[0]
            return xh[:n].numpy() if xh.dtype in (torch.complex64, torch.int8) else xh[:n].to(torch.float64).numpy()
        res["cpu_baseline"] = cpu_baseline(host_sample, C, flops / C, in_kind=kind_in)
    print(json.dumps(res), flush=True)


def compare_paths(xe, inputs, torch, dev, stream, steps=10):
    """Every kernel path on the 256-station, 1024-channel, 1024-sample workload
    with complex-int8 values (exact in every input type, so the FP32 and MFMA
    forms are compared at the same, exact, accuracy).  Each path gets a
    roofline object: the roof is min(compute peak, algorithmic intensity x
    8 TB/s); frac is the algorithmic bandwidth over 8 TB/s for an HBM-bound
    path and the executed flop rate over the compute peak otherwise (both at
    most 1 for a physical kernel), with the algorithmic and executed rates,
    the measured achievable peak of the instruction and the counter traffic
    (profiles/traffic.json, null if the kernel changed since)."""
    out = {}
    S, C, T = 256, 1024, 1024
    xi = inputs.ci8_gaussian(C, T, S, seed=3, device=dev)
    flops = xe.flops(S, C, T)
    hbm_in = {"ci8": C * T * S * 4, "cf16": C * T * S * 8, "cbf16": C * T * S * 8, "cf32": C * T * S * 16}
    vis_bytes = C * (S * (S + 1) // 2) * 4 * 8
    cases = [("int8_mfma", "ci8", None, "int8_mfma_TOPS", "i8_mfma", "p256_ci8_dma_b64", "dma"),
             ("f16_mfma", "cf16", None, "fp16_mfma_TF", "f16_mfma", "p256_cf16_dma_b64", "dma"),
             ("bf16_mfma", "cbf16", None, "bf16_mfma_TF", "bf16_mfma", "p256_cbf16_dma_b64", "dma"),
             ("f32_mfma", "cf32", {"kernel": xe.XC_KERNEL_MFMA}, "fp32_mfma_TF", "f32_mfma16",
              "p256_cf32_mfma_mfma16_b64", "mfma16"),
             ("f32_mfma_4products", "cf32", {"kernel": xe.XC_KERNEL_MFMA, "product": xe.XC_PRODUCT_FOUR},
              "fp32_mfma_TF", "f32_mfma16", "p256_cf32_mfma4_mfma16_b64", "mfma16"),
             ("f32_valu", "cf32", {"kernel": xe.XC_KERNEL_VALU}, "fp32_valu_TF", "f32_fma", "p256_cf32_valu_valu_b32",
              "valu")]
    probes = {}
    for name, kind, cfg, peak_key, probe, traffic_key, src in cases:
        if kind == "ci8":
            x = xi
        elif kind == "cf16":
            x = xi.to(torch.float16)
        elif kind == "cbf16":
            x = xi.to(torch.bfloat16)
        else:
            x = torch.view_as_complex(xi.to(torch.float32))
        ot = xe.XC_OUT_CI32 if kind == "ci8" else xe.XC_OUT_CF32
        o = torch.empty(xe.vis_shape(C, S, ot), dtype=torch.int32 if kind == "ci8" else torch.complex64, device=dev)
        r = xe.resolve_config((xe.in_type_of(x)[0], C, T, S, 2), ot, config=cfg)
        ms = time_launches(lambda: xe.correlate_into(x, o, config=cfg, stream=stream), steps, 2, stream)
        sec = ms * 1e-3
        tf = flops / sec / 1e12
        byts = hbm_in[kind] + vis_bytes
        ai = flops / byts
        peak = PEAKS[peak_key]
        hbm_roof = ai * PEAKS["hbm_GBs"] / 1e3
        roof = min(peak, hbm_roof)
        if src == "mfma16":
            ex = executed_flops_mfma16(S, C, T, r["time_split"], r["product"])
        elif src == "valu":
            ex = executed_flops_valu(S, C, T, r["tile_w"], r["tile_h"], r["time_chunk"])
        else:
            ex = executed_flops_mfma32_b64(S, C, T, r["time_chunk"])
        if probe not in probes:
            probes[probe] = xe.measure_peak(probe)
        bound = "hbm" if hbm_roof < peak else ("alu" if src == "valu" else "mfma")
        frac = (byts / sec / 1e9 / PEAKS["hbm_GBs"]) if bound == "hbm" else (ex / sec / 1e12 / peak)
        out[name] = {"workload": "256 stations, 1024 channels, 1024 samples (int8 values)", "config": r,
                     "ms": round(ms, 4), "TFLOP/s": round(tf, 2),
                     "roofline": {"bound": bound, "achieved": round(tf, 2), "peak": round(roof, 1),
                                  "unit": "TFLOP/s", "frac": round(frac, 4),
                                  "traffic": load_traffic(traffic_key, src) if traffic_key else None,
                                  "compute_peak": peak, "hbm_roof": round(hbm_roof, 1),
                                  "algorithmic_intensity_flop_per_B": round(ai, 1),
                                  "algorithmic_bytes": byts, "algorithmic_GB/s": round(byts / sec / 1e9, 1),
                                  "executed_flops_per_launch": ex,
                                  "executed_TFLOP/s": round(ex / sec / 1e12, 2),
                                  "executed_frac_of_compute_peak": round(ex / sec / 1e12 / peak, 4),
                                  "peak_achievable": round(probes[probe], 1), "achievable_probe": probe,
                                  "executed_frac_of_achievable": round(ex / sec / 1e12 / probes[probe], 4)}}
        del x, o
    torch.cuda.empty_cache()
    return out


def batch_bench(xe, inputs, torch, dev, stream, kind, steps=5):
    """32 sub-arrays of uneven shape (stations uniform in [24, 576], channels
    uniform in [16, 1024], 768 samples) as one graph-replayed batch plan,
    against one xc_correlate launch per sub-array."""
    shapes = inputs.subarray_shapes(32, seed=4)
    xs, outs = [], []
    for k, (S, C, T) in enumerate(shapes):
        if kind == "ci8":
            xs.append(inputs.ci8_gaussian(C, T, S, seed=1000 + k, device=dev))
            outs.append(torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CI32), dtype=torch.int32, device=dev))
        else:
            xs.append(inputs.cn_gaussian(C, T, S, seed=1000 + k, device=dev))
            outs.append(torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=dev))
    flops = sum(xe.flops(S, C, T) for S, C, T in shapes)
    plan = xe.BatchPlan(xs, outs, use_graph=True, stream=stream)
    ms_plan = time_launches(lambda: plan.run(stream), steps, 1, stream)
    # tuned per shape bucket (the tuner runs on the first item of each bucket
    # the cache file lacks; the file is scratch, kept for this run only)
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.jsonl")
        t0 = time.perf_counter()
        tplan = xe.BatchPlan(xs, outs, use_graph=True, stream=stream, tune_cache=cache)
        tune_s = time.perf_counter() - t0
        ms_tuned = time_launches(lambda: tplan.run(stream), steps, 1, stream)
        with open(cache) as f:
            tuned = [json.loads(l) for l in f if l.strip()]
        tplan.close()

    def each():
        for x, o in zip(xs, outs):
            xe.correlate_into(x, o, stream=stream)
    ms_each = time_launches(each, steps, 1, stream)
    n_units = plan.units
    plan.close()
    in_bytes = sum(x.numel() * x.element_size() for x in xs)
    out_bytes = sum(o.numel() * o.element_size() for o in outs)
    del xs, outs
    torch.cuda.empty_cache()
    return {"workload": "32 sub-arrays, stations U[24,576], channels U[16,1024], 768 samples, "
                        + ("complex int8" if kind == "ci8" else "complex64 CN(0,1)"),
            "units": n_units, "algorithmic_flops": flops, "in_GB": round(in_bytes / 1e9, 2),
            "out_GB": round(out_bytes / 1e9, 2),
            "batch_graph_ms": round(ms_plan, 3), "batch_TFLOP/s": round(flops / ms_plan / 1e9, 1),
            "tuned_batch_graph_ms": round(ms_tuned, 3), "tuned_batch_TFLOP/s": round(flops / ms_tuned / 1e9, 1),
            "tuned_buckets": len(tuned), "tuning_s": round(tune_s, 1),
            "tuned_choices": sorted({(t["kernel"], t["block"], t["time_split"], t["staging"], t["product"],
                                      t["tile_w"], t["tile_h"]) for t in tuned}),
            "per_item_launches_ms": round(ms_each, 3), "per_item_TFLOP/s": round(flops / ms_each / 1e9, 1)}


def ingest_bench(xe, inputs, torch, dev, stream, reps=5):
    """Host ingest (Sections 3.6 and 4.4): the lofar64 block (complex float32)
    and the p256 block (complex int8) held in pinned host memory, copied to the
    device group by group and correlated.  Reports the pinned host-to-device
    bandwidth, perf_max,global = AI_global x that bandwidth, the end-to-end
    rate with copies overlapped (async) or in order with the computation
    (sync), station-major input transposed on the GPU, the transpose's own
    device bandwidth, and how much a concurrent copy slows the kernel."""
    out = {}

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    for name, S, C, T, kind in [("lofar64_cf32", 64, 256, 768, "cf32"), ("p256_ci8", 256, 1024, 1024, "ci8")]:
        if kind == "cf32":
            x, _ = inputs.point_sources(C, T, S, seed=2, device=dev)
            in_type, sample = xe.XC_IN_CF32, 16
        else:
            x = inputs.ci8_gaussian(C, T, S, seed=3, device=dev)
            in_type, sample = xe.XC_IN_CI8, 4
        host_tm = x.cpu().pin_memory()
        flops = xe.flops(S, C, T)
        nbytes = C * T * S * sample
        ai_global = flops / nbytes
        dev_buf = torch.empty_like(x)
        h2d_ms = timed(lambda: dev_buf.copy_(host_tm, non_blocking=True), reps)
        h2d = nbytes / (h2d_ms * 1e-3) / 1e9
        o = torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CI32 if kind == "ci8" else xe.XC_OUT_CF32),
                        dtype=torch.int32 if kind == "ci8" else torch.complex64, device=dev)
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < 0.2:       # steady clock, as for the headline
            timed(lambda: xe.correlate_into(x, o, stream=stream), 4)
        kernel_ms = timed(lambda: xe.correlate_into(x, o, stream=stream), 20)
        r = {"workload": f"{S} stations, {C} channels, {T} samples, {kind} in pinned host memory",
             "host_bytes": nbytes, "h2d_GB/s": round(h2d, 2), "ai_global_flop_per_B": round(ai_global, 1),
             "perf_max_global_TFLOP/s": round(ai_global * h2d / 1e3, 2),
             "device_resident_ms": round(kernel_ms, 4),
             "device_resident_TFLOP/s": round(flops / kernel_ms / 1e9, 1)}
        ing = xe.Ingest(in_type, S, C, T, layout=xe.XC_LAYOUT_TIME_MAJOR)
        r["channels_per_group"] = ing.channels_per_group
        for tag, ov in (("async", True), ("sync", False)):
            ms = timed(lambda: ing.run(host_tm, out=o, overlap=ov, stream=stream), reps)
            r[f"time_major_{tag}_ms"] = round(ms, 3)
            r[f"time_major_{tag}_TFLOP/s"] = round(flops / ms / 1e9, 2)
        r["time_major_async_frac_of_perf_max_global"] = round(
            r["time_major_async_TFLOP/s"] / r["perf_max_global_TFLOP/s"], 3)
        ing.close()
        # group size: fewer, larger copies against a longer pipeline fill
        by_group = {}
        for mib in (8, 32):
            g = max(1, min(C, (mib << 20) // (T * S * sample)))
            ing = xe.Ingest(in_type, S, C, T, layout=xe.XC_LAYOUT_TIME_MAJOR, channels_per_group=g)
            by_group[f"{g}_channels"] = {
                "async_ms": round(timed(lambda: ing.run(host_tm, out=o, overlap=True, stream=stream), reps), 3),
                "sync_ms": round(timed(lambda: ing.run(host_tm, out=o, overlap=False, stream=stream), reps), 3)}
            ing.close()
        r["time_major_by_group"] = by_group
        del host_tm
        if kind == "cf32":
            # station-major (natural) host layout, transposed on the GPU
            x_sm = x.permute(0, 2, 1, 3).contiguous()
            host_sm = x_sm.cpu().pin_memory()
            ing = xe.Ingest(in_type, S, C, T, layout=xe.XC_LAYOUT_STATION_MAJOR)
            ms = timed(lambda: ing.run(host_sm, out=o, overlap=True, stream=stream), reps)
            r["station_major_async_ms"] = round(ms, 3)
            r["station_major_async_TFLOP/s"] = round(flops / ms / 1e9, 2)
            ing.close()
            del host_sm
            tr_ms = timed(lambda: xe.transpose_to_time_major(x_sm, out=dev_buf, stream=stream), 20)
            r["device_transpose_ms"] = round(tr_ms, 4)
            r["device_transpose_GB/s"] = round(2 * nbytes / (tr_ms * 1e-3) / 1e9, 1)
            # device-resident station-major block correlated directly (corner turn in the LDS copies)
            sm_ms = timed(lambda: xe.correlate_into(x_sm, o, stream=stream, layout=xe.XC_LAYOUT_STATION_MAJOR), 20)
            r["station_major_kernel_ms"] = round(sm_ms, 4)
            r["station_major_kernel_TFLOP/s"] = round(flops / sm_ms / 1e9, 1)
            del x_sm
            # the kernel while a 1 GiB pinned copy runs on another stream
            big_h = torch.empty(1 << 30, dtype=torch.uint8).pin_memory()
            big_d = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
            cs = torch.cuda.Stream()
            torch.cuda.synchronize()
            with torch.cuda.stream(cs):
                big_d.copy_(big_h, non_blocking=True)
            n_k = max(1, int(0.5 * (1 << 30) / max(h2d, 1.0) / 1e6 / kernel_ms))   # kernels within half the copy
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(n_k):
                xe.correlate_into(x, o, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            during = e0.elapsed_time(e1) / n_k
            r["kernel_during_copy_ms"] = round(during, 4)
            r["kernel_slowdown_during_copy"] = round(during / kernel_ms, 3)
            del big_h, big_d
        out[name] = r
        del x, o, dev_buf
        torch.cuda.empty_cache()
    return out


def small_launch_bench(xe, inputs, torch, dev, stream, n=1000):
    """The 8-station workload (8 stations, 16 channels, 256 samples; 4.7e6
    flop): bound by launch latency, timed as n back-to-back launches and as
    the same n launches captured in one HIP graph and replayed."""
    S, C, T = 8, 16, 256
    x = inputs.cn_gaussian(C, T, S, seed=1, device=dev)
    o = torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=dev)
    eager = time_launches(lambda: xe.correlate_into(x, o, stream=stream), n, 50, stream)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            xe.correlate_into(x, o, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(n):
            xe.correlate_into(x, o, stream=side)
    torch.cuda.synchronize()
    replay = time_launches(lambda: g.replay(), 5, 2, torch.cuda.current_stream()) / n
    flops = xe.flops(S, C, T)
    # the integration split over workgroups (partial sums added in a fixed order)
    split = {}
    for k in (4, 16, 64):
        ms = time_launches(lambda: xe.correlate_into(x, o, stream=stream, split=k), n // 4, 20, stream)
        split[str(k)] = round(ms * 1e3, 2)
    best = min(split, key=lambda k: split[k])
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gs, stream=side):
        for _ in range(n):
            xe.correlate_into(x, o, stream=side, split=int(best))
    torch.cuda.synchronize()
    replay_split = time_launches(lambda: gs.replay(), 5, 2, torch.cuda.current_stream()) / n
    return {"workload": f"{S} stations, {C} channels, {T} samples, complex64 CN(0,1)",
            "eager_us_per_launch": round(eager * 1e3, 2), "graph_us_per_launch": round(replay * 1e3, 2),
            "eager_TFLOP/s": round(flops / (eager * 1e-3) / 1e12, 3),
            "graph_TFLOP/s": round(flops / (replay * 1e-3) / 1e12, 3),
            "split_eager_us_per_launch": split, "split_best": int(best),
            "split_graph_us_per_launch": round(replay_split * 1e3, 2),
            "split_graph_TFLOP/s": round(flops / (replay_split * 1e-3) / 1e12, 3)}


def fengine_bench(xe, inputs, torch, dev, stream, steps=20):
    """F-engine: 64 stations x 2 pol of CN(0,1) sample streams through a
    256-channel, 16-tap polyphase filter bank into 768 frames (the lofar64
    block: 256 channels x 768 samples x 64 stations), then correlated.  The
    filter bank is HBM-bound: algorithmic bytes = samples in + channels out
    (8 bytes each); the two kernels also write and read an intermediate of the
    output's size.  Flops per output sample: 4 per tap (complex x real) plus
    5 log2 N for the FFT."""
    S, N, M, T = 64, 256, 16, 768
    n_in = (T + M - 1) * N
    z = inputs.station_streams(S, n_in, seed=6, device=dev)
    taps = torch.from_numpy(inputs.pfb_taps(N, M)).to(dev)
    fb = xe.Pfb(S, N, M, n_in)
    x = torch.empty(fb.out_shape(), dtype=torch.complex64, device=dev)
    o = torch.empty(xe.vis_shape(N, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=dev)
    ms_f = time_launches(lambda: fb.run(z, taps, out=x, stream=stream), steps, 3, stream)
    ms_x = time_launches(lambda: xe.correlate_into(x, o, stream=stream), steps, 3, stream)

    def fx():
        fb.run(z, taps, out=x, stream=stream)
        xe.correlate_into(x, o, stream=stream)
    ms_fx = time_launches(fx, steps, 3, stream)
    # one kernel into the station-major layout, correlated from it
    SM = xe.XC_LAYOUT_STATION_MAJOR
    xs = torch.empty(fb.out_shape(SM), dtype=torch.complex64, device=dev)
    ms_fs = time_launches(lambda: fb.run(z, taps, out=xs, stream=stream, layout=SM), steps, 3, stream)
    ms_xs = time_launches(lambda: xe.correlate_into(xs, o, stream=stream, layout=SM), steps, 3, stream)

    def fxs():
        fb.run(z, taps, out=xs, stream=stream, layout=SM)
        xe.correlate_into(xs, o, stream=stream, layout=SM)
    ms_fxs = time_launches(fxs, steps, 3, stream)
    alg = (z.numel() + x.numel()) * 8
    moved = alg + 2 * x.numel() * 8
    flops_f = x.numel() * (4 * M + 5 * math.log2(N))
    flops_x = xe.flops(S, N, T)
    fb.close()
    # HBM bytes of one filter-bank run (both kernels) from the committed counter summary
    tf, tt = load_traffic("fengine_filter_fft", "pfb"), load_traffic("fengine_corner_turn", "pfb")
    traffic = tf + tt if tf is not None and tt is not None else None
    r = {"workload": f"{S} stations x 2 pol, {n_in} samples per stream -> {N} channels x {T} frames, {M} taps",
         "filter_bank_ms": round(ms_f, 4),
         "filter_bank_Gsamples/s": round(z.numel() / (ms_f * 1e-3) / 1e9, 1),
         "roofline": {"bound": "hbm", "achieved": round(alg / (ms_f * 1e-3) / 1e9, 1), "peak": PEAKS["hbm_GBs"],
                      "unit": "GB/s", "frac": round(alg / (ms_f * 1e-3) / 1e9 / PEAKS["hbm_GBs"], 4),
                      "traffic": traffic, "bytes_moved_incl_intermediate_GB/s": round(moved / (ms_f * 1e-3) / 1e9, 1)},
         "filter_bank_TFLOP/s": round(flops_f / (ms_f * 1e-3) / 1e12, 2),
         "correlator_ms": round(ms_x, 4), "f_then_x_ms": round(ms_fx, 4),
         "f_then_x_correlator_TFLOP/s": round(flops_x / (ms_fx * 1e-3) / 1e12, 1),
         "station_major": {
             "note": "one kernel writes x[N][S][T][2]; the correlator takes it as station-major input",
             "filter_bank_ms": round(ms_fs, 4),
             "filter_bank_Gsamples/s": round(z.numel() / (ms_fs * 1e-3) / 1e9, 1),
             "roofline": {"bound": "hbm", "achieved": round(alg / (ms_fs * 1e-3) / 1e9, 1),
                          "peak": PEAKS["hbm_GBs"], "unit": "GB/s",
                          "frac": round(alg / (ms_fs * 1e-3) / 1e9 / PEAKS["hbm_GBs"], 4),
                          "traffic": load_traffic("fengine_filter_fft_sm", "pfb")},
             "correlator_ms": round(ms_xs, 4), "f_then_x_ms": round(ms_fxs, 4),
             "f_then_x_correlator_TFLOP/s": round(flops_x / (ms_fxs * 1e-3) / 1e12, 1)}}
    del z, x, xs, o
    torch.cuda.empty_cache()
    return r


def stream_all(xe, inputs, torch, args):
    """The streaming measurements.  One stream at the real-time rate with
    staggered folds (integration ends spread over the groups' turns) for every
    fold length k of --stream-ks (deadline k P per block), each over
    --stream-blocks blocks after a warm-up integration; the
    headline run is the smallest k whose block p99 meets the deadline.  Beside
    it: k = 8 with all channels folded every 8 blocks (the unstaggered
    schedule); two streams at the real-time rate with k = --stream-two-k,
    their integrations' ends spread over the groups' turns and their folds
    run one at a time; and --stream-multi streams requested at once (the
    server admits what fits in 90 % of free device memory), whose saturated
    run gives the device's sustained fold rate."""
    out = {}
    ks = [int(v) for v in args.stream_ks.split(",") if v.strip()]
    runs = [stream_bench(xe, inputs, torch, 1, k, args.stream_blocks, spread_ends=True) for k in ks]
    if runs:
        meeting = [r for r in runs if r["block_p99_ms"][0] <= r["deadline_ms"]]
        head = dict(min(meeting, key=lambda r: r["k"]) if meeting else max(runs, key=lambda r: r["k"]))
        head["smallest_k_meeting_block_p99"] = min(r["k"] for r in meeting) if meeting else None
        head["k_sweep"] = [{key: r[key] for key in ("k", "deadline_ms", "block_p50_ms", "block_p99_ms",
                                                     "block_max_ms", "block_misses", "blocks", "fold_p99_ms",
                                                     "sustained_TFLOP/s", "throughput_vs_realtime",
                                                     "producer_stalls")} for r in runs]
        one = next((r for r in runs if r["k"] == 1), None)
        if one is not None:
            S, C, bt = 512, 4096, 256
            acc = C * (S * (S + 1) // 2) * 4 * 8
            blk = C * bt * S * 4
            rmw = 2 * acc + blk
            head["k1_arithmetic"] = {
                "deadline_ms": one["deadline_ms"], "fold_bytes_GB": round(rmw / 1e9, 2),
                "fold_ms_at_8TBs": round(rmw / 8e12 * 1e3, 3),
                "fold_ms_measured": round(xe.flops(S, C, bt) / (one["sustained_TFLOP/s"][0] * 1e12) * 1e3, 3),
                "note": "every block reads and rewrites the whole accumulator: "
                        "HBM time alone is 88 % of the block period at the published peak"}
        out["stream"] = head
    if args.stream_ref_blocks > 0:
        out["stream_all_channels"] = stream_bench(xe, inputs, torch, 1, args.stream_fold, args.stream_ref_blocks,
                                                  staggered=False)
    on_time = 0          # streams kept in real time with every block on time, in the runs above
    if runs and any(r["block_misses"][0] == 0 for r in runs):
        on_time = 1
    if args.stream_two_k > 0:
        two = stream_bench(xe, inputs, torch, 2, args.stream_two_k, args.stream_blocks, spread_ends=True,
                           ordered=True)
        two["all_blocks_on_time"] = two["streams_admitted"] == 2 and all(m == 0 for m in two["block_misses"])
        out["stream_two"] = two
        if two["all_blocks_on_time"]:
            on_time = 2
    out["streams_all_blocks_on_time"] = on_time
    if args.stream_multi > 0:
        m = stream_bench(xe, inputs, torch, args.stream_multi, args.stream_fold, args.stream_multi_blocks,
                         spread_ends=True, ordered=True)
        # saturated (the admitted streams fall behind): the device's fold rate at this k
        m["device_sustained_TFLOP/s"] = round(sum(m["sustained_TFLOP/s"]), 1)
        out["stream_multi"] = m
    return out


def stream_bench(xe, inputs, torch, n_streams, k, n_blocks, S=512, C=4096, bt=256, bpi=192, staggered=True,
                 spread_ends=False, ordered=False):
    """Streaming: 512 stations, 4096 channels, complex int8 blocks of 256
    samples arriving every P = 256 / 49152 s (192 blocks = one second per
    integration), every channel folded every k blocks into resident int32
    accumulators (staggered: one of k channel groups per block; otherwise all
    channels every k blocks).  Arrivals are simulated: every ring slot is
    filled once with distinct random blocks and a block 'arrives' at its
    scheduled host time t0 + n P.  Block latency = completion of the last fold
    covering it - its arrival, against the deadline k P; fold latency =
    completion - arrival of the block that triggered it.  Streams that the
    server refuses for lack of device memory are counted, not run.
    spread_ends: each channel group folds its leftover of an integration at
    its next turn; ordered: the streams' folds run one at a time in enqueue
    order."""
    P = bt / 49152.0
    torch.cuda.empty_cache()    # the admission budget is a share of the free device memory
    srv = xe.Server()
    srv.set_fold_order(ordered)
    desc = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=2 * k, in_type=xe.XC_IN_CI8,
                          acc_type=xe.XC_OUT_CI32, block_period_s=P, staggered=staggered, spread_ends=spread_ends)
    fp = xe.Server.footprint(desc)
    sids, admitted, refused = [], 0, 0
    for _ in range(n_streams):
        try:
            sids.append(srv.open(desc))
            admitted += 1
        except xe.XengineError as e:
            if e.status_name != "XC_ERR_ADMISSION":
                raise
            refused += 1
    # fill every ring slot with distinct samples
    for sid in sids:
        for slot in range(2 * k):
            ptr = srv.acquire(sid)
            t = xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8)
            t.copy_(inputs.ci8_gaussian(C, bt, S, seed=7000 + 31 * sid + slot, device="cuda:0", chunk_channels=512))
            srv.commit(sid, time.monotonic_ns())
    torch.cuda.synchronize()
    for sid in sids:
        srv.stats(sid)
    def feed(n_feed):
        stalls = 0
        t0 = time.monotonic_ns()
        for n in range(n_feed):
            due = t0 + int(n * P * 1e9)
            while time.monotonic_ns() < due:
                pass
            for sid in sids:
                waited = False
                while True:
                    try:
                        srv.acquire(sid)
                        break
                    except xe.XengineError as e:
                        if e.status_name != "XC_ERR_BACKPRESSURE":
                            raise
                        waited = True
                stalls += waited    # blocks whose ring slot was still being folded at arrival
                srv.commit(sid, due)
        return stalls

    # warm-up: the rest of the first integration at the real-time rate
    feed(bpi - 2 * k)
    for sid in sids:
        srv.reset_stats(sid)
    # the producer loop runs without the Python garbage collector, whose pauses
    # would delay commits past their scheduled arrival and count as latency
    gc.collect()
    gc.disable()
    try:
        stalls = feed(n_blocks)
    finally:
        gc.enable()
    per = [srv.stats(sid) for sid in sids]
    for sid in sids:
        srv.close_stream(sid)
    srv.close()
    need = xe.flops(S, C, bt) / P / 1e12
    return {"workload": f"{S} stations, {C} channels, complex int8 blocks of {bt} samples every "
                        f"{P * 1e3:.3f} ms, {bpi} blocks per integration, every channel folded every {k} blocks "
                        + ("(staggered: one channel group per block)" if staggered else "(all channels at once)"),
            "k": k, "staggered": staggered, "spread_ends": spread_ends, "fold_order": ordered,
            "streams_requested": n_streams, "streams_admitted": admitted, "streams_refused": refused,
            "footprint_GB": round(fp / 1e9, 1), "deadline_ms": round(k * P * 1e3, 3),
            "block_p50_ms": [round(p["p50_ms"], 3) for p in per],
            "block_p99_ms": [round(p["p99_ms"], 3) for p in per],
            "block_max_ms": [round(p["max_ms"], 3) for p in per],
            "block_misses": [p["misses"] for p in per], "blocks": [p["blocks"] for p in per],
            "on_time_fraction": [round(1.0 - p["misses"] / max(p["blocks"], 1), 4) for p in per],
            "fold_deadline_ms": round(per[0]["fold_deadline_ms"], 3) if per else None,
            "fold_p50_ms": [round(p["fold_p50_ms"], 3) for p in per],
            "fold_p99_ms": [round(p["fold_p99_ms"], 3) for p in per],
            "fold_max_ms": [round(p["fold_max_ms"], 3) for p in per],
            "folds": [p["folds"] for p in per], "fold_misses": [p["fold_misses"] for p in per],
            "integrations": [p["integrations"] for p in per],
            "sustained_TFLOP/s": [round(p["tflops"], 1) for p in per],
            "throughput_vs_realtime": [round(p["tflops"] / need, 3) for p in per],
            "producer_stalls": stalls, "realtime_TFLOP/s_needed_per_stream": round(need, 1)}


if __name__ == "__main__":
    main()
