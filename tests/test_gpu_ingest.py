"""GPU: host ingest.  Channel groups copied from host memory (overlapping the
previous group's correlation, or in order with it), station-major input
transposed on the GPU, give exactly the visibilities of the device-resident
path on the time-major block (the same kernels run on the same channel data);
the layout transpose is an exact permutation of the samples."""
import numpy as np
import pytest
import torch

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import inputs
from tests.helpers import gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TM, SM = xe.XC_LAYOUT_TIME_MAJOR, xe.XC_LAYOUT_STATION_MAJOR
IN_TYPES = {"cf32": xe.XC_IN_CF32, "ci8": xe.XC_IN_CI8, "cf16": xe.XC_IN_CF16, "cbf16": xe.XC_IN_CBF16}


def _samples(kind, C, T, S, seed):
    if kind == "cf32":
        return inputs.cn_gaussian(C, T, S, seed=seed, device=DEV)
    xi = inputs.ci8_gaussian(C, T, S, seed=seed, device=DEV)
    return xi if kind == "ci8" else xi.to(torch.float16 if kind == "cf16" else torch.bfloat16)


def _station_major(x):
    """[C, T, S, ...] -> [C, S, T, ...] (the natural order)."""
    return x.permute(0, 2, 1, *range(3, x.dim())).contiguous()


def _bits(t):
    return t.detach().cpu().contiguous().view(torch.uint8)


@pytest.mark.parametrize("kind", list(IN_TYPES))
@pytest.mark.parametrize("shape", [(3, 45, 70), (1, 1, 1), (2, 32, 33), (1, 100, 64)],
                         ids=lambda s: "C%d_T%d_S%d" % s)
def test_transpose_is_exact(kind, shape):
    C, T, S = shape
    x = _samples(kind, C, T, S, seed=5 + S)
    got = xe.transpose_to_time_major(_station_major(x))
    torch.cuda.synchronize()
    assert torch.equal(_bits(got), _bits(x))


@pytest.mark.parametrize("kind", ["cf32", "ci8", "cf16"])
@pytest.mark.parametrize("layout", [TM, SM], ids=["time_major", "station_major"])
@pytest.mark.parametrize("overlap", [True, False], ids=["async", "sync"])
@pytest.mark.parametrize("group", [1, 3, 0], ids=["g1", "g3", "gdefault"])
def test_ingest_matches_device_path(kind, layout, overlap, group):
    C, T, S = 7, 50, 70          # ragged stations, time and groups (3 does not divide 7)
    x = _samples(kind, C, T, S, seed=17)
    ref = gpu_vis_numpy(xe.correlate(x))
    host = (x if layout == TM else _station_major(x)).cpu().pin_memory()
    ing = xe.Ingest(IN_TYPES[kind], S, C, T, layout=layout, channels_per_group=group)
    got = ing.run(host, overlap=overlap)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_vis_numpy(got), ref)
    ing.close()


@pytest.mark.parametrize("config", [{"kernel": xe.XC_KERNEL_VALU, "time_chunk": 16, "time_split": 4},
                                    {"kernel": xe.XC_KERNEL_MFMA, "block": 32},
                                    {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "time_split": 1}],
                         ids=["valu_direct", "mfma32_transposed", "mfma64_direct"])
def test_ingest_station_major_fp32_kernels(config):
    """Station-major complex float32 groups: the kernels that corner-turn in
    their loads read the staged group directly, the 32-station matrix-core
    kernel after the GPU transpose; every path gives the device result."""
    C, T, S = 5, 70, 45
    x = _samples("cf32", C, T, S, seed=29)
    ref = gpu_vis_numpy(xe.correlate(x, config=config))
    ing = xe.Ingest(xe.XC_IN_CF32, S, C, T, layout=SM, channels_per_group=2)
    got = gpu_vis_numpy(ing.run(_station_major(x).cpu().pin_memory(), config=config))
    torch.cuda.synchronize()
    assert np.array_equal(got, ref)
    ing.close()


@pytest.mark.parametrize("layout", [TM, SM], ids=["time_major", "station_major"])
def test_ingest_fp32_64_stations_against_oracle(layout):
    """The two-time-group FP32 kernel on 64-station blocks, fed group by group
    from pinned memory: identical to the device path, within 1e-5 of the oracle."""
    C, T, S = 6, 96, 64
    x = _samples("cf32", C, T, S, seed=23)
    host = (x if layout == TM else _station_major(x)).cpu().pin_memory()
    ing = xe.Ingest(xe.XC_IN_CF32, S, C, T, layout=layout, channels_per_group=4)
    got = gpu_vis_numpy(ing.run(host))
    torch.cuda.synchronize()
    assert np.array_equal(got, gpu_vis_numpy(xe.correlate(x)))
    assert rel_err(got, oracle_vis(x)) <= 1e-5


def test_ingest_reuse_accumulate_and_pageable_memory():
    """Back-to-back runs on one plan reuse the staging slots only after their
    previous group is correlated; accumulation adds over time exactly (int8);
    pageable host memory gives the same result as pinned."""
    C, T, S = 5, 64, 40
    x1 = _samples("ci8", C, T, S, seed=41)
    x2 = _samples("ci8", C, T, S, seed=42)
    ing = xe.Ingest(xe.XC_IN_CI8, S, C, T, layout=SM, channels_per_group=2)
    h1 = _station_major(x1).cpu()                  # pageable
    h2 = _station_major(x2).cpu().pin_memory()
    out = ing.run(h1)
    ing.run(h2, out=out, accumulate=True)
    second = ing.run(h2)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_vis_numpy(out), oracle_vis(torch.cat([x1, x2], dim=1)))
    assert np.array_equal(gpu_vis_numpy(second), oracle_vis(x2))
    ing.close()


def test_ingest_rejects_bad_host_tensors():
    ing = xe.Ingest(xe.XC_IN_CF32, 8, 2, 16, layout=TM)
    x = _samples("cf32", 2, 16, 8, seed=3)
    with pytest.raises(ValueError):
        ing.run(x)                                  # device tensor
    with pytest.raises(ValueError):
        ing.run(_station_major(x).cpu())            # wrong layout (shape)
    with pytest.raises(ValueError):
        ing.run(x.cpu().to(torch.complex128))       # wrong dtype
    ing.close()


@pytest.mark.parametrize("shape", [(3, 70, 100), (2, 64, 768), (1, 1, 1), (4, 130, 33), (2, 8, 256), (1, 129, 200)],
                         ids=["S70_T100", "S64_T768", "S1_T1", "S130_T33", "S8_T256", "S129_T200"])
@pytest.mark.parametrize("config", [None, {"time_split": 1}, {"time_split": 2, "product": xe.XC_PRODUCT_FOUR},
                                    {"time_split": 1, "product": xe.XC_PRODUCT_FOUR},
                                    {"kernel": xe.XC_KERNEL_VALU, "time_chunk": 32, "time_split": 8},
                                    {"kernel": xe.XC_KERNEL_VALU, "time_chunk": 16, "time_split": 1}],
                         ids=["auto", "ts1", "ts2_p4", "ts1_p4", "valu_ts8", "valu_ts1"])
def test_station_major_kernel_matches_time_major(shape, config):
    """The station-major kernels corner-turn in their sample loads (copies into
    LDS, or loads into registers): what they stage, and so their results bit
    for bit, are those of the time-major kernel with the same configuration on
    the transposed block."""
    C, S, T = shape
    x = _samples("cf32", C, T, S, seed=900 + S + T)
    cfg = dict(config or {})
    if not cfg:
        # AUTO: the one-channel kernel on at most 16 stations, else the 64-station matrix-core kernel
        cfg = {"kernel": xe.XC_KERNEL_VALU, "block": 16} if S <= 16 else {"kernel": xe.XC_KERNEL_MFMA, "block": 64}
    elif cfg.get("kernel") != xe.XC_KERNEL_VALU:
        cfg = {"kernel": xe.XC_KERNEL_MFMA, "block": 64, **cfg}
    ref = xe.correlate(x, config=cfg)
    got = xe.correlate(_station_major(x), config=config, layout=SM)
    assert torch.equal(_bits(got), _bits(ref))


def test_station_major_against_oracle_with_accumulation():
    C, S, T = 3, 70, 300
    x1 = _samples("cf32", C, T, S, seed=931)
    x2 = _samples("cf32", C, 77, S, seed=932)
    out = xe.correlate(_station_major(x1), layout=SM)
    assert rel_err(gpu_vis_numpy(out), oracle_vis(x1)) <= 1e-5
    xe.correlate(_station_major(x2), out=out, accumulate=True, layout=SM)
    assert rel_err(gpu_vis_numpy(out), oracle_vis(torch.cat([x1, x2], dim=1))) <= 1e-5


@pytest.mark.parametrize("kind", ["ci8", "cf16", "cbf16"])
@pytest.mark.parametrize("shape", [(2, 64, 64), (1, 130, 97), (3, 20, 5), (2, 251, 300), (1, 1, 7)],
                         ids=lambda s: "C%d_S%d_T%d" % s)
def test_station_major_int8_16bit_matches_time_major(kind, shape):
    """int8 and 16-bit station-major input: the 4-byte copies gather each
    station's word from its own series into the time-major kernel's LDS image,
    so the result equals the time-major kernel's bit for bit (and the oracle:
    int8 and integer-valued 16-bit samples are exact), for ragged station
    counts, ragged time tails and diagonal and off-diagonal block pairs."""
    C, S, T = shape
    x = _samples(kind, C, T, S, seed=950 + S + T)
    ref = xe.correlate(x)
    got = xe.correlate(_station_major(x), layout=SM)
    assert torch.equal(_bits(got), _bits(ref))
    xo = x.to(torch.int8) if kind != "ci8" else x
    o = oracle_vis(xo)
    g = gpu_vis_numpy(got)
    if kind == "ci8":
        assert np.array_equal(g, o)
    else:
        assert np.array_equal(g, o[..., 0] + 1j * o[..., 1])


def test_station_major_int8_accumulates_and_rejects_register_staging():
    C, S, T = 2, 68, 200
    x1 = _samples("ci8", C, T, S, seed=961)
    x2 = _samples("ci8", C, 33, S, seed=962)
    out = xe.correlate(_station_major(x1), layout=SM)
    xe.correlate(_station_major(x2), out=out, accumulate=True, layout=SM)
    assert np.array_equal(gpu_vis_numpy(out), oracle_vis(torch.cat([x1, x2], dim=1)))
    for cfg in ({"kernel": xe.XC_KERNEL_MFMA, "staging": xe.XC_STAGING_REGISTERS},
                {"kernel": xe.XC_KERNEL_MFMA, "block": 32}, {"kernel": xe.XC_KERNEL_VALU}):
        with pytest.raises(xe.XengineError) as e:
            xe.correlate(_station_major(x1), layout=SM, config=cfg)
        assert e.value.status_name in ("XC_ERR_UNSUPPORTED", "XC_ERR_INVALID_ARG")
