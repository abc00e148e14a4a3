"""GPU parity: the HIP kernels against the oracle, element by element.

Bars: complex-int8 -> int32 bit-exact; complex-float32 inputs within 1e-5
normwise; 16-bit float inputs: accumulation error against the oracle on the
same (rounded) samples within 1e-5 normwise, total error against the oracle on
the unrounded samples within the per-element rounding bound (and 2e-3
normwise on a workload-sized block), and exact on integer-valued samples whose
partial sums stay below 2^24."""
import numpy as np
import pytest
import torch

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import inputs
from tests.helpers import assert_hermitian_autos, gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FP32_TOL = 1e-5

VALU = [dict(kernel=xe.XC_KERNEL_VALU, time_chunk=tc, time_split=ts)
        for tc, ts in [(16, 1), (16, 2), (16, 4), (32, 2), (32, 4), (32, 8)]]
# the other register tiles (the default is 4 x 2)
VALU += [dict(kernel=xe.XC_KERNEL_VALU, tile_w=w, tile_h=h, time_chunk=tc, time_split=ts)
         for w, h in [(4, 4), (8, 2), (2, 2)] for tc, ts in [(16, 1), (32, 4)]]
MFMA = dict(kernel=xe.XC_KERNEL_MFMA)
# complex-float32 matrix-core variants: 32x32 tiles on 32-station blocks, and
# 16x16 tiles on 64-station blocks with one or two time groups, each with the
# three-product (default) and the four-product form
MFMA_F32 = [dict(kernel=xe.XC_KERNEL_MFMA, block=32), dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=1),
            dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=2),
            dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=1, product=xe.XC_PRODUCT_FOUR),
            dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=2, product=xe.XC_PRODUCT_FOUR)]

# (S, C, T): tiny, ragged station counts across block edges, ragged time tails
SHAPES = [(1, 2, 1), (3, 1, 5), (8, 3, 17), (33, 2, 100), (64, 2, 64), (70, 1, 300), (130, 1, 77)]


def _cf32(S, C, T, seed):
    return inputs.cn_gaussian(C, T, S, seed=seed, device=DEV)


def _cfg_id(c):
    if c["kernel"] == xe.XC_KERNEL_VALU:
        tile = "_t%dx%d" % (c["tile_w"], c["tile_h"]) if "tile_w" in c else ""
        return "valu_tc%d_ts%d%s" % (c["time_chunk"], c["time_split"], tile)
    return "mfma_b%d_ts%d%s" % (c.get("block", 0), c.get("time_split", 0),
                                "_p4" if c.get("product") == xe.XC_PRODUCT_FOUR else "")


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "S%d_C%d_T%d" % s)
@pytest.mark.parametrize("cfg", VALU + MFMA_F32, ids=_cfg_id)
def test_cf32_parity(shape, cfg):
    S, C, T = shape
    x = _cf32(S, C, T, seed=S * 1000 + T)
    v = xe.correlate(x, config=cfg)
    torch.cuda.synchronize()
    got, ref = gpu_vis_numpy(v), oracle_vis(x)
    assert rel_err(got, ref) <= FP32_TOL, rel_err(got, ref)
    assert_hermitian_autos(got, S)


# the one-channel kernel for arrays of at most 16 stations (the default for
# complex float32 there): station counts 1..16, integrations across its
# 128-step chunks (1, 2, 77, 128, 129, 300, 1000 steps), 1..17 channels
SMALL = dict(kernel=xe.XC_KERNEL_VALU, block=16)
SMALL_SHAPES = [(1, 1, 1), (1, 4, 300), (2, 3, 129), (5, 17, 128), (8, 16, 256), (13, 3, 77), (16, 5, 1000),
                (16, 1, 2)]


@pytest.mark.parametrize("shape", SMALL_SHAPES, ids=lambda s: "S%d_C%d_T%d" % s)
@pytest.mark.parametrize("cfg", [None, SMALL], ids=["auto", "explicit"])
def test_small_array_kernel(shape, cfg):
    """Within 1e-5 of the oracle, Hermitian autocorrelations, accumulation
    adding exactly the same sums again; station-major input gives the same
    bits; the integration split within 1e-5."""
    S, C, T = shape
    if cfg is not None:     # (AUTO may also take a configuration tuned for the shape's bucket)
        assert xe.resolve_config((xe.XC_IN_CF32, C, T, S, 2), config=cfg)["block"] == 16
    x = _cf32(S, C, T, seed=7 * S + T)
    v = xe.correlate(x, config=cfg)
    v2 = v.clone()
    xe.correlate(x, out=v2, accumulate=True, config=cfg)
    vs = xe.correlate(x.permute(0, 2, 1, 3).contiguous(), config=cfg, layout=xe.XC_LAYOUT_STATION_MAJOR)
    vt = xe.correlate(x, config=SMALL)
    vp = xe.correlate(x, config=cfg, split=3)
    torch.cuda.synchronize()
    ref = oracle_vis(x)
    got = gpu_vis_numpy(v)
    assert rel_err(got, ref) <= FP32_TOL, rel_err(got, ref)
    assert_hermitian_autos(got, S)
    assert torch.equal(v2, v + v)
    assert torch.equal(vs, vt)
    assert rel_err(gpu_vis_numpy(vp), ref) <= FP32_TOL


# int8 kernels: the default (staged straight into LDS when S % 4 == 0), the
# register-staged one on 64-station blocks, and 32-station blocks; extra shapes
# with S % 4 == 0 give the direct-to-LDS kernel diagonal and off-diagonal
# blocks, ragged blocks and ragged time tails
I8_CFGS = [None, dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS),
           dict(kernel=xe.XC_KERNEL_MFMA, block=32)]
I8_SHAPES = SHAPES + [(4, 1, 5), (68, 2, 100), (128, 1, 97), (132, 2, 33), (192, 1, 64)]


@pytest.mark.parametrize("shape", I8_SHAPES, ids=lambda s: "S%d_C%d_T%d" % s)
@pytest.mark.parametrize("out_type", [xe.XC_OUT_CI32, xe.XC_OUT_CF32], ids=["ci32", "cf32"])
@pytest.mark.parametrize("cfg", I8_CFGS, ids=["default", "b64_regs", "b32"])
def test_ci8_bit_exact(shape, out_type, cfg):
    S, C, T = shape
    x = inputs.ci8_gaussian(C, T, S, seed=S + 7 * T, device=DEV)
    v = xe.correlate(x, out_type=out_type, config=cfg)
    torch.cuda.synchronize()
    ref = oracle_vis(x)
    got = gpu_vis_numpy(v)
    if out_type == xe.XC_OUT_CI32:
        assert np.array_equal(got, ref)
    else:  # int32 sums converted to float: exact below 2^24
        assert np.array_equal(got, ref[..., 0] + 1j * ref[..., 1])


# unit roundoff and half the smallest subnormal spacing of the 16-bit formats
HALF_U = {torch.float16: 2.0 ** -11, torch.bfloat16: 2.0 ** -8}
HALF_ETA = {torch.float16: 2.0 ** -25, torch.bfloat16: 2.0 ** -134}


def _half_bound(xf, dtype):
    """Per-element bound on |V(rounded samples) - V(exact samples)|: rounding
    each complex component to a 16-bit format moves a sample a by at most
    u |a| + eta, so each product a conj(b) moves by at most
    (2u + u^2) |a||b| + eta (|a| + |b|) (1 + u), summed over time; plus the
    FP32 accumulation, at most T 2^-24 of the magnitude sum."""
    x = xf.detach().cpu().numpy().astype(np.complex128)
    mag = np.abs(x)
    T = x.shape[1]
    vabs = oracle_vis(torch.from_numpy(mag.astype(np.complex128)).to(torch.complex64)).real
    u, eta = HALF_U[dtype], HALF_ETA[dtype]
    s = mag.sum(axis=1)                                  # [C, S, P]
    C, S, P = s.shape
    lin = np.zeros_like(vabs)
    for j in range(S):
        for i in range(j + 1):
            b = j * (j + 1) // 2 + i
            lin[:, b] = s[:, i, :, None] + s[:, j, None, :]
    return (2 * u + u * u + T * 2.0 ** -24) * vabs * 1.001 + eta * (1 + u) * lin * 1.001


# 16-bit kernels: the default (staged straight into LDS when S is even), the
# register-staged one on 64-station blocks, and 32-station blocks
HALF_CFGS = [None, dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS),
             dict(kernel=xe.XC_KERNEL_MFMA, block=32)]


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16], ids=["f16", "bf16"])
@pytest.mark.parametrize("shape", I8_SHAPES, ids=lambda s: "S%d_C%d_T%d" % s)
@pytest.mark.parametrize("cfg", HALF_CFGS, ids=["default", "b64_regs", "b32"])
def test_half_parity(shape, dtype, cfg):
    S, C, T = shape
    xf = _cf32(S, C, T, seed=S * 31 + T)
    xh = torch.view_as_real(xf).to(dtype).contiguous()
    v = xe.correlate(xh, config=cfg)
    torch.cuda.synchronize()
    got = gpu_vis_numpy(v)
    acc_err = rel_err(got, oracle_vis(xh))          # same rounded samples: accumulation only
    assert acc_err <= FP32_TOL, acc_err
    err = np.abs(got - oracle_vis(xf))              # unrounded samples: quantisation + accumulation
    assert np.all(err <= _half_bound(xf, dtype)), float((err / _half_bound(xf, dtype)).max())
    assert_hermitian_autos(got, S)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16], ids=["f16", "bf16"])
def test_half_normwise_on_workload_shape(dtype):
    """64 stations, 768 samples of CN(0,1) noise (16 of the 256 channels):
    total error against the FP64 oracle on the unrounded samples <= 2e-3."""
    xf = _cf32(64, 16, 768, seed=2)
    xh = torch.view_as_real(xf).to(dtype).contiguous()
    got = gpu_vis_numpy(xe.correlate(xh))
    tot = rel_err(got, oracle_vis(xf))
    assert tot <= 2e-3, tot


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16], ids=["f16", "bf16"])
@pytest.mark.parametrize("cfg", HALF_CFGS, ids=["default", "b64_regs", "b32"])
def test_half_exact_on_integer_samples(dtype, cfg):
    S, C, T = 70, 2, 200
    xi = inputs.ci8_gaussian(C, T, S, seed=5, device=DEV)
    xh = xi.to(dtype)                                # |v| <= 127: exact in f16 and bf16
    v = xe.correlate(xh, config=cfg)
    torch.cuda.synchronize()
    ref = oracle_vis(xi)
    assert np.abs(ref).max() < 2 ** 24
    assert np.array_equal(gpu_vis_numpy(v), ref[..., 0] + 1j * ref[..., 1])


@pytest.mark.parametrize("cfg", [VALU[2]] + MFMA_F32, ids=_cfg_id)
def test_accumulate_mode(cfg):
    S, C, T = 40, 3, 96
    x1 = _cf32(S, C, T, seed=11)
    x2 = _cf32(S, C, T, seed=12)
    v = xe.correlate(x1, config=cfg)
    xe.correlate(x2, out=v, accumulate=True, config=cfg)
    torch.cuda.synchronize()
    ref = oracle_vis(torch.cat([x1, x2], dim=1))     # additivity over time
    assert rel_err(gpu_vis_numpy(v), ref) <= FP32_TOL


@pytest.mark.parametrize("ts", [1, 2])
def test_three_product_forward_error_bound(ts):
    """The three-product form on strongly correlated samples (one common
    signal in every station plus weak noise, so that for most baselines the
    imaginary part is tiny next to P1, P2 and P3, the case its cancellation
    hurts most): every element lies within the forward error bounds of
    single-precision sums of T products, with M = sum_t |a_t| |b_t| and
    u = 2^-24: |d Re V| <= (T + 4) u M (P1 + P2, where |ar br| + |ai bi| <=
    |a| |b|) and |d Im V| <= 3 (T + 4) u M (P3 - P1 + P2, where
    |ar + ai| |br - bi| <= 2 |a| |b|); and the normwise error within the
    single-precision bar."""
    S, C, T = 96, 2, 700
    common = inputs.cn_gaussian(C, T, 1, seed=31, device=DEV)
    x = (10.0 * common + 0.01 * _cf32(S, C, T, seed=32)).contiguous()
    cfg = dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=ts, product=xe.XC_PRODUCT_THREE)
    got = gpu_vis_numpy(xe.correlate(x, config=cfg))
    ref = oracle_vis(x)
    mag = oracle_vis(x.abs().to(torch.complex64)).real     # sum_t |a_t| |b_t| (|x| rounded to float32)
    bound = (T + 4) * 2.0 ** -24 * mag * (1 + 1e-6)
    err_re, err_im = np.abs(got.real - ref.real), np.abs(got.imag - ref.imag)
    assert np.all(err_re <= bound), float(np.max(err_re / bound))
    assert np.all(err_im <= 3 * bound), float(np.max(err_im / (3 * bound)))
    assert rel_err(got, ref) <= FP32_TOL
    assert_hermitian_autos(got, S)


@pytest.mark.parametrize("S", [66, 68])
def test_accumulate_int_exact(S):
    C, T = 2, 128
    x1 = inputs.ci8_gaussian(C, T, S, seed=21, device=DEV)
    x2 = inputs.ci8_gaussian(C, T, S, seed=22, device=DEV)
    v = xe.correlate(x1)
    xe.correlate(x2, out=v, accumulate=True)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_vis_numpy(v), oracle_vis(torch.cat([x1, x2], dim=1)))


@pytest.mark.parametrize("S", [71, 132])
@pytest.mark.parametrize("kind", ["ci8_ci32", "ci8_cf32", "f16", "bf16"])
def test_direct_store_accumulate_exact(kind, S):
    """Accumulate mode of the int8 and 16-bit kernel that copies straight into
    LDS and stores tiles from its accumulators (two calls into one output),
    on integer-valued samples so that every sum is exact in the output type
    (at most 320 x 2 x 127^2 < 2^24): bit for bit the oracle's result over the
    concatenated integration.  S = 71 is one full and one partial 64-station
    block (copied in 4-byte words for both sample types); S = 132 is two full
    blocks and a four-station edge block (16-byte copies), with off-diagonal
    pairs."""
    C, T = 2, 160
    x1 = inputs.ci8_gaussian(C, T, S, seed=41, device=DEV)
    x2 = inputs.ci8_gaussian(C, T, S, seed=42, device=DEV)
    cfg = dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_LDS)
    if kind in ("f16", "bf16"):
        dt = torch.float16 if kind == "f16" else torch.bfloat16
        a, b, out_type = x1.to(dt), x2.to(dt), None          # |v| <= 127: exact in both
    else:
        a, b = x1, x2
        out_type = xe.XC_OUT_CI32 if kind == "ci8_ci32" else xe.XC_OUT_CF32
    v = xe.correlate(a, config=cfg, out_type=out_type)
    xe.correlate(b, out=v, accumulate=True, config=cfg)
    torch.cuda.synchronize()
    ref = oracle_vis(torch.cat([x1, x2], dim=1))
    got = gpu_vis_numpy(v)
    if kind == "ci8_ci32":
        assert np.array_equal(got, ref)
    else:
        assert np.array_equal(got, ref[..., 0] + 1j * ref[..., 1])


@pytest.mark.parametrize("S", [9, 12])
def test_int32_worst_case(S):
    """All samples (127, -127): V = 2 * 127^2 * T exactly, at a ragged T."""
    C, T = 1, 1000
    x = torch.empty((C, T, S, 2, 2), dtype=torch.int8, device=DEV)
    x[..., 0] = 127
    x[..., 1] = -127
    v = xe.correlate(x)
    torch.cuda.synchronize()
    got = gpu_vis_numpy(v)
    assert np.all(got[..., 0] == 2 * 127 * 127 * T) and np.all(got[..., 1] == 0)


def test_delta_conjugation_and_numbering():
    S, C, T = 70, 2, 40
    i, j, p, q, t0, c = 5, 66, 0, 1, 33, 1
    x = torch.zeros((C, T, S, 2), dtype=torch.complex64, device=DEV)
    x[c, t0, i, p] = 1
    x[c, t0, j, q] = 1j
    for cfg in VALU[2:3] + MFMA_F32:
        v = gpu_vis_numpy(xe.correlate(x, config=cfg))
        expect = np.zeros_like(v)
        expect[c, xe.baseline_index(i, j), p, q] = -1j
        expect[c, xe.baseline_index(i, i), p, p] = 1
        expect[c, xe.baseline_index(j, j), q, q] = 1
        assert np.array_equal(v, expect)


def test_config1_full():
    """8 stations, 16 channels, 256 samples, CN(0,1): every output."""
    x = inputs.cn_gaussian(16, 256, 8, seed=1, device=DEV)
    ref = oracle_vis(x)
    for cfg in VALU + MFMA_F32:
        assert rel_err(gpu_vis_numpy(xe.correlate(x, config=cfg)), ref) <= FP32_TOL


def test_config2_full():
    """64 stations, 256 channels, 768 samples, noise plus three point sources:
    every output, both FP32 kernels, in the configurations the benchmark times."""
    x, _ = inputs.point_sources(256, 768, 64, seed=2, device=DEV)
    ref = oracle_vis(x)
    for cfg in VALU[2:] + MFMA_F32 + [None]:
        got = gpu_vis_numpy(xe.correlate(x, config=cfg))
        assert rel_err(got, ref) <= FP32_TOL
        assert_hermitian_autos(got, 64)


@pytest.mark.parametrize("shape", [(70, 70, 45), (128, 66, 20), (96, 64, 33)], ids=lambda s: "S%d_C%d_T%d" % s)
def test_valu_longest_first_order(shape):
    """At least 64 channels on two to four 32-station blocks: the vector-ALU
    launch runs each XCD's off-diagonal block pairs before its diagonal ones,
    over contiguous channel ranges (70 and 66 channels leave the last range
    short).  Every output against the oracle, for each register tile."""
    S, C, T = shape
    x = _cf32(S, C, T, seed=S + C + T)
    ref = oracle_vis(x)
    for cfg in [VALU[4], VALU[0]] + VALU[6:]:
        got = gpu_vis_numpy(xe.correlate(x, config=cfg))
        assert rel_err(got, ref) <= FP32_TOL, cfg
        assert_hermitian_autos(got, S)


def test_config3_sampled_channels():
    """256 stations, 1024 channels, 1024 samples of complex int8: int8 MFMA is
    bit-exact, the same values as f16/bf16 are exact, and the FP32 twin is
    within 1e-5, on sampled channels (first, last, and two inside)."""
    C, T, S = 1024, 1024, 256
    x = inputs.ci8_gaussian(C, T, S, seed=3, device=DEV)
    chans = [0, 1, 517, C - 1]
    ref = oracle_vis(x, chans)
    for cfg in I8_CFGS[:2]:
        v = xe.correlate(x, config=cfg)
        assert np.array_equal(gpu_vis_numpy(v, chans), ref)
        del v
    refc = ref[..., 0] + 1j * ref[..., 1]
    for dtype in (torch.float16, torch.bfloat16):
        for cfg in HALF_CFGS[:2]:
            vh = xe.correlate(x.to(dtype), config=cfg)
            assert np.array_equal(gpu_vis_numpy(vh, chans), refc)
            del vh
    xf = torch.view_as_complex(x.to(torch.float32))
    for cfg in [VALU[2]] + MFMA_F32:
        vf = xe.correlate(xf, config=cfg)
        assert rel_err(gpu_vis_numpy(vf, chans), refc) <= FP32_TOL
        del vf


@pytest.mark.parametrize("kind", ["cf32_mfma_p3", "cf32_mfma_p4", "cf32_valu", "ci8", "ci8_regs", "cf16", "cbf16"])
def test_large_ragged_station_count(kind):
    """520 stations (eight full 64-station blocks and a ragged ninth: 45 block
    pairs per channel, diagonal and off-diagonal), ragged time: every output."""
    S, C, T = 520, 2, 37
    if kind.startswith("cf32"):
        x = _cf32(S, C, T, seed=520)
        cfg = {"cf32_mfma_p3": dict(kernel=xe.XC_KERNEL_MFMA, product=xe.XC_PRODUCT_THREE),
               "cf32_mfma_p4": dict(kernel=xe.XC_KERNEL_MFMA, product=xe.XC_PRODUCT_FOUR),
               "cf32_valu": dict(kernel=xe.XC_KERNEL_VALU)}[kind]
        got, ref = gpu_vis_numpy(xe.correlate(x, config=cfg)), oracle_vis(x)
        assert rel_err(got, ref) <= FP32_TOL
        assert_hermitian_autos(got, S)
        return
    xi = inputs.ci8_gaussian(C, T, S, seed=521, device=DEV)
    ref = oracle_vis(xi)
    if kind.startswith("ci8"):
        cfg = None if kind == "ci8" else dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS)
        assert np.array_equal(gpu_vis_numpy(xe.correlate(xi, config=cfg)), ref)
        return
    x = xi.to(torch.float16 if kind == "cf16" else torch.bfloat16)     # exact: integer samples
    assert np.array_equal(gpu_vis_numpy(xe.correlate(x)), ref[..., 0] + 1j * ref[..., 1])


def test_int32_bound_at_the_longest_integration():
    """T = 66572, the longest integration int32 holds exactly: all samples
    (127, -127) give 2 * 127^2 * T = 2147450408 in every XX/YY/XY/YX real
    part, through the int8 kernels (direct-to-LDS and register-staged)."""
    S, C, T = 8, 1, 66572
    x = torch.empty((C, T, S, 2, 2), dtype=torch.int8, device=DEV)
    x[..., 0] = 127
    x[..., 1] = -127
    for cfg in (None, dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS),
                dict(kernel=xe.XC_KERNEL_MFMA, block=32)):
        got = gpu_vis_numpy(xe.correlate(x, config=cfg))
        assert np.all(got[..., 0] == 2 * 127 * 127 * T) and np.all(got[..., 1] == 0)
    assert 2 * 127 * 127 * T <= 2 ** 31 - 1


SPLIT_CFGS = [("cf32", dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=2)),
              ("cf32", dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=1, product=xe.XC_PRODUCT_FOUR)),
              ("cf32", dict(kernel=xe.XC_KERNEL_MFMA, block=32)),
              ("cf32", dict(kernel=xe.XC_KERNEL_VALU)),
              ("ci8", None),
              ("ci8", dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS)),
              ("ci8", dict(kernel=xe.XC_KERNEL_MFMA, block=32)),
              ("cf16", None)]


@pytest.mark.parametrize("kind,cfg", SPLIT_CFGS, ids=["f32_b64ts2", "f32_b64ts1p4", "f32_b32", "f32_valu", "i8_lds",
                                                      "i8_regs", "i8_b32", "f16_lds"])
@pytest.mark.parametrize("split", [2, 7, 1000])
def test_split_integration(kind, cfg, split):
    """The integration cut into pieces over workgroups, partial sums added in
    a fixed order: int8 bit-exact, 16-bit exact on integer samples, FP32
    within 1e-5; accumulation adds over time exactly as without the split."""
    S, C, T = 70, 3, 101
    if kind == "cf32":
        x1, x2 = _cf32(S, C, T, seed=61), _cf32(S, C, T, seed=62)
    else:
        x1 = inputs.ci8_gaussian(C, T, S, seed=61, device=DEV)
        x2 = inputs.ci8_gaussian(C, T, S, seed=62, device=DEV)
        if kind == "cf16":
            x1, x2 = x1.to(torch.float16), x2.to(torch.float16)
    v = xe.correlate(x1, config=cfg, split=split)
    xe.correlate(x2, out=v, accumulate=True, config=cfg, split=split)
    torch.cuda.synchronize()
    src = torch.cat([x1, x2], dim=1)
    got = gpu_vis_numpy(v)
    if kind == "cf32":
        assert rel_err(got, oracle_vis(src)) <= FP32_TOL
        assert_hermitian_autos(got, S)
    else:
        ref = oracle_vis(src.to(torch.int8) if kind == "cf16" else src)
        assert np.array_equal(got, ref if kind == "ci8" else ref[..., 0] + 1j * ref[..., 1])
