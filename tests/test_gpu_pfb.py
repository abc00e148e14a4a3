"""GPU: the F-engine (polyphase filter bank into the correlator's input)
against its oracle, and the F -> X chain against the two oracles composed.

Bar: single-precision filter and FFT, within 1e-5 normwise of the fp64
oracle (the FIR sums M terms and the FFT has log2 N stages, each with
rounding of order 2^-24 relative to the values it combines)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1702_00844_amd as xe
from oracle import pfb as opfb
from paper_1702_00844_amd import inputs
from tests.helpers import gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("N", [256, 512])
@pytest.mark.parametrize("M", [1, 4, 16])
@pytest.mark.parametrize("S,extra,T", [(1, 0, 1), (3, 77, 21), (2, 255, 40)], ids=["S1_T1", "S3_T21", "S2_T40"])
@pytest.mark.parametrize("weighted", [False, True], ids=["plain", "weighted"])
def test_pfb_matches_oracle(N, M, S, extra, T, weighted):
    n_in = (T + M - 1) * N + extra                      # ragged tail of unused samples
    z = inputs.station_streams(S, n_in, seed=N + M + S, device=DEV)
    taps = torch.from_numpy(inputs.pfb_taps(N, M)).to(DEV)
    w = None
    if weighted:
        g = torch.Generator(device="cpu").manual_seed(9)
        w = torch.polar(torch.rand((S, 2, N), generator=g) + 0.5,
                        torch.rand((S, 2, N), generator=g) * 6.283).to(torch.complex64).to(DEV)
    fb = xe.Pfb(S, N, M, n_in)
    assert fb.n_frames == T
    x = fb.run(z, taps, w)
    torch.cuda.synchronize()
    ref = opfb.pfb_channelize(z.cpu().numpy(), taps.cpu().numpy(), N,
                              None if w is None else w.cpu().numpy())
    got = x.cpu().numpy().astype(np.complex128)
    assert got.shape == ref.shape == (N, T, S, 2)
    assert _rel(got, ref) <= TOL, _rel(got, ref)
    fb.close()


@pytest.mark.parametrize("N", [256, 512])
@pytest.mark.parametrize("M", [1, 4, 16])
@pytest.mark.parametrize("S,extra,T", [(1, 0, 1), (3, 77, 21), (2, 255, 40), (5, 3, 16)],
                         ids=["S1_T1", "S3_T21", "S2_T40", "S5_T16"])
@pytest.mark.parametrize("weighted", [False, True], ids=["plain", "weighted"])
def test_pfb_station_major_matches_oracle(N, M, S, extra, T, weighted):
    """The one-kernel station-major output x[N][S][T][2]: within the bar of the
    fp64 oracle, and bit-identical to the time-major output turned around."""
    n_in = (T + M - 1) * N + extra
    z = inputs.station_streams(S, n_in, seed=40 + M + S, device=DEV)
    taps = torch.from_numpy(inputs.pfb_taps(N, M)).to(DEV)
    w = None
    if weighted:
        g = torch.Generator(device="cpu").manual_seed(19)
        w = torch.polar(torch.rand((S, 2, N), generator=g) + 0.5,
                        torch.rand((S, 2, N), generator=g) * 6.283).to(torch.complex64).to(DEV)
    fb = xe.Pfb(S, N, M, n_in)
    xs = fb.run(z, taps, w, layout=xe.XC_LAYOUT_STATION_MAJOR)
    xt = fb.run(z, taps, w)
    torch.cuda.synchronize()
    assert tuple(xs.shape) == (N, S, T, 2)
    assert torch.equal(xs.permute(0, 2, 1, 3), xt)
    ref = opfb.pfb_channelize(z.cpu().numpy(), taps.cpu().numpy(), N, None if w is None else w.cpu().numpy())
    got = xs.permute(0, 2, 1, 3).cpu().numpy().astype(np.complex128)
    assert _rel(got, ref) <= TOL, _rel(got, ref)
    fb.close()


def test_pfb_station_major_feeds_the_correlator():
    """Station streams -> one-kernel station-major filter bank -> correlator on
    station-major input, against the two oracles composed."""
    N, M, S, T = 256, 4, 5, 33
    n_in = (T + M - 1) * N
    z = inputs.station_streams(S, n_in, seed=12, device=DEV)
    taps = torch.from_numpy(inputs.pfb_taps(N, M)).to(DEV)
    fb = xe.Pfb(S, N, M, n_in)
    v = xe.correlate(fb.run(z, taps, layout=xe.XC_LAYOUT_STATION_MAJOR), layout=xe.XC_LAYOUT_STATION_MAJOR)
    torch.cuda.synchronize()
    ref = oracle.correlate_f64(opfb.pfb_channelize(z.cpu().numpy(), taps.cpu().numpy(), N))
    assert rel_err(gpu_vis_numpy(v), ref) <= 2 * TOL
    fb.close()


def test_pfb_tone_closed_form():
    """Taps with equal branch sums c: a tone at bin k0 lands in channel k0 with
    amplitude c N, every other channel at rounding level."""
    N, M, S, T = 256, 8, 2, 12
    k0 = 37
    h = np.random.default_rng(3).standard_normal((M, N)).astype(np.float64)
    c = 0.75
    h[M - 1] = c - h[:M - 1].sum(0)
    n = np.arange((T + M - 1) * N)
    amp = np.array([[1.0, 0.5], [2.0, 1.5]])
    phi = np.array([[0.3, -1.1], [2.0, 0.9]])
    zn = amp[:, :, None] * np.exp(1j * (phi[:, :, None] + 2 * np.pi * k0 * n[None, None, :] / N))
    z = torch.from_numpy(zn.astype(np.complex64)).to(DEV)
    taps = torch.from_numpy(h.ravel().astype(np.float32)).to(DEV)
    fb = xe.Pfb(S, N, M, zn.shape[-1])
    x = fb.run(z, taps).cpu().numpy().astype(np.complex128)
    expect = np.zeros((N, T, S, 2), complex)
    expect[k0] = (c * N * amp * np.exp(1j * phi))[None]
    # rounding: the input is complex64 and the taps float32 (relative ~1e-7 each), sums of M N terms
    assert np.max(np.abs(x - expect)) <= 1e-4 * c * N * amp.max()
    fb.close()


@pytest.mark.parametrize("kernel", [xe.XC_KERNEL_MFMA, xe.XC_KERNEL_VALU], ids=["mfma", "valu"])
def test_f_then_x_against_oracles(kernel):
    """Station streams -> filter bank -> correlator, against the correlation
    oracle applied to the filter-bank oracle's output."""
    N, M, S, T = 256, 4, 5, 33
    n_in = (T + M - 1) * N
    z = inputs.station_streams(S, n_in, seed=11, device=DEV)
    taps = torch.from_numpy(inputs.pfb_taps(N, M)).to(DEV)
    fb = xe.Pfb(S, N, M, n_in)
    v = xe.correlate(fb.run(z, taps), config={"kernel": kernel})
    torch.cuda.synchronize()
    xr = opfb.pfb_channelize(z.cpu().numpy(), taps.cpu().numpy(), N)           # [N][T][S][2], complex128
    ref = oracle.correlate_f64(xr)
    assert rel_err(gpu_vis_numpy(v), ref) <= 2 * TOL
    fb.close()


def test_pfb_rejects_bad_tensors():
    fb = xe.Pfb(2, 256, 4, 4 * 256)
    z = inputs.station_streams(2, 4 * 256, device=DEV)
    taps = torch.from_numpy(inputs.pfb_taps(256, 4)).to(DEV)
    with pytest.raises(ValueError):
        fb.run(z[:, :, :-1].contiguous(), taps)
    with pytest.raises(ValueError):
        fb.run(z, taps[:-1].contiguous())
    with pytest.raises(ValueError):
        fb.run(z.cpu(), taps.cpu())
    fb.close()
