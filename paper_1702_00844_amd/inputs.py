"""Seeded synthetic inputs shaped like the paper's LOFAR workloads.

This module only *draws* sample blocks; it holds none of the correlator's
arithmetic and is shared by the tests, the benchmark and the smoke check.
The paper's real station data is not available: these generators stand in
for it, with the shapes of Section 2 (dual-polarised stations, integrations of
768 samples at 763 Hz, i.e. about one second) and the value distributions
listed below.

Layout of every sample block (time-major, as the GPU variant of Section 4.4
stores it): ``x[c][t][s][p]`` complex, channel c, time t, station s,
polarisation p (0 = X, 1 = Y).

* complex float: ``torch.complex64`` tensor of shape [C, T, S, P];
* complex int8 : ``torch.int8`` tensor of shape [C, T, S, P, 2] (re, im).

Generators draw from a ``torch.Generator`` on the requested device, seeded
with ``seed``; the same call on the same device gives the same block.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _gen(device, seed: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def cn_gaussian(C: int, T: int, S: int, P: int = 2, seed: int = 1,
                device="cpu", sigma: float = 1.0) -> torch.Tensor:
    """Circular complex Gaussian CN(0, sigma^2): re, im i.i.d. N(0, sigma^2/2),
    so that E|x|^2 = sigma^2.  Returns complex64 [C, T, S, P]."""
    g = _gen(device, seed)
    ri = torch.randn((C, T, S, P, 2), generator=g, device=device, dtype=torch.float32)
    ri.mul_(sigma / math.sqrt(2.0))
    return torch.view_as_complex(ri)


def ci8_gaussian(C: int, T: int, S: int, P: int = 2, seed: int = 3,
                 device="cpu", sigma: float = 32.0, chunk_channels: int = 64) -> torch.Tensor:
    """Complex int8 samples: re, im = clamp(rint(N(0, sigma^2)), -127, 127).
    -128 never occurs.  Returns int8 [C, T, S, P, 2]."""
    g = _gen(device, seed)
    out = torch.empty((C, T, S, P, 2), dtype=torch.int8, device=device)
    for c0 in range(0, C, chunk_channels):
        c1 = min(C, c0 + chunk_channels)
        r = torch.randn((c1 - c0, T, S, P, 2), generator=g, device=device, dtype=torch.float32)
        r.mul_(sigma).round_().clamp_(-127, 127)
        out[c0:c1] = r.to(torch.int8)
        del r
    return out


def point_sources(C: int, T: int, S: int, P: int = 2, seed: int = 2, device="cpu",
                  n_sources: int = 3, amplitude: float = 0.1, f0_hz: float = 150e6,
                  channel_width_hz: float = 763.0, max_delay_s: float = 5e-6):
    """Noise plus unpolarised point sources with geometric delays.

    x[c][t][s][p] = n[c][t][s][p] + A * sum_k u_k[c][t][p] * exp(i phi[k][c][s]),
    phi[k][c][s] = -2 pi f_c tau[k][s],  f_c = f0 + c * channel_width,
    with n, u_k ~ CN(0, 1) independent and tau[k][s] ~ U(-max_delay, max_delay).

    Returns (x complex64 [C, T, S, P], params) where params holds numpy arrays
    ``phase`` [K, C, S] (radians), ``tau`` [K, S], ``freq`` [C] and ``amplitude``.
    """
    rng = np.random.default_rng(seed)
    tau = rng.uniform(-max_delay_s, max_delay_s, size=(n_sources, S))
    freq = f0_hz + channel_width_hz * np.arange(C, dtype=np.float64)
    phase = -2.0 * np.pi * freq[None, :, None] * tau[:, None, :]          # [K, C, S]
    steer = torch.from_numpy(np.exp(1j * phase)).to(device)                # complex128
    g = _gen(device, seed)
    ri = torch.randn((C, T, S, P, 2), generator=g, device=device, dtype=torch.float64)
    ri.mul_(1.0 / math.sqrt(2.0))
    x = torch.view_as_complex(ri)
    for k in range(n_sources):
        uk = torch.randn((C, T, 1, P, 2), generator=g, device=device, dtype=torch.float64)
        uk.mul_(1.0 / math.sqrt(2.0))
        uk = torch.view_as_complex(uk)                                       # [C, T, 1, P]
        x.add_(amplitude * uk * steer[k][:, None, :, None])
    params = {"phase": phase, "tau": tau, "freq": freq, "amplitude": amplitude}
    return x.to(torch.complex64), params


def tones(C: int, T: int, S: int, P: int = 2, seed: int = 5, n_tones: int = 3,
          device="cpu", dtype=torch.complex128):
    """Noise-free sum of tones with distinct frequency bins:

    x[c][t][s][p] = sum_k a_k exp(i (2 pi m_k t / T + phi[k][c][s] + psi[k][p]))

    with distinct m_k modulo T.  Returns (x [C, T, S, P], params) with numpy
    arrays ``a`` [K], ``m`` [K], ``phi`` [K, C, S], ``psi`` [K, P].
    """
    rng = np.random.default_rng(seed)
    assert n_tones <= T
    m = rng.choice(T, size=n_tones, replace=False)
    a = rng.uniform(0.5, 1.5, size=n_tones)
    phi = rng.uniform(-np.pi, np.pi, size=(n_tones, C, S))
    psi = rng.uniform(-np.pi, np.pi, size=(n_tones, P))
    t = np.arange(T, dtype=np.float64)
    x = np.zeros((C, T, S, P), dtype=np.complex128)
    for k in range(n_tones):
        carrier = np.exp(1j * 2.0 * np.pi * m[k] * t / T)                  # [T]
        x += a[k] * (carrier[None, :, None, None]
                     * np.exp(1j * phi[k])[:, None, :, None]
                     * np.exp(1j * psi[k])[None, None, None, :])
    params = {"a": a, "m": m, "phi": phi, "psi": psi}
    return torch.from_numpy(x).to(device=device, dtype=dtype), params


def subarray_shapes(n_items: int = 32, seed: int = 4, s_range=(24, 576),
                    c_range=(16, 1024), n_times: int = 768):
    """Shapes of a batch of uneven sub-arrays: stations uniform in s_range,
    channels uniform in c_range (inclusive), fixed integration length.
    Returns a list of (n_stations, n_channels, n_times)."""
    rng = np.random.default_rng(seed)
    S = rng.integers(s_range[0], s_range[1] + 1, size=n_items)
    C = rng.integers(c_range[0], c_range[1] + 1, size=n_items)
    return [(int(s), int(c), int(n_times)) for s, c in zip(S, C)]


def station_streams(S: int, n_in: int, P: int = 2, seed: int = 6, device="cpu",
                    sigma: float = 1.0) -> torch.Tensor:
    """Station sample streams before channelisation: complex64 [S, P, n_in],
    CN(0, sigma^2) noise (the F-engine's input, station-major)."""
    g = _gen(device, seed)
    ri = torch.randn((S, P, n_in, 2), generator=g, device=device, dtype=torch.float32)
    ri.mul_(sigma / math.sqrt(2.0))
    return torch.view_as_complex(ri)


def pfb_taps(n_channels: int, n_taps: int) -> np.ndarray:
    """Prototype filter of an N-channel, M-tap polyphase filter bank: a sinc of
    N samples per lobe under a Hann window, M N coefficients (float32).  A
    data recipe, not part of the filter bank's arithmetic: the filter bank
    takes any real taps."""
    N, M = int(n_channels), int(n_taps)
    k = np.arange(M * N, dtype=np.float64) + 0.5
    h = np.sinc((k - M * N / 2.0) / N) * (0.5 - 0.5 * np.cos(2.0 * np.pi * k / (M * N)))
    return h.astype(np.float32)
