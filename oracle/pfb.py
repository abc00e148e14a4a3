"""Polyphase filter bank (F-engine) oracle -- TEST INFRASTRUCTURE ONLY.

The paper's processing chain (Section 2, Figure 1) filters each station's
data stream into frequency channels (and compensates signal-path delays)
before the correlator; the channels of the correlation equation are that
stage's output.  The paper fixes no filter design, so this is the reading
taken (the GPU library implements the same definition):

A critically sampled polyphase filter bank with N channels and M taps per
channel, prototype filter h[0 .. M N - 1] (real, given), applied to each
station's and polarisation's complex sample stream z[0 .. n_in - 1]:

    u[t][n] = sum_{m=0}^{M-1} h[m N + n] * z[(t + m) N + n]          (n < N)
    y[t][k] = sum_{n=0}^{N-1} u[t][n] * exp(-2 pi i k n / N)         (k < N)
    x[k][t][s][p] = w[s][p][k] * y_{s,p}[t][k]                         (w optional)

for the T = floor(n_in / N) - M + 1 frames t whose window lies in the input.
The output is the correlator's channel-major, time-major input x[c][t][s][p]:
the corner turn of an FX correlator (Section 7).  A per-(station,
polarisation, channel) complex weight w carries delay compensation (a phase
slope over the channels), bandpass or gain corrections.

Only tests/ and bench.py's CPU-baseline leg use this module; it shares no
code with the GPU library.  ``pfb_brute`` is a loop-only twin for tiny
shapes (no FFT, no vectorisation).  Pins: tests/test_oracle_pfb.py.
"""
from __future__ import annotations

import cmath
import math

import numpy as np


def n_frames(n_in: int, n_channels: int, n_taps: int) -> int:
    return n_in // n_channels - n_taps + 1


def pfb_channelize(z, taps, n_channels: int, weights=None) -> np.ndarray:
    """z: complex [S][P][n_in]; taps: real [M N]; weights: complex [S][P][N] or
    None.  Returns complex128 x[N][T][S][P]."""
    z = np.asarray(z).astype(np.complex128)
    h = np.asarray(taps).astype(np.float64)
    N = int(n_channels)
    M = h.size // N
    if M * N != h.size or M < 1:
        raise ValueError("taps must hold M * n_channels values")
    S, P, n_in = z.shape
    T = n_frames(n_in, N, M)
    if T < 1:
        raise ValueError("input shorter than one filter window")
    hb = h.reshape(M, N)                                   # hb[m][n] = h[m N + n]
    frames = z[:, :, :(T + M - 1) * N].reshape(S, P, T + M - 1, N)   # frames[f][n] = z[f N + n]
    u = np.zeros((S, P, T, N), dtype=np.complex128)
    for m in range(M):
        u += hb[m] * frames[:, :, m:m + T, :]
    y = np.fft.fft(u, axis=-1)                             # sum over n of u[n] exp(-2 pi i k n / N)
    if weights is not None:
        y = y * np.asarray(weights).astype(np.complex128)[:, :, None, :]
    return np.ascontiguousarray(y.transpose(3, 2, 0, 1))


def pfb_brute(z, taps, n_channels: int, weights=None) -> list:
    """The same definition with plain loops and a direct DFT; tiny shapes only.
    Returns nested lists x[k][t][s][p]."""
    N = int(n_channels)
    h = [float(v) for v in np.asarray(taps).ravel()]
    M = len(h) // N
    S, P, n_in = len(z), len(z[0]), len(z[0][0])
    T = n_in // N - M + 1
    x = [[[[0j for _ in range(P)] for _ in range(S)] for _ in range(T)] for _ in range(N)]
    for s in range(S):
        for p in range(P):
            for t in range(T):
                u = [sum(h[m * N + n] * complex(z[s][p][(t + m) * N + n]) for m in range(M)) for n in range(N)]
                for k in range(N):
                    acc = 0j
                    for n in range(N):
                        acc += u[n] * cmath.exp(-2j * math.pi * k * n / N)
                    if weights is not None:
                        acc *= complex(weights[s][p][k])
                    x[k][t][s][p] = acc
    return x
