"""Pins of the polyphase-filter-bank oracle (CPU).

The oracle (oracle/pfb.py) is checked against what its definition fixes
without reusing its own formula: a loop-only brute force with a direct DFT,
closed forms for a tone at a bin centre and for an impulse, linearity, the
exact effect of the weights and of a one-frame delay.  A mutation test plants
plausible mistakes in copies of the oracle's source and checks that the pins
reject each one."""
import math
import os
import types

import numpy as np
import pytest

from oracle import pfb as P_ORACLE

RNG = np.random.default_rng(1702)
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "pfb.py")


def _cn(*shape):
    return (RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)) / math.sqrt(2)


# -- pins, each taking the filter-bank function under test -------------------

def pin_brute_force(pfb):
    S, P, N, M = 2, 2, 8, 3
    n_in = N * 7 + 5                                   # ragged tail: 5 samples unused
    z = _cn(S, P, n_in)
    h = RNG.standard_normal(M * N)
    w = _cn(S, P, N)
    got = pfb(z, h, N, w)
    ref = np.array(P_ORACLE.pfb_brute(z.tolist(), h, N, w.tolist()))
    assert got.shape == ref.shape == (N, 7 - M + 1, S, P)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def pin_tone(pfb):
    """Taps whose branch sums are all c: a tone at bin k0 gives c N at k0, 0 elsewhere."""
    S, P, N, M, T = 2, 2, 16, 4, 5
    h = RNG.standard_normal((M, N))
    c = 1.7
    h[M - 1] = c - h[:M - 1].sum(0)
    k0 = 5
    n = np.arange((T + M - 1) * N)
    amp = RNG.uniform(0.5, 2.0, (S, P))
    phi = RNG.uniform(-np.pi, np.pi, (S, P))
    z = amp[:, :, None] * np.exp(1j * phi)[:, :, None] * np.exp(2j * np.pi * k0 * n / N)[None, None, :]
    x = pfb(z, h.ravel(), N)
    expect = np.zeros((N, T, S, P), complex)
    expect[k0] = (c * N * amp * np.exp(1j * phi))[None, :, :]
    assert np.max(np.abs(x - expect)) <= 1e-9 * c * N


def pin_impulse(pfb):
    """A unit sample at f0 N + n0 of one stream: y[t][k] = h[(f0 - t) N + n0] e^{-2 pi i k n0 / N}."""
    S, P, N, M, T = 3, 2, 8, 4, 6
    h = RNG.standard_normal(M * N)
    f0, n0, s0, p0 = 6, 3, 1, 1
    z = np.zeros((S, P, (T + M - 1) * N), complex)
    z[s0, p0, f0 * N + n0] = 1.0
    x = pfb(z, h, N)
    expect = np.zeros((N, T, S, P), complex)
    for t in range(T):
        m = f0 - t
        if 0 <= m < M:
            expect[:, t, s0, p0] = h[m * N + n0] * np.exp(-2j * np.pi * np.arange(N) * n0 / N)
    assert np.max(np.abs(x - expect)) <= 1e-12


def pin_linearity_weights_delay(pfb):
    S, P, N, M, T = 2, 2, 8, 3, 6
    n_in = (T + M - 1) * N
    h = RNG.standard_normal(M * N)
    z1, z2 = _cn(S, P, n_in), _cn(S, P, n_in)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    x1, x2 = pfb(z1, h, N), pfb(z2, h, N)
    assert np.allclose(pfb(a * z1 + b * z2, h, N), a * x1 + b * x2, rtol=0, atol=1e-12)
    w = _cn(S, P, N)
    xw = pfb(z1, h, N, w)
    assert np.allclose(xw, x1 * w.transpose(2, 0, 1)[:, None, :, :], rtol=0, atol=1e-12)
    # one frame of delay (N samples) shifts the output by one frame
    zd = np.concatenate([np.zeros((S, P, N), complex), z1], axis=-1)
    xd = pfb(zd, h, N)
    assert np.allclose(xd[:, 1:], x1, rtol=0, atol=1e-12)


PINS = [pin_brute_force, pin_tone, pin_impulse, pin_linearity_weights_delay]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(P_ORACLE.pfb_channelize)


# -- mutations: each must fail at least one pin ------------------------------

MUTANTS = {
    "taps_reversed": ("u += hb[m] * frames", "u += hb[M - 1 - m] * frames"),
    "inverse_dft": ("np.fft.fft(u, axis=-1)", "np.fft.ifft(u, axis=-1) * N"),
    "frame_off_by_one": ("frames[:, :, m:m + T, :]", "frames[:, :, m + 1:m + 1 + T, :] if m + 1 + T <= T + M - 1 else frames[:, :, m:m + T, :]"),
    "output_transposed": ("y.transpose(3, 2, 0, 1)", "y.transpose(3, 2, 1, 0)"),
    "weights_conjugated": ("y = y * np.asarray(weights).astype(np.complex128)[:, :, None, :]",
                           "y = y * np.conj(np.asarray(weights).astype(np.complex128))[:, :, None, :]"),
    "last_tap_dropped": ("for m in range(M):", "for m in range(M - 1):"),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_reject_mutant(name):
    src = open(ORACLE_SRC).read()
    old, new = MUTANTS[name]
    assert old in src, name
    mod = types.ModuleType("pfb_mutant")
    exec(compile(src.replace(old, new), ORACLE_SRC + "[" + name + "]", "exec"), mod.__dict__)
    failures = 0
    for pin in PINS:
        try:
            pin(mod.pfb_channelize)
        except (AssertionError, ValueError):
            failures += 1
    assert failures >= 1, f"mutant {name} passes every pin"
