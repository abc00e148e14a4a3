"""Checks that pin the oracle to what the correlation definition fixes.

Each check takes the oracle library handle (so the mutation test can run the
same checks against deliberately broken copies of the oracle) and raises
AssertionError when the oracle disagrees with:

* a library routine: numpy's complex matmul X X^H per channel (the
  correlation of Section 2 is the Hermitian product of the station-polarisation
  by time sample matrix with itself), and an exact int64 matmul of the
  real-stacked form for complex-int8 samples;
* closed forms: a delta input that fixes the conjugated factor, the baseline
  numbering and the polarisation order; noise-free tones whose visibilities
  are T * sum_k a_k^2 exp(i(phi_ki - phi_kj)) exp(i(psi_kp - psi_kq));
* invariants: Hermitian autocorrelation blocks, real non-negative XX/YY
  autocorrelations, Cauchy-Schwarz, additivity over time, exact scaling,
  common-phase invariance, channel independence, station relabelling;
* special cases: zero input, a single station, a single time step (rank one),
  and the int32 worst case.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import brute

RTOL_F64 = 1e-13


def _bl(i, j):
    return j * (j + 1) // 2 + i


def _rand_cx(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _rand_i8(rng, shape, lim=127):
    return rng.integers(-lim, lim + 1, size=shape + (2,), dtype=np.int64).astype(np.int8)


def _gram_blocks(x):
    """Per channel G = X X^H with X[(s,p)][t]; returns [C, 2S, 2S] complex128."""
    C, T, S, P = x.shape
    X = np.transpose(x, (0, 2, 3, 1)).reshape(C, S * P, T)   # rows (s, p), cols t
    return X @ np.conj(np.transpose(X, (0, 2, 1)))


def _to_square(vis, S, P):
    """Scatter packed V[c][b][p][q] into [C, S*P, S*P] (upper blocks only, rest nan)."""
    C = vis.shape[0]
    out = np.full((C, S * P, S * P), np.nan + 0j)
    for j in range(S):
        for i in range(j + 1):
            out[:, i * P:(i + 1) * P, j * P:(j + 1) * P] = vis[:, _bl(i, j)]
    return out


def check_numpy_gram(lib, seed=11, C=3, T=97, S=13, P=2):
    rng = np.random.default_rng(seed)
    x = _rand_cx(rng, (C, T, S, P))
    vis = oracle.correlate_f64(x, lib)
    G = _gram_blocks(x)
    V = _to_square(vis, S, P)
    mask = ~np.isnan(V)
    assert np.isfinite(vis).all(), "unwritten or non-finite outputs"
    err = np.linalg.norm(V[mask] - G[mask]) / np.linalg.norm(G[mask])
    assert err < RTOL_F64, f"oracle vs numpy X X^H: rel err {err}"


def check_int_stacked(lib, seed=12, C=2, T=61, S=9, P=2):
    rng = np.random.default_rng(seed)
    x = _rand_i8(rng, (C, T, S, P))
    vis = oracle.correlate_i64(x, lib)
    xr = x[..., 0].astype(np.int64)
    xi = x[..., 1].astype(np.int64)
    # rows (s, p), columns t; Re = Ar Br^T + Ai Bi^T, Im = Ai Br^T - Ar Bi^T
    Xr = np.transpose(xr, (0, 2, 3, 1)).reshape(C, S * P, T)
    Xi = np.transpose(xi, (0, 2, 3, 1)).reshape(C, S * P, T)
    K = np.concatenate([Xr, Xi], axis=2)                 # [C, N, 2T]
    re = K @ np.transpose(K, (0, 2, 1))
    im = np.concatenate([Xi, -Xr], axis=2) @ np.transpose(K, (0, 2, 1))
    for j in range(S):
        for i in range(j + 1):
            got = vis[:, _bl(i, j)]
            assert np.array_equal(got[..., 0], re[:, i * P:(i + 1) * P, j * P:(j + 1) * P]), (i, j)
            assert np.array_equal(got[..., 1], im[:, i * P:(i + 1) * P, j * P:(j + 1) * P]), (i, j)


def check_delta(lib):
    """x[c][t0][i][p] = 1, x[c][t0][j][q] = i (imaginary unit), else 0.
    Then V_ij,pq = 1 * conj(i) = -i, V_ii,pp = 1, V_jj,qq = 1, all else 0."""
    C, T, S, P = 2, 5, 6, 2
    for (i, j, p, q, t0, c) in [(1, 4, 0, 1, 3, 1), (0, 5, 1, 0, 0, 0), (2, 3, 1, 1, 4, 1)]:
        x = np.zeros((C, T, S, P), dtype=np.complex128)
        x[c, t0, i, p] = 1.0
        x[c, t0, j, q] = 1.0j
        vis = oracle.correlate_f64(x, lib)
        expect = np.zeros_like(vis)
        expect[c, _bl(i, j), p, q] = -1j
        expect[c, _bl(i, i), p, p] = 1.0
        expect[c, _bl(j, j), q, q] = 1.0
        assert np.array_equal(vis, expect), ("delta", i, j, p, q)
        xi8 = np.zeros((C, T, S, P, 2), dtype=np.int8)
        xi8[c, t0, i, p, 0] = 1
        xi8[c, t0, j, q, 1] = 1
        vi = oracle.correlate_i64(xi8, lib)
        ei = np.zeros_like(vi)
        ei[c, _bl(i, j), p, q, 1] = -1
        ei[c, _bl(i, i), p, p, 0] = 1
        ei[c, _bl(j, j), q, q, 0] = 1
        assert np.array_equal(vi, ei), ("delta int", i, j, p, q)


def check_tones(lib, seed=13, C=3, T=64, S=7, P=2, K=3):
    rng = np.random.default_rng(seed)
    m = rng.choice(T, size=K, replace=False)
    a = rng.uniform(0.5, 1.5, size=K)
    phi = rng.uniform(-np.pi, np.pi, size=(K, C, S))
    psi = rng.uniform(-np.pi, np.pi, size=(K, P))
    t = np.arange(T)
    x = np.zeros((C, T, S, P), dtype=np.complex128)
    for k in range(K):
        x += a[k] * np.exp(1j * (2 * np.pi * m[k] * t / T))[None, :, None, None] \
            * np.exp(1j * phi[k])[:, None, :, None] * np.exp(1j * psi[k])[None, None, None, :]
    vis = oracle.correlate_f64(x, lib)
    for c in range(C):
        for j in range(S):
            for i in range(j + 1):
                for p in range(P):
                    for q in range(P):
                        expect = T * sum(a[k] ** 2 * np.exp(1j * (phi[k, c, i] - phi[k, c, j]))
                                         * np.exp(1j * (psi[k, p] - psi[k, q])) for k in range(K))
                        got = vis[c, _bl(i, j), p, q]
                        assert abs(got - expect) <= 1e-10 * T, ("tones", c, i, j, p, q, got, expect)


def check_invariants(lib, seed=14, C=2, T=33, S=8, P=2):
    rng = np.random.default_rng(seed)
    x = _rand_cx(rng, (C, T, S, P))
    vis = oracle.correlate_f64(x, lib)
    scale = np.abs(vis).max()
    # autocorrelation blocks: Hermitian, real non-negative diagonal
    for s in range(S):
        blk = vis[:, _bl(s, s)]
        assert np.all(blk[:, 0, 0].imag == 0) and np.all(blk[:, 1, 1].imag == 0), "auto imag"
        assert np.all(blk[:, 0, 0].real >= 0) and np.all(blk[:, 1, 1].real >= 0), "auto sign"
        assert np.allclose(blk[:, 1, 0], np.conj(blk[:, 0, 1]), rtol=0, atol=1e-14 * scale), "YX=conj XY"
    # Cauchy-Schwarz
    for j in range(S):
        for i in range(j + 1):
            for p in range(P):
                for q in range(P):
                    lhs = np.abs(vis[:, _bl(i, j), p, q]) ** 2
                    rhs = vis[:, _bl(i, i), p, p].real * vis[:, _bl(j, j), q, q].real
                    assert np.all(lhs <= rhs * (1 + 1e-12) + 1e-300), "Cauchy-Schwarz"
    # scaling by 2 is exact: V -> 4V
    assert np.array_equal(oracle.correlate_f64(2 * x, lib), 4 * vis), "scaling"
    # common phase rotation leaves V unchanged (to rounding)
    rot = oracle.correlate_f64(x * np.exp(0.7j), lib)
    assert np.abs(rot - vis).max() <= 1e-13 * scale, "phase invariance"
    # additivity in time
    split = 13
    v1 = oracle.correlate_f64(x[:, :split], lib)
    v2 = oracle.correlate_f64(x[:, split:], lib)
    assert np.abs(v1 + v2 - vis).max() <= 1e-13 * scale, "additivity"
    # channel independence
    y = x.copy()
    y[1] += 0.5
    vy = oracle.correlate_f64(y, lib)
    assert np.array_equal(vy[0], vis[0]) and not np.allclose(vy[1], vis[1]), "channel independence"
    # station relabelling: swapping stations a < b maps V_ab,pq to conj(V_ab,qp)
    a_, b_ = 2, 5
    perm = list(range(S))
    perm[a_], perm[b_] = b_, a_
    vp = oracle.correlate_f64(x[:, :, perm], lib)
    for p in range(P):
        for q in range(P):
            assert np.allclose(vp[:, _bl(a_, b_), p, q], np.conj(vis[:, _bl(a_, b_), q, p]),
                               rtol=0, atol=1e-13 * scale), "relabel"
    assert np.allclose(vp[:, _bl(a_, a_)], vis[:, _bl(b_, b_)], rtol=0, atol=1e-13 * scale), "relabel auto"
    # integer additivity is exact
    xi = _rand_i8(rng, (C, T, S, P))
    wi = oracle.correlate_i64(xi, lib)
    assert np.array_equal(oracle.correlate_i64(xi[:, :split], lib)
                          + oracle.correlate_i64(xi[:, split:], lib), wi), "int additivity"
    for s in range(S):
        assert np.all(wi[:, _bl(s, s), 0, 0, 1] == 0) and np.all(wi[:, _bl(s, s), 1, 1, 1] == 0)
        assert np.array_equal(wi[:, _bl(s, s), 1, 0, 0], wi[:, _bl(s, s), 0, 1, 0])
        assert np.array_equal(wi[:, _bl(s, s), 1, 0, 1], -wi[:, _bl(s, s), 0, 1, 1])


def check_special_cases(lib, seed=15):
    rng = np.random.default_rng(seed)
    # zero in, zero out
    z = np.zeros((2, 4, 3, 2), dtype=np.complex128)
    assert np.array_equal(oracle.correlate_f64(z, lib), np.zeros((2, 6, 2, 2), dtype=np.complex128))
    # one station: autocorrelations only, equal to the per-pol sums
    x = _rand_cx(rng, (2, 9, 1, 2))
    v = oracle.correlate_f64(x, lib)
    assert v.shape == (2, 1, 2, 2)
    for p in range(2):
        for q in range(2):
            ref = np.sum(x[:, :, 0, p] * np.conj(x[:, :, 0, q]), axis=1)
            assert np.allclose(v[:, 0, p, q], ref, rtol=1e-14, atol=0)
    # one time step: V_ij,pq = x_ip conj(x_jq) exactly (a single product)
    x = _rand_cx(rng, (1, 1, 5, 2))
    v = oracle.correlate_f64(x, lib)
    for j in range(5):
        for i in range(j + 1):
            for p in range(2):
                for q in range(2):
                    a, b = x[0, 0, i, p], x[0, 0, j, q]
                    expect = complex(a.real * b.real + a.imag * b.imag, a.imag * b.real - a.real * b.imag)
                    assert v[0, _bl(i, j), p, q] == expect
    # int32 worst case: every sample (127, -127)
    T = 100
    w = np.zeros((1, T, 3, 2, 2), dtype=np.int8)
    w[..., 0] = 127
    w[..., 1] = -127
    vi = oracle.correlate_i64(w, lib)
    assert np.all(vi[..., 0] == 2 * 127 * 127 * T) and np.all(vi[..., 1] == 0)


def check_brute(lib, seed=16):
    rng = np.random.default_rng(seed)
    C, T, S, P = 2, 5, 4, 2
    x = _rand_cx(rng, (C, T, S, P))
    ref = brute.correlate_complex(x.tolist())
    vis = oracle.correlate_f64(x, lib)
    for (c, i, j, p, q), val in ref.items():
        assert abs(vis[c, _bl(i, j), p, q] - val) <= 1e-15 * max(1.0, abs(val)) * 8, (c, i, j, p, q)
    xi = _rand_i8(rng, (C, T, S, P))
    refi = brute.correlate_int([[[[tuple(int(v) for v in xi[c, t, s, p]) for p in range(P)]
                                  for s in range(S)] for t in range(T)] for c in range(C)])
    vi = oracle.correlate_i64(xi, lib)
    for (c, i, j, p, q), (re, im) in refi.items():
        assert vi[c, _bl(i, j), p, q, 0] == re and vi[c, _bl(i, j), p, q, 1] == im, (c, i, j, p, q)


ALL_CHECKS = [check_delta, check_numpy_gram, check_int_stacked, check_tones,
              check_invariants, check_special_cases, check_brute]
