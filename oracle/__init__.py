"""Correlator oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementation of the correlation of van Nieuwpoort & Romein,
"Correlating Radio Astronomy Signals with Many-Core Hardware", Section 2
(the correlation equation):

    V[c][b(i,j)][p][q] = sum_t x[c][t][i][p] * conj(x[c][t][j][q]),
    0 <= i <= j < S,  b(i,j) = j(j+1)/2 + i,

computed per channel as the Hermitian Gram matrix of the time steps' sample
vectors (one rank-one update per time step, time ascending), whose 2x2
blocks on and above the block diagonal are then packed into V.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1702_00844_amd``) and never imports it.

The arithmetic lives in ``xc_oracle.c`` (double for floating-point inputs,
int64 for complex-int8 inputs); this module only marshals numpy arrays.
``brute.py`` holds a pure-Python twin for tiny shapes.

Pins (tests/test_oracle_pins.py): numpy's complex matmul X X^H (a library
routine), an exact int64 matmul of the real-stacked form, closed forms for delta
and tone inputs, a statistical closed form for point sources, and the
invariants the definition implies (Hermitian autocorrelations, real
non-negative XX/YY autos, Cauchy-Schwarz, additivity in time, scaling, phase
and station-permutation symmetry, channel independence, degenerate shapes and
the int32 worst case).  A mutation test plants mistakes in copies of
``xc_oracle.c`` and checks that the pins catch each one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "xc_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]

_lock = threading.Lock()
_cached = {}


def build(source: str = SOURCE, output: str = LIBRARY) -> str:
    """Compile the oracle with gcc (plain C, no GPU code)."""
    tmp = output + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, source], check=True)
    os.replace(tmp, output)
    return output


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    c_i32, c_i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_correlate_f64.argtypes = [vp, c_i32, c_i32, c_i32, c_i32, vp]
    lib.oracle_correlate_f64.restype = None
    lib.oracle_correlate_i64.argtypes = [vp, c_i32, c_i32, c_i32, c_i32, vp]
    lib.oracle_correlate_i64.restype = None
    lib.oracle_n_baselines.argtypes = [c_i32]
    lib.oracle_n_baselines.restype = c_i64
    return lib


def load(path: str = LIBRARY) -> ctypes.CDLL:
    """Load (building first if missing or older than the source)."""
    with _lock:
        if path in _cached:
            return _cached[path]
        if path == LIBRARY and (not os.path.exists(path)
                                or os.path.getmtime(path) < os.path.getmtime(SOURCE)):
            build()
        lib = _bind(ctypes.CDLL(path))
        _cached[path] = lib
        return lib


def n_baselines(n_stations: int) -> int:
    """Number of station pairs including autocorrelations, S(S+1)/2 (Section 2)."""
    return n_stations * (n_stations + 1) // 2


def baseline_index(i: int, j: int) -> int:
    """Dense baseline number b(i,j) = j(j+1)/2 + i for 0 <= i <= j."""
    assert 0 <= i <= j
    return j * (j + 1) // 2 + i


def correlate_f64(x, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """x: complex array [C, T, S, P] (any precision; widened exactly to
    complex128).  Returns complex128 [C, B, P, P]."""
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
    C, T, S, P = x.shape
    B = n_baselines(S)
    vis = np.full((C, B, P, P), np.nan + 1j * np.nan, dtype=np.complex128)
    lib.oracle_correlate_f64(x.ctypes.data, S, P, C, T, vis.ctypes.data)
    return vis


def correlate_i64(x, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """x: int8 array [C, T, S, P, 2] (re, im).  Returns int64 [C, B, P, P, 2]."""
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(x), dtype=np.int8)
    C, T, S, P, two = x.shape
    assert two == 2
    B = n_baselines(S)
    vis = np.full((C, B, P, P, 2), np.iinfo(np.int64).min, dtype=np.int64)
    lib.oracle_correlate_i64(x.ctypes.data, S, P, C, T, vis.ctypes.data)
    return vis


def threads() -> int:
    """OpenMP threads the oracle will use (OMP_NUM_THREADS, else all cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.strip().isdigit():
        return int(env)
    return os.cpu_count() or 1
