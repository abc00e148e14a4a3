"""Pure-Python twin of the oracle for tiny shapes -- TEST INFRASTRUCTURE ONLY.

Follows the correlation equation of Section 2 with Python's own complex and
integer numbers (no numpy arithmetic): one explicit sum over time per
(channel, station pair, polarisation pair).  Used to cross-check the C oracle on inputs of a few
stations and times.
"""
from __future__ import annotations


def correlate_complex(samples):
    """samples: nested lists [C][T][S][P] of Python complex.
    Returns {(c, i, j, p, q): complex} for every 0 <= i <= j."""
    out = {}
    for c, block in enumerate(samples):
        T = len(block)
        S = len(block[0])
        P = len(block[0][0])
        for j in range(S):
            for i in range(j + 1):
                for p in range(P):
                    for q in range(P):
                        acc = 0j
                        for t in range(T):
                            acc += block[t][i][p] * block[t][j][q].conjugate()
                        out[(c, i, j, p, q)] = acc
    return out


def correlate_int(samples):
    """samples: nested lists [C][T][S][P] of (re, im) Python int pairs.
    Returns {(c, i, j, p, q): (re, im)} with exact integer sums."""
    out = {}
    for c, block in enumerate(samples):
        T = len(block)
        S = len(block[0])
        P = len(block[0][0])
        for j in range(S):
            for i in range(j + 1):
                for p in range(P):
                    for q in range(P):
                        re = im = 0
                        for t in range(T):
                            ar, ai = block[t][i][p]
                            br, bi = block[t][j][q]
                            # (ar + i ai)(br - i bi)
                            re += ar * br + ai * bi
                            im += ai * br - ar * bi
                        out[(c, i, j, p, q)] = (re, im)
    return out
