"""Mutation test of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, the conjugate on the wrong factor, a transposed
index, a shortened loop, a skipped block), builds it, and checks that at least one of the pins
in ``tests/oracle_pins.py`` rejects it.  The real oracle source is never
modified.
"""
import os

import pytest

import oracle
from tests import oracle_pins as pins

# name -> (text at the mutation site, its replacement, which occurrence of the
# text: the double-precision routine comes first in the source, the int64 one
# second)
MUTANTS = {
    "conj_wrong_factor_f64": ("gi[r * n + u] += ui * wr - ur * wi;", "gi[r * n + u] += ur * wi - ui * wr;", 0),
    "dropped_term_re_f64": ("gr[r * n + u] += ur * wr + ui * wi;", "gr[r * n + u] += ur * wr;", 0),
    "wrong_sign_re_f64": ("gr[r * n + u] += ur * wr + ui * wi;", "gr[r * n + u] += ur * wr - ui * wi;", 0),
    "no_conjugate_f64": ("gi[r * n + u] += ui * wr - ur * wi;", "gi[r * n + u] += ui * wr + ur * wi;", 0),
    "transposed_baseline": ("return j * (j + 1) / 2 + i;", "return i * (i + 1) / 2 + j;", 0),
    "pol_swap_output": ("const int64_t g = (i * P + p) * n + (j * P + q);",
                        "const int64_t g = (i * P + q) * n + (j * P + p);", 0),
    "pol_major_rows": ("const int64_t g = (i * P + p) * n + (j * P + q);",
                       "const int64_t g = (p * S + i) * n + (q * S + j);", 0),
    "pack_lower_block": ("const int64_t g = (i * P + p) * n + (j * P + q);",
                         "const int64_t g = (j * P + q) * n + (i * P + p);", 0),
    "short_time_loop_f64": ("for (int64_t t = 0; t < T; t++) {\n        const double",
                            "for (int64_t t = 1; t < T; t++) {\n        const double", 0),
    "no_autocorrelations": ("for (int64_t u = (r / P) * P; u < n; u++) {",
                            "for (int64_t u = (r / P + 1) * P; u < n; u++) {", 0),
    "missing_cross_pol_auto": ("for (int64_t u = (r / P) * P; u < n; u++) {", "for (int64_t u = r; u < n; u++) {", 0),
    "conj_wrong_factor_i64": ("gi[r * n + u] += ui * wr - ur * wi;", "gi[r * n + u] += ur * wi - ui * wr;", 1),
    "dropped_term_re_i64": ("gr[r * n + u] += ur * wr + ui * wi;", "gr[r * n + u] += ur * wr;", 1),
    "station_swap_i64": ("const int64_t wr = at[2 * u], wi = at[2 * u + 1];",
                         "const int64_t wr = at[2 * r], wi = at[2 * r + 1];", 0),
}


def _replace_nth(src, before, after, nth):
    pos = -1
    for _ in range(nth + 1):
        pos = src.index(before, pos + 1)
    return src[:pos] + after + src[pos + len(before):]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_kill_mutant(name, tmp_path):
    before, after, nth = MUTANTS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(before) > nth, f"mutation site for {name} not found"
    mutant_c = tmp_path / f"{name}.c"
    mutant_c.write_text(_replace_nth(src, before, after, nth))
    lib = oracle.load(oracle.build(str(mutant_c), str(tmp_path / f"lib{name}.so")))
    failures = []
    for check in pins.ALL_CHECKS:
        try:
            check(lib)
        except AssertionError as e:
            failures.append((check.__name__, str(e)[:80]))
    assert failures, f"mutant {name} survived every pin"
