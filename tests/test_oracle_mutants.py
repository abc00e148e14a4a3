"""Mutation test of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, the conjugate on the wrong factor, a transposed
index, a shortened loop), builds it, and checks that at least one of the pins
in ``tests/oracle_pins.py`` rejects it.  The real oracle source is never
modified.
"""
import os

import pytest

import oracle
from tests import oracle_pins as pins

MUTANTS = {
    "conj_wrong_factor_f64": ("sum_im += a[1] * b[0] - a[0] * b[1];",
                              "sum_im += a[0] * b[1] - a[1] * b[0];"),
    "dropped_term_re_f64": ("sum_re += a[0] * b[0] + a[1] * b[1];",
                            "sum_re += a[0] * b[0];"),
    "wrong_sign_re_f64": ("sum_re += a[0] * b[0] + a[1] * b[1];",
                          "sum_re += a[0] * b[0] - a[1] * b[1];"),
    "no_conjugate_f64": ("sum_im += a[1] * b[0] - a[0] * b[1];",
                         "sum_im += a[1] * b[0] + a[0] * b[1];"),
    "transposed_baseline": ("return j * (j + 1) / 2 + i;",
                            "return i * (i + 1) / 2 + j;"),
    "pol_swap_output": ("double *v = vis + 2 * (((ch * B + bl) * P + pol1) * P + pol2);",
                        "double *v = vis + 2 * (((ch * B + bl) * P + pol2) * P + pol1);"),
    "pol_swap_input": ("const double *a = x + 2 * (((ch * T + t) * S + station1) * P + pol1);",
                       "const double *a = x + 2 * (((ch * T + t) * S + station1) * P + pol2);"),
    "short_time_loop_f64": ("for (int64_t t = 0; t < T; t++) {\n                            const double",
                            "for (int64_t t = 1; t < T; t++) {\n                            const double"),
    "no_autocorrelations": ("for (int64_t station1 = 0; station1 <= station2; station1++) {\n"
                            "                for (int64_t pol1 = 0; pol1 < P; pol1++) {\n"
                            "                    for (int64_t pol2 = 0; pol2 < P; pol2++) {\n"
                            "                        double",
                            "for (int64_t station1 = 0; station1 < station2; station1++) {\n"
                            "                for (int64_t pol1 = 0; pol1 < P; pol1++) {\n"
                            "                    for (int64_t pol2 = 0; pol2 < P; pol2++) {\n"
                            "                        double"),
    "conj_wrong_factor_i64": ("sum_im += ai * br - ar * bi;", "sum_im += ar * bi - ai * br;"),
    "dropped_term_re_i64": ("sum_re += ar * br + ai * bi;", "sum_re += ar * br;"),
    "station_swap_i64": ("const int8_t *b = x + 2 * (((ch * T + t) * S + station2) * P + pol2);",
                         "const int8_t *b = x + 2 * (((ch * T + t) * S + station1) * P + pol2);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_kill_mutant(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(before) == 1, f"mutation site for {name} not found exactly once"
    mutant_c = tmp_path / f"{name}.c"
    mutant_c.write_text(src.replace(before, after))
    lib = oracle.load(oracle.build(str(mutant_c), str(tmp_path / f"lib{name}.so")))
    failures = []
    for check in pins.ALL_CHECKS:
        try:
            check(lib)
        except AssertionError as e:
            failures.append((check.__name__, str(e)[:80]))
    assert failures, f"mutant {name} survived every pin"
