"""The oracle's pins must catch plausible mistakes.

Each case compiles a copy of the oracle's C source with one planted mistake (a
dropped term, a wrong index, a shifted loop bound, a flipped tie-break or
sign) into a temporary directory, points the oracle wrapper at it, and checks
that at least one pin from test_oracle fails.  Everything runs on the CPU.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "qubo_oracle.c")

MUTANTS = {
    "drop_diagonal": ("double row = (double)Q[(int64_t)i * ldq + i];", "double row = 0.0;"),
    "transposed_operand": ("row += (double)Q[(int64_t)i * ldq + j];", "row += (double)Q[(int64_t)j * ldq + i];"),
    "inner_loop_off_by_one": ("for (int j = i + 1; j < n; ++j)\n            if ((mask >> j) & 1u)\n                row += (double)",
                              "for (int j = i + 2; j < n; ++j)\n            if ((mask >> j) & 1u)\n                row += (double)"),
    "int_drop_diagonal": ("int64_t row = (int64_t)Q[(int64_t)i * ldq + i];", "int64_t row = 0;"),
    "tie_break_reversed": ("return ea < eb || (ea == eb && ma < mb);\n}\n\nstatic int before_i",
                           "return ea < eb || (ea == eb && ma > mb);\n}\n\nstatic int before_i"),
    "int_tie_break_reversed": ("return ea < eb || (ea == eb && ma < mb);\n}\n\n/* Insert",
                               "return ea < eb || (ea == eb && ma > mb);\n}\n\n/* Insert"),
    "logz_sign": ("double w = exp(-beta * e - M);", "double w = exp(beta * e - M);"),
    "grad_misses_diagonal": ("for (int j = i; j < n; ++j)", "for (int j = i + 1; j < n; ++j)"),
    "grad_sign": ("G[e] = (i <= j) ? -beta * nsum_val(&s) : 0.0;", "G[e] = (i <= j) ? beta * nsum_val(&s) : 0.0;"),
    "f64_drop_diagonal": ("double row = Q[(int64_t)i * ldq + i];", "double row = 0.0;"),
    "f64_transposed_operand": ("row += Q[(int64_t)i * ldq + j];", "row += Q[(int64_t)j * ldq + i];"),
    "i64_drop_diagonal": ("int64_t row = Q[(int64_t)i * ldq + i];", "int64_t row = 0;"),
    "f64_topk_skips_a_state": ("for (uint64_t x = a; x < b; ++x)\n            insert_d(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_d(",
                               "for (uint64_t x = a + 1; x < b; ++x)\n            insert_d(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_d("),
}

PINS = [
    pins.test_energy_equals_pair_sum_int,
    pins.test_energy_equals_pair_sum_float,
    pins.test_energy_equals_naive_xQx,
    pins.test_delta_rule_eq2,
    pins.test_ties_go_to_lowest_natural_mask,
    pins.test_c_main_example_signed_reading,
    pins.test_diagonal_closed_form,
    pins.test_logz_closed_forms,
    pins.test_grad_closed_forms,
    pins.test_grad_against_bruteforce_moments,
    pins.test_f64_energy_within_rounding_of_exact_sum,
    lambda: pins.test_topk_f64_and_i64_equal_bruteforce(5, 32),
    pins.test_i64_matches_i32_on_int32_values_and_diagonal_closed_form,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "mutant.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", "-o", str(so), str(cfile), "-lm"])
    monkeypatch.setattr(oracle, "LIB_PATH", str(so))
    monkeypatch.setattr(oracle, "_lib", None)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failures += 1
    monkeypatch.setattr(oracle, "_lib", None)
    assert failures >= 1, f"no pin caught mutant {name}"
