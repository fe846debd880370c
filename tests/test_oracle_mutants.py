"""Every plausible mistake planted in the oracle must fail at least one pin.

Each mutant is the oracle's C source with one textual change, compiled to a
temporary library on the CPU.  The list covers dropped terms, wrong signs,
swapped penalties, a transposed matrix, wrong indices and a lost floor, and
in the traceback the end-cell and tie rules, the start condition and the
gap kinds.
"""
import os
import subprocess

import pytest

import oracle
import pins

MUTANTS = {
    "drop_E_term": ("h = imax(h, e);", "(void)e;"),
    "drop_F_term": ("h = imax(h, f);", "(void)f;"),
    "drop_diag_term": ("h = imax(h, h_diag + sbt);", "(void)sbt;"),
    "no_zero_floor": ("int32_t h = 0;", "int32_t h = -1000000;"),
    "E_ext_sign": ("e_row[j] - alpha", "e_row[j] + alpha"),
    "F_ext_sign": ("f - alpha", "f + alpha"),
    "E_open_uses_alpha": ("h_row[j] - beta", "h_row[j] - alpha"),
    "F_open_uses_alpha": ("h_left - beta", "h_left - alpha"),
    "E_ext_uses_beta": ("e_row[j] - alpha", "e_row[j] - beta"),
    "transposed_matrix": ("matrix[(int32_t)q[j - 1] * alphabet + s_res]",
                          "matrix[s_res * alphabet + (int32_t)q[j - 1]]"),
    "E_from_diagonal": ("h_row[j] - beta", "h_diag - beta"),
    "stale_left": ("h_left = h;", "(void)0;"),
    "diag_not_advanced": ("h_diag = h_row[j];", "(void)0;"),
    "best_last_column_only": ("if (h > best)", "if (h > best && j == m)"),
    "best_last_row_only": ("if (h > best)", "if (h > best && i == n)"),
    "query_off_by_one": ("q[j - 1] * alphabet", "q[j < m ? j : j - 1] * alphabet"),
    # traceback (oracle_sw_align)
    "align_end_at_last_max": ("if (h > best) {", "if (h >= best) {"),
    "align_E_before_diag": ("else if (h == d) code = 0;\n            else if (h == e) code = 1;",
                            "else if (h == e) code = 1;\n            else if (h == d) code = 0;"),
    "align_F_before_diag": ("if (h == 0) code = 4;\n            else if (h == d) code = 0;",
                            "if (h == 0) code = 4;\n            else if (h == f && h != e) code = 2;\n"
                            "            else if (h == d) code = 0;"),
    "align_extend_before_open": ("if (e_open >= e_ext) code |= 8;", "if (e_open > e_ext) code |= 8;"),
    "align_runs_past_zero": ("(dir[(size_t)(i - 2) * (size_t)m + (size_t)(j - 2)] & 4)", "0"),
    "align_gap_ops_swapped": ("run_op = src == 1 ? 2u : 1u;", "run_op = src == 1 ? 1u : 2u;"),
    "align_F_open_uses_alpha": ("f_open = h_left - beta;", "f_open = h_left - alpha;"),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle.SRC) as fh:
        return fh.read()


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(tmp_path, source, name):
    before, after = MUTANTS[name]
    assert source.count(before) >= 1, f"mutation site for {name} not found"
    mutated = source.replace(before, after, 1)
    src = tmp_path / "mutant.c"
    src.write_text(mutated)
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", lib, str(src)], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    failing = pins.failing_checks(oracle.Oracle(lib))
    assert failing, f"mutant {name} passed every pin"
