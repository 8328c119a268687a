"""Plausible mistakes planted in a copy of the oracle (on the CPU) must each fail a pin.

Each mutation is a textual edit of oracle/omp_oracle.c: a dropped term, a wrong
sign, a wrong index, a transposed operand, a wrong comparison. The mutant is
compiled into a temporary directory and run through every pin; at least one pin
must raise. This shows the pins constrain the oracle rather than restate it.
"""
import os
import shutil
import subprocess

import pytest

from tests.oracle_pins import PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "omp_oracle.c")

MUTATIONS = {
    "no_column_normalisation": ("double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, r, M)) / nu[n];",
                                "double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, r, M));"),
    "no_abs": ("double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, r, M)) / nu[n];",
               "double s = dot_atom(A + (size_t)n * (size_t)lda, r, M) / nu[n];"),
    "norm_squared": ("nu[n] = sqrt(s);", "nu[n] = s;"),
    "select_with_y": ("double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, r, M)) / nu[n];",
                      "double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, yd, M)) / nu[n];"),
    "tie_to_highest": ("if (s > best) { second = best;", "if (s >= best) { second = best;"),
    "no_second_track": ("else if (s > second) second = s;", "else if (s > second) second = s * 0.5;"),
    "no_mask": ("if (selected[n] || nu[n] == 0.0) continue;", "if (nu[n] == 0.0) continue;"),
    "backsub_transposed": ("s -= W[(size_t)c * M + i] * x[c];", "s -= W[(size_t)i * M + c] * x[c];"),
    "residual_sign": ("for (int m = 0; m < M; ++m) r[m] -= (double)a[m] * x[j];",
                      "for (int m = 0; m < M; ++m) r[m] += (double)a[m] * x[j];"),
    "residual_drops_last": ("    for (int j = 0; j < k; ++j) {\n      const float *a = A + (size_t)support[j] * (size_t)lda;\n      for (int m = 0; m < M; ++m) r[m] -=",
                            "    for (int j = 0; j < k - 1; ++j) {\n      const float *a = A + (size_t)support[j] * (size_t)lda;\n      for (int m = 0; m < M; ++m) r[m] -="),
    "reflector_not_applied_to_b": ("for (int i = j; i < M; ++i) b[i] -= t * wj[i];", "(void)t;"),
    "stop_on_ge": ("while (k < S && rn > eps_eff)", "while (k < S && rn >= eps_eff)"),
    "householder_beta_wrong": ("double beta = (vtv > 0.0) ? 2.0 / vtv : 0.0;", "double beta = (vtv > 0.0) ? 1.0 / vtv : 0.0;"),
    "per_signal_eps_ignored": ("double eb = eps_arr ? (double)eps_arr[b] : eps;", "double eb = eps;"),
    "per_signal_S_ignored": ("int Sb = S_arr ? S_arr[b] : S;", "int Sb = S;"),
    "per_signal_eps_wrong_row": ("double eb = eps_arr ? (double)eps_arr[b] : eps;",
                                 "double eb = eps_arr ? (double)eps_arr[0] : eps;"),
    "per_signal_S_wrong_row": ("int Sb = S_arr ? S_arr[b] : S;", "int Sb = S_arr ? S_arr[b > 0 ? b - 1 : 0] : S;"),
    "forced_pick_scored_as_best": ("      spick = fabs(dot_atom(A + (size_t)pick * (size_t)lda, r, M)) / nu[pick];",
                                   "      spick = best;"),
    "forced_prefix_ignored": ("    if (k < nprefix) {\n      pick = prefix[k];", "    if (k < 0) {\n      pick = prefix[k];"),
    "forced_prefix_one_short": ("    if (k < nprefix) {\n      pick = prefix[k];", "    if (k + 1 < nprefix) {\n      pick = prefix[k];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_fails_a_pin(orc, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib_path = str(tmp_path / "libmutant.so")
    orc.build(str(mpath), lib_path)
    lib = orc.load(lib_path)
    failed = []
    for pin in PINS:
        try:
            pin(orc, lib)
        except (AssertionError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"mutation {name} passed every pin"
