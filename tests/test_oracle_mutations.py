"""Planted mistakes: each case patches a copy of the oracle's C source with a
plausible error (dropped term, wrong tie rule, transposed index, missing
normalisation, the literal ICP start at zero, ...), builds it in a temp dir and
checks that at least one pin from test_oracle_pins fails against it.  This
shows the pins constrain every part of the oracle.  All on the CPU."""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "sivf_oracle.c")).read()

MUTATIONS = {
    "tie_highest_index": (
        "                    if (r > best) {\n                        second = best;",
        "                    if (r >= best) {\n                        second = best;",
        [lambda: pins.test_dyadic_golden_iteration_by_iteration(),
         lambda: pins.test_exact_ties_break_to_lowest_index()]),
    "icp_start_at_zero_as_printed": (
        "                best = own_prev[i];",
        "                best = 0.0;",
        [lambda: pins.test_icp_filtered_equals_unfiltered_every_iteration(1)]),
    "transposed_dense_index": (
        "            if (r >= 0) mt[r * k + j] = cval[p];",
        "            if (r >= 0) mt[(int64_t)j * used + r] = cval[p];",
        [lambda: pins.test_assign_matches_exact_rational_argmax(0)]),
    "dropped_last_term": (
        "            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {\n                double v = xval(val, val_f64, p);",
        "            for (int64_t p = rp[i]; p + 1 < rp[i + 1]; ++p) {\n                double v = xval(val, val_f64, p);",
        [lambda: pins.test_assign_matches_exact_rational_argmax(1)]),
    "missing_normalisation": (
        "                    rv[j][e] = w[p] / nr;",
        "                    rv[j][e] = w[p];",
        [lambda: pins.test_update_matches_dense_numpy(pins.np.float64)]),
    "wrong_sign_in_sum": (
        "w[col[p]] = w[col[p]] + xval(val, val_f64, p);",
        "w[col[p]] = w[col[p]] - xval(val, val_f64, p);",
        [lambda: pins.test_update_matches_dense_numpy(pins.np.float64)]),
    "empty_cluster_zeroed": (
        "                int64_t m = prev_cp[j + 1] - prev_cp[j];\n                nnz[j] = m;",
        "                int64_t m = 0;\n                nnz[j] = m;",
        [lambda: pins.test_empty_cluster_keeps_previous_centroid()]),
    "square_not_summed_in_order": (
        "            for (int64_t p = 0; p < d; ++p) s = s + w[p] * w[p];",
        "            for (int64_t p = 0; p < d; ++p) s = s + w[p];",
        [lambda: pins.test_update_matches_dense_numpy(pins.np.float64)]),
    "invariant_part_first": (
        "        q0[s] = term_ptr[s];\n        q1[s] = term_ptr[s] + mf0[s];",
        "        q0[s] = term_ptr[s] + mf1[s];\n        q1[s] = term_ptr[s];",
        [lambda: pins.test_ivf_layout_and_roundtrip()]),
    "relaxed_icp_condition_reversed": (
        "acc[a_prev[i]] >= own_prev[i];",
        "acc[a_prev[i]] <= own_prev[i];",
        [lambda: pins.test_relaxed_icp_equals_unfiltered_every_iteration(3)]),
    "cbicp_counts_invariant": (
        "c += (lam_prev[cid[q]] == 0);",
        "c += (lam_prev[cid[q]] != 0);",
        [lambda: pins.test_sivf_and_cbicp_counts_equal_and_not_above_ivf()]),
    "soft_missing_tau_in_grad": (
        "ds[j] = -g * exp(s[j] / tau - lse[q]) / tau;",
        "ds[j] = -g * exp(s[j] / tau - lse[q]);",
        [lambda: pins.test_soft_backward_finite_differences()]),
    "soft_lse_without_shift": (
        "    return m + log(z);",
        "    return log(z);",
        [lambda: pins.test_soft_forward_matches_scipy_logsumexp()]),
    "soft_dx_wrong_operand": (
        "acc = acc + ds[j] * C[(int64_t)j * d + col[p]];",
        "acc = acc + ds[j] * C[(int64_t)j * d + (col[p] + 1) % d];",
        [lambda: pins.test_soft_backward_finite_differences()]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new, checks = MUTATIONS[name]
    assert SRC.count(old) == 1, "mutation anchor must match exactly once"
    src = tmp_path / "mut.c"
    src.write_text(SRC.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, str(src), "-o", str(so), "-lm"])
    saved = oracle._load()
    oracle._lib = oracle._bind(str(so))
    try:
        failed = 0
        for chk in checks:
            try:
                chk()
            except AssertionError:
                failed += 1
        assert failed >= 1, "no pin caught mutation %r" % name
    finally:
        oracle._lib = saved
