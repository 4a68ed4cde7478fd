"""Planted mistakes in a copy of the oracle must be caught by its pins.

Each case applies one textual change to a temporary copy of the C oracle
(never to the committed file), builds it with gcc, and runs the pin suite
against that build in a subprocess; the suite must fail.  CPU only.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fps_oracle.c")

MUTANTS = {
    "tie_dropped": ("if (fabs(x) < jb->tau) {", "if (fabs(x) <= jb->tau) {"),
    "zeros_kept": ("if (x == 0.0) {", "if (x != x) {"),
    "block_skipped_in_step": ("w->acc[c] = E->val[p] + w->acc[c];", "w->acc[c] = 0.0 + w->acc[c];"),
    "identity_term_lost": ("w->acc[r] = fma(a, 1.0, w->acc[r]);", "w->acc[r] = fma(a, 0.0, w->acc[r]);"),
    "coefficient_index_shift": ("const int k = i * q + j;", "const int k = i * q + j + (j > 0);"),
    "shortcut_ignored": ("        if (g) {\n", "        if (0) {\n"),
    "horner_step_missing": ("for (int i = start; i <= b - 1 && rc == ORC_OK; ++i)",
                            "for (int i = start + 1; i <= b - 1 && rc == ORC_OK; ++i)"),
    "powers_not_filtered": ("rc = orc_spgemm(Z, Pp[j], NULL, tau, &P[j + 1], &st, nthreads);",
                            "rc = orc_spgemm(Z, Pp[j], NULL, 0.0, &P[j + 1], &st, nthreads);"),
    "horner_not_filtered": ("rc = orc_spgemm(Pp[q], &S, &Bh, tau, &T, &st, nthreads);",
                            "rc = orc_spgemm(Pp[q], &S, &Bh, 0.0, &T, &st, nthreads);"),
    "transposed_left_operand": ("const double a = A->val[p];\n            for (int64_t t = B->row_ptr[k];",
                                "const double a = A->val[p];\n            for (int64_t t = B->row_ptr[k]; (void)0,"),
    "product_weight_dropped": ("w->acc[c] = fma(a, B->val[t], w->acc[c]);",
                               "w->acc[c] = fma(1.0, B->val[t], w->acc[c]);"),
    "dropped_norm_not_recorded": ("w->drop_colsum[c] += fabs(x);", "w->drop_colsum[c] += 0.0;"),
    "alg1_candidate_tie": ("if (a > 0.0 && a <= t) cs[C->col[p]]", "if (a > 0.0 && a < t) cs[C->col[p]]"),
    "alg1_drop_tie": ("if (fabs(C->val[p]) <= t) continue;", "if (fabs(C->val[p]) < t) continue;"),
    "alg1_single_iteration": ("} while (c > target && it < max_iter);", "} while (0);"),
    "alg1_threshold_update": ("        m = c / t;\n", "        m = c * t;\n"),
    "fnt_wrong_power_norm": ("d = d + z[q * (b - 1 - j)] * (beta + z[q - k] * sprev);",
                             "d = d + z[q * (b - 1 - j)] * (beta + z[q - k + 1] * sprev);"),
    "fnt_budget_not_shared": ("zeta[k] = eps / (d * M);", "zeta[k] = eps / d;"),
    "fnt_beta_power_shift": ("beta = beta + A_(i * q + kk) * z[kk - k];", "beta = beta + A_(i * q + kk) * z[kk - k + 1];"),
    "fnt_state_norm_no_power": ("ns[i] = nb[b - 1 - i] + z[q] * ns[i - 1];", "ns[i] = nb[b - 1 - i] + ns[i - 1];"),
    "fnt_sigma_weight_shift": ("sigma[j] = eps / (z[q * (b - 1 - j)] * M);",
                               "sigma[j] = eps / (z[q * (b - 1 - j) + (j > 0)] * M);"),
    "alg1_norm_rounded_down": ("cs[C->col[p]] += (uint64_t)ceil(a * s);", "cs[C->col[p]] += (uint64_t)floor(a * s);"),
    "adaptive_horner_unfiltered": ("if (rc == ORC_OK) rc = orc_alg1_filter(&T, sigma[i], e_r, 200, &a1);",
                                   "if (rc == ORC_OK) rc = orc_alg1_filter(&T, INFINITY, e_r, 200, &a1);"),
    "normest_no_transpose": ("apply_power(Z, p, 1, s, zt, tmp);", "apply_power(Z, p, 0, s, zt, tmp);"),
    "normest_first_iterate_only": ("if (k > itmax) break;", "if (k > 0) break;"),
    "normest_argmax_is_min": ("if (fabs(zt[i]) > hmax) {", "if (hmax < 0.0 || fabs(zt[i]) < hmax) {"),
    "lemma1_alpha_min": ("if (r > alpha) alpha = r;", "if (alpha == 0.0 || r < alpha) alpha = r;"),
    "lemma1_no_root": ("const double r = pow(z[k], 1.0 / (double)k);", "const double r = z[k];"),
    "theta_off_by_one": ("if (T[m] <= 0.5 * eps_tol) {", "if (T[m + 1] <= 0.5 * eps_tol) {"),
    "theta_full_budget": ("if (T[m] <= 0.5 * eps_tol) {", "if (T[m] <= eps_tol) {"),
    "theta_tail_index": ("T[m] = T[m + 1] + fabs(a[m]) * z[m];", "T[m] = T[m + 1] + fabs(a[m]) * z[m + 1];"),
    "q_ceil_sqrt": ("while ((int64_t)(q + 1) * (q + 1) <= (int64_t)(N - 1)) ++q;",
                    "while ((int64_t)q * q < (int64_t)(N - 1)) ++q;"),
}


MULTI = {"shortcut_ignored", "horner_step_missing"}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    if name == "transposed_left_operand":
        # replace the product loop by one over the transpose of the left operand:
        # row r takes column r of A (a transposed operand), found by a scan
        old = ("        for (int64_t p = A->row_ptr[r]; p < A->row_ptr[r + 1]; ++p) {\n"
               "            const int64_t k = A->col[p];\n"
               "            const double a = A->val[p];\n")
        new = ("        for (int64_t kk = 0; kk < A->n; ++kk)\n"
               "        for (int64_t p = A->row_ptr[kk]; p < A->row_ptr[kk + 1]; ++p) {\n"
               "            if (A->col[p] != r) continue;\n"
               "            const int64_t k = kk;\n"
               "            const double a = A->val[p];\n")
    # the schedule logic appears in both drivers (fixed and adaptive filter); a
    # mistake there is planted in every copy
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    if name not in MULTI:
        assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_exact.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
