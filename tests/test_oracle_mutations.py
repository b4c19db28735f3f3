"""The oracle pins must catch plausible mistakes: each case plants one mistake in a copy
of the oracle source (on the CPU), builds it, and checks that the pin suite fails."""
import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "vbarms_oracle.c")

MUTATIONS = {
    "cosine_strict": ("if (lhs >= rhs) group[j] = i;", "if (lhs > rhs) group[j] = i;"),
    "cosine_no_square": ("double lhs = (double)c * (double)c;", "double lhs = (double)c;"),
    "gepp_update_sign": ("a[r * m + c] = a[r * m + c] - a[r * m + k] * a[k * m + c];",
                         "a[r * m + c] = a[r * m + c] + a[r * m + k] * a[k * m + c];"),
    "gepp_no_row_swap": ("if (pr != k)\n            for (int c = 0; c < m; ++c)", "if (0)\n            for (int c = 0; c < m; ++c)"),
    "fwd_skips_swaps": ("if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }\n    for (int r = 0; r < m; ++r) {",
                        "if (0) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }\n    for (int r = 0; r < m; ++r) {"),
    "row_solve_u_multiplies": ("e[c] = s / lu[c * m + c];", "e[c] = s * lu[c * m + c];"),
    "row_solve_lp_swap_order": ("for (int k = m - 1; k >= 0; --k)\n        if (piv[k] != k) { double t = e[k];",
                                "for (int k = 0; k < m; ++k)\n        if (piv[k] != k) { double t = e[k];"),
    "drop_no_square": ("return s < thr * thr;", "return s < thr;"),
    "schur_sign": ("s[r * nK + c] = s[r * nK + c] - wb[r * mi + q] * gb[q * nK + c];",
                   "s[r * nK + c] = s[r * nK + c] + wb[r * mi + q] * gb[q * nK + c];"),
    "schur_transposed_g": ("- wb[r * mi + q] * gb[q * nK + c];", "- wb[r * mi + q] * gb[c * mi + q];"),
    "scale_cols_unscaled": ("double v = fabs(L->s1[A->rb[I] + r] * b[r * nJ + c]);", "double v = fabs(b[r * nJ + c]);"),
    "indset_one_direction": ("for (int64_t k = tp[I]; k < tp[I + 1]; ++k) marked[tr[k]] = 1;", ""),
    "ilut_update_sign": ("wj[r * nJ + c] = wj[r * nJ + c] - wk[r * mk + q] * ub[q * nJ + c];",
                         "wj[r * nJ + c] = wj[r * nJ + c] + wk[r * mk + q] * ub[q * nJ + c];"),
    "ilut_keeps_dropped_multiplier": ("if (drop_block(m, mk, wk, t)) { state[k] = 2; continue; }", ""),
    "ilut_drop_before_solve": (
        "for (int r = 0; r < m; ++r) { row_solve_u(mk, dk, wk + r * mk); row_solve_lp(mk, dk, pk, wk + r * mk); }\n"
        "            if (drop_block(m, mk, wk, t)) { state[k] = 2; continue; }",
        "if (drop_block(m, mk, wk, t)) { state[k] = 2; continue; }\n"
        "            for (int r = 0; r < m; ++r) { row_solve_u(mk, dk, wk + r * mk); row_solve_lp(mk, dk, pk, wk + r * mk); }"),
    "ilut_u_test_square": ("if (K > i && !drop_block(m, bm_cs(A, K), acc + slot[K], t))",
                           "if (K > i && !drop_block(m, m < bm_cs(A, K) ? m : bm_cs(A, K), acc + slot[K], t))"),
    "ilut_u_never_dropped": ("if (K > i && !drop_block(m, bm_cs(A, K), acc + slot[K], t))",
                             "if (K > i && (t <= 1.0 || !drop_block(m, bm_cs(A, K), acc + slot[K], t)))"),
    "weighted_order_ascending": ("if (a->w > b->w) return -1;\n    if (a->w < b->w) return 1;",
                                 "if (a->w > b->w) return 1;\n    if (a->w < b->w) return -1;"),
    "weighted_order_no_diag_norm_root": ("double f = sqrt(ss);", "double f = ss;"),
    "graph_strict_threshold": ("if ((double)nnz >= mu * (double)el) {", "if ((double)nnz > mu * (double)el) {"),
    "graph_row_adjacency_only": ("{ adj[af[i]++] = col[k]; adj[af[col[k]]++] = i; }", "{ adj[af[i]++] = col[k]; }"),
    "graph_candidates_descending": ("while (b >= 0 && first[cand[b]] > first[v])", "while (b >= 0 && first[cand[b]] < first[v])"),
    "graph_no_diagonal_blocks": ("        stamp[I] = I;\n        elems += (int64_t)sz[I] * sz[I];\n", ""),
    "apply_wrong_output_scale": ("x[rows[r]] = L->s2[rows[r]] * z[L->rest_rb[j] + r];",
                                 "x[rows[r]] = L->s1[rows[r]] * z[L->rest_rb[j] + r];"),
    "group_seed_neighbours_only": ("        for (int a = 0; a < nm; ++a) {\n            int I = mem[a];",
                                   "        for (int a = 0; a < 1; ++a) {\n            int I = mem[a];"),
    "group_cap_strict": ("if (rows + bm_rs(A, u) > gmax) continue;", "if (rows + bm_rs(A, u) >= gmax) continue;"),
    "group_stop_at_first_misfit": ("if (rows + bm_rs(A, u) > gmax) continue;", "if (rows + bm_rs(A, u) > gmax) break;"),
    "group_w_member_offset": ("tmp[r * mg + goff[I] + c] = eb[r * nI + c];", "tmp[r * mg + c] = eb[r * nI + c];"),
    "group_g_member_offset": ("tmp[(goff[I] + r) * nJ + c] = fb[r * nJ + c];", "tmp[r * nJ + c] = fb[r * nJ + c];"),
    "group_d_offsets_swapped": ("d[(goff[I] + r) * m + goff[J] + c] = blk[r * nJ + c];",
                                "d[(goff[J] + r) * m + goff[I] + c] = blk[r * nJ + c];"),
    "group_opening_order": ("        if (gid[I] >= 0) gid[I] = gnew[gid[I]];", "        if (gid[I] >= 0) gid[I] = gid[I];"),
    "group_apply_reads_packed_rows": ("for (int r = 0; r < m; ++r) yi[r] = L->s1[rows[r]] * b[rows[r]];",
                                      "for (int r = 0; r < m; ++r) yi[r] = L->s1[rows[r]] * b[L->is_rb[i] + r];"),
    "apply_skips_g_correction": ("yi[r] = yi[r] - gb[r * nK + q] * z[L->rest_rb[K] + q];", "yi[r] = yi[r];"),
    "last_solve_skips_l": ("for (int q = 0; q < nK; ++q) xi[r] = xi[r] - b[r * nK + q] * xk[q];\n        }\n    }\n    for (int i = p - 1;",
                           "for (int q = 0; q < nK; ++q) xi[r] = xi[r];\n        }\n    }\n    for (int i = p - 1;"),
    "gmres_givens_sign": ("H[(k + 1) * m + j] = -sn[k] * a + cs[k] * c;", "H[(k + 1) * m + j] = sn[k] * a + cs[k] * c;"),
    "gmres_mgs_uses_stale": ("double hk = dot(n, vn, V + (size_t)k * n);", "double hk = dot(n, V + (size_t)j * n, V + (size_t)k * n);"),
    "vbcsr_transposed_entry": ("row[boff[lo] + (int64_t)(r - bptr[I]) * nJ + (c - bptr[J])] = val[k];",
                               "row[boff[lo] + (int64_t)(c - bptr[J]) * m + (r - bptr[I])] = val[k];"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(lib), str(mutated), "-lm"])
    env = dict(os.environ, VBARMS_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutation {name}:\n{r.stdout[-2000:]}"
