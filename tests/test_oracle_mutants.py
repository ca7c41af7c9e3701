"""Plant plausible mistakes in a copy of the oracle source and check that at
least one pin catches each of them (a dropped term, a wrong sign, index or
comparison, a transposed operand, the garbled pseudocode read literally).
Each mutant is a text substitution that must match exactly once."""
import os
import shutil
import tempfile

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "pr_oracle.c")

MUTANTS = {
    "eq2_drops_self_term": ("(C0 + alpha * (c - R[v] / dv))", "(C0 + alpha * (c))"),
    "eq2_sign": ("1.0 / (1.0 - alpha / dv)", "1.0 / (1.0 + alpha / dv)"),
    "frontier_flag_literal_zero": ("if (rel > tau_f) dN[v] = 1;", "if (rel > tau_f) dN[v] = 0;"),
    "no_carry_forward": ("if (!dV[v]) { Rn[v] = R[v]; continue; }", "if (!dV[v]) { continue; }"),
    "teleport_not_divided_by_n": ("const double C0 = (1.0 - alpha) / (double)n;\n  int32_t it = 0;\n  double d = 0.0;\n  int converged = 0;\n  const double t0",
                                  "const double C0 = (1.0 - alpha);\n  int32_t it = 0;\n  double d = 0.0;\n  int converged = 0;\n  const double t0"),
    "static_no_damping": ("Rn[v] = C0 + alpha * c;\n    }", "Rn[v] = C0 + c;\n    }"),
    "in_lists_transposed": ("a->in_src[i] = src[a->in_eid[i]];", "a->in_src[i] = dst[a->in_eid[i]];"),
    "outdeg_from_in_lists": ("a->out_deg[u] = (int32_t)(a->out_off[u + 1] - a->out_off[u]);",
                             "a->out_deg[u] = (int32_t)(a->in_off[u + 1] - a->in_off[u]);"),
    "stop_strict_less": ("if (d <= tol) { converged = 1; break; }\n  }\n  if (seconds)", "if (d < tol) { converged = 1; break; }\n  }\n  if (seconds)"),
    "dfp_stop_strict_less": ("if (d <= tol) { converged = 1; break; }\n    expand_affected", "if (d < tol) { converged = 1; break; }\n    expand_affected"),
    "linf_is_l1": ("if (t > d) d = t;", "d += t;"),
    "deletion_target_unmarked": ("dN[del_src[i]] = 1; dV[del_dst[i]] = 1;", "dN[del_src[i]] = 1;"),
    "expand_over_in_lists": ("for (int64_t i = a->out_off[u]; i < a->out_off[u + 1]; ++i) dV[a->out_tgt[i]] = 1;",
                             "for (int64_t i = a->in_off[u]; i < a->in_off[u + 1]; ++i) dV[a->in_src[i]] = 1;"),
    "prune_uses_frontier_direction": ("if (prune && rel <= tau_p) dV[v] = 0;", "if (prune && rel > tau_p) dV[v] = 0;"),
    "relative_change_min": ("double rel = dr / (r > R[v] ? r : R[v]);", "double rel = dr / (r < R[v] ? r : R[v]);"),
    "ppr_teleport_index_transposed": ("(1.0 - alpha) * s[(size_t)v * (size_t)k + (size_t)j]", "(1.0 - alpha) * s[(size_t)j * (size_t)n + (size_t)v]"),
    "weighted_weight_of_wrong_edge": ("c = c + w[a.in_eid[i]] * R[a.in_src[i]];", "c = c + w[a.out_eid[i]] * R[a.in_src[i]];"),
    "adjoint_transposed": ("c = c + w[a.out_eid[i]] * L[a.out_tgt[i]];", "c = c + w[a.in_eid[i]] * L[a.in_src[i]];"),
    "adjoint_edge_grad_transposed": ("grad_w[e] = alpha * r[src[e]] * L[dst[e]];", "grad_w[e] = alpha * r[dst[e]] * L[src[e]];"),
    "adjoint_grad_s_undamped": ("grad_s[v] = (1.0 - alpha) * L[v];", "grad_s[v] = L[v];"),
    "dt_closure_one_level": ("while (head < tail) {", "while (0) {"),
    "rows_outdeg_of_target": ("else c = c + x / (double)(out_off[u + 1] - out_off[u]);",
                              "else c = c + x / (double)(out_off[v + 1] - out_off[v]);"),
    "rows_undamped": ("out[i] = t + alpha * c;", "out[i] = t + c;"),
    "rows_teleport_vector_major": ("(1.0 - alpha) * s[(size_t)v * (size_t)ld + (size_t)j] : C0;",
                                   "(1.0 - alpha) * s[(size_t)j * (size_t)n + (size_t)v] : C0;"),
    "rows_weight_ignored": ("if (w) c = c + w[e] * x;", "if (w) c = c + x;"),
    "dt_deletion_target_unmarked": ("{ dV[del_dst[i]] = 1; dN[del_src[i]] = 1; }", "{ dN[del_src[i]] = 1; }"),
    "df_uses_eq2": ("else r = C0 + alpha * c;",
                    "else r = 1.0 / (1.0 - alpha / dv) * (C0 + alpha * (c - R[v] / dv));"),
    "nd_ignores_start_vector": ("R[v] = Rn[v] = init ? init[v] : 1.0 / (double)n;\n  const double C0",
                                "R[v] = Rn[v] = 1.0 / (double)n;\n  const double C0"),
    "weighted_ignores_start_vector": ("R[v] = Rn[v] = init ? init[v] : 1.0 / (double)n;\n  int32_t it",
                                      "R[v] = Rn[v] = 1.0 / (double)n;\n  int32_t it"),
    "edges_processed_doubled": ("edges += a.in_off[v + 1] - a.in_off[v];",
                                "edges += 2 * (a.in_off[v + 1] - a.in_off[v]);"),
    "affected_max_frozen_at_initial": ("if (aff > affmax) affmax = aff;", "affmax = aff0;"),
    "affected_ever_initial_only": ("if (dV[v]) ever[v] = 1;", "if (dV[v] && it == 0) ever[v] = 1;"),
}


def test_mutations_match_exactly_once():
    text = open(SRC).read()
    for name, (old, _) in MUTANTS.items():
        assert text.count(old) == 1, name


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_some_pin_catches(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1
    mdir = tmp_path / "oracle_mutant"
    mdir.mkdir()
    src = mdir / "pr_oracle.c"
    src.write_text(text.replace(old, new))
    so = str(mdir / "liboracle_mutant.so")
    import subprocess
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-shared", "-fPIC", "-o", so,
                    str(src), "-lm"], check=True)
    lib = oracle.load(so)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError, FloatingPointError):
            caught.append(pin.__name__)
    assert caught, f"no pin detects mutant {name}"
