"""Mutation check of the oracle's pins (CPU only).

Each mutant is a plausible mistake planted in a temporary copy of the oracle
source (a flipped sign, a wrong operator, a dropped term, a transposed index,
a swapped branch); the copy is compiled on the CPU and at least one pin must
reject it.  The real oracle is untouched.
"""
import os

import pytest

import oracle
import pins

MUTANTS = {
    "update_sign": ("fma(-f[i], p[j], T_(tb, i, j))", "fma(f[i], p[j], T_(tb, i, j))"),
    "pivot_row_mul": ("p[j] = T_(tb, l, j) / pe;", "p[j] = T_(tb, l, j) * pe;"),
    "pricing_argmin": ("if (e < 0 || v > best)", "if (e < 0 || v < best)"),
    "ratio_argmax": ("ratio < rmin ||", "ratio > rmin ||"),
    "ratio_candidates": ("if (!(a > eps_piv)) continue;", "if (!(a < -eps_piv)) continue;"),
    "dual_sign": ("y[i] = sense[i] == 0 ? -d : d;", "y[i] = -d;"),
    "phase1_dropped_terms": ("if (art[i]) acc = acc + T_(&tb, i, j);", "if (art[i]) acc = T_(&tb, i, j);"),
    "surplus_sign": ("T_(&tb, i, n + i) = art[i] ? -1.0 : 1.0;", "T_(&tb, i, n + i) = 1.0;"),
    "ge_not_negated": ("s[i] = art[i] ? (ge ? 1.0 : -1.0) : (ge ? -1.0 : 1.0);",
                       "s[i] = art[i] ? (ge ? 1.0 : -1.0) : 1.0;"),
    "infeasible_test_flipped": ("if (T_(&tb, row_w, rhs) > eps_feas * (1.0 + w0))",
                                "if (T_(&tb, row_w, rhs) < eps_feas * (1.0 + w0))"),
    "x_transposed_index": ("x[tb.basis[i]] = T_(&tb, i, rhs);", "x[tb.basis[i]] = T_(&tb, i, tb.basis[i]);"),
    "objective_sign": ("double z = -T_(&tb, row_obj, rhs);", "double z = T_(&tb, row_obj, rhs);"),
    "logicals_not_priced": ("for (int32_t j = 0; j < jart; ++j) {\n            double v = T_(&tb, ro, j);",
                            "for (int32_t j = 0; j < n; ++j) {\n            double v = T_(&tb, ro, j);"),
    "leaving_tiebreak": ("tb.basis[i] < tb.basis[l]", "tb.basis[i] > tb.basis[l]"),
    "no_anticycling": ("if (degen_run >= bland_after) {", "if (0) {"),
    "hyperbox_swapped": ("x[i] = c[i] < 0.0 ? l[i] : u[i];", "x[i] = c[i] < 0.0 ? u[i] : l[i];"),
    "hyperbox_tie_lower": ("x[i] = c[i] < 0.0 ? l[i] : u[i];", "x[i] = c[i] <= 0.0 ? l[i] : u[i];"),
    "batch_y_at_col_off": ("x + col_off[k], y + row_off[k]", "x + col_off[k], y + col_off[k]"),
    "batch_a_at_row_off": ("A + a_off[k], b + row_off[k]", "A + row_off[k], b + row_off[k]"),
    "batch_kind_inverted": ("if (kind[k] == 1) {", "if (kind[k] != 0 && m[k] != 0) {"),
    "batch_iters_not_reset": ("            iters[k] = 0;\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle.SOURCES[0]).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/absent"
    mpath = os.path.join(tmp_path, "mutant.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.lib(oracle.build(src=mpath, out=os.path.join(tmp_path, "libmutant.so")))
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} survived every pin"
