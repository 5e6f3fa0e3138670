"""Planted mistakes in a copy of the oracle must fail the pins (no GPU).

Each case below edits one step of the oracle's source in a temporary copy
(a dropped term, a wrong sign, an exchanged operand, a wrong index), builds
it, routes the oracle through it, and checks that at least one of the pin
tests named for it fails.  The committed oracle is never modified.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_apps as A
import test_oracle_bounds as B
import test_oracle_coupled as CP
import test_oracle_eft as E
import test_oracle_paper as P
import test_oracle_tree as T

SRC = os.path.dirname(oracle.__file__)

F64, F32 = np.float64, np.float32

MUTANTS = [
    # (name, original text, planted text, pins expected to catch it)
    ("two_diff_printed_orientation",
     "T b_lost = b_virt - b;\n    T a_lost = a - a_virt;",
     "T b_lost = b - b_virt;\n    T a_lost = a_virt - a;",
     [lambda: E.test_two_diff_is_exact(F64)]),
    ("two_sum_dropped_a_part",
     "r.z1 = a_lost + b_lost;\n    return r;\n}\n\n/* Two-Diff",
     "r.z1 = b_lost;\n    return r;\n}\n\n/* Two-Diff",
     [lambda: E.test_two_sum_is_exact(F64)]),
    ("atf1_wrong_sign",
     "z.z1 = (x1 + y1) + s.z1;",
     "z.z1 = (x1 - y1) + s.z1;",
     [lambda: B.test_general_twofold_bound("add", F64)]),
    ("stf1_dotted_x_wrong_sign",
     "z.z1 = d.z1 - y1;",
     "z.z1 = d.z1 + y1;",
     [lambda: E.test_add_sub_with_dotted_operand_is_strict(F64, "sub")]),
    ("mtf1_dropped_p11",
     "z.z1 = (p.z1 + p11) + (p01 + p10);",
     "z.z1 = p.z1 + (p01 + p10);",
     [lambda: B.test_general_twofold_bound("mul", F64)]),
    ("mtf1_exchanged_operand",
     "T p10 = x1 * y0;\n    T p11 = x1 * y1;",
     "T p10 = x1 * y1;\n    T p11 = x1 * y1;",
     [lambda: B.test_general_twofold_bound("mul", F64)]),
    ("mtf1_dropped_e00",
     "z.z1 = (p.z1 + p11) + (p01 + p10);",
     "z.z1 = p11 + (p01 + p10);",
     [lambda: B.test_general_twofold_bound("mul", F64)]),
    ("dtf1_dropped_r1",
     "T c0 = r0 + r1;\n    T d0 = y0 + y1;",
     "T c0 = r0;\n    T d0 = y0 + y1;",
     [lambda: B.test_general_twofold_bound("div", F64)]),
    ("dtf1_divisor_not_renormalised",
     "T d0 = y0 + y1;",
     "T d0 = y0;",
     [lambda: B.test_general_twofold_bound("div", F64)]),
    ("dtf111_remainder_sign",
     "T r1 = FMA(-z0, y0, x0);\n    PAIR z;",
     "T r1 = FMA(z0, y0, -x0);\n    PAIR z;",
     [lambda: E.test_dotted_division_is_strict_and_coupled(F64)]),
    ("rpf1_dropped_low_part",
     "v.z1 = (u1 + h) / ((T)2 * v0);",
     "v.z1 = h / ((T)2 * v0);",
     [lambda: B.test_sqrt_bound(F64), lambda: P.test_worked_examples(P.EXAMPLES["examples"][2], F64)]),
    ("rtf1_final_sum_wrong_sign",
     "z.z1 = w.z0 + w.z1;",
     "z.z1 = w.z0 - w.z1;",
     [lambda: B.test_sqrt_bound(F64)]),
    ("axpy_exchanged_scalar_part",
     "PAIR t = x1 ? NM(mul_tt)(a[0], a[1], x0[i], x1[i])",
     "PAIR t = x1 ? NM(mul_tt)(a[0], a[0], x0[i], x1[i])",
     [lambda: B.test_axpy_bound(F64)]),
    ("horner_wrong_coefficient_index",
     "r = NM(add_td)(m.z0, m.z1, c[k]);",
     "r = NM(add_td)(m.z0, m.z1, c[k + 1]);",
     [lambda: B.test_horner_bound(F64)]),
    ("tree_strided_pairing",
     "node[i] = NM(add_tt)(node[2 * i].z0, node[2 * i].z1,\n                                 node[2 * i + 1].z0, node[2 * i + 1].z1);",
     "node[i] = NM(add_tt)(node[i].z0, node[i].z1,\n                                 node[i + w / 2].z0, node[i + w / 2].z1);",
     [lambda: T.test_z0_is_the_plain_pairwise_sum(1000, F64)]),
    ("tree_node_error_dropped",
     "    for (int64_t w = m; w > 1; w /= 2)\n        for (int64_t i = 0; i < w / 2; ++i)\n            node[i] = NM(add_tt)(",
     "    for (int64_t w = m; w > 1; w /= 2)\n        for (int64_t i = 0; i < w / 2; ++i)\n            node[i] = NM(plainish_add)(",
     [lambda: T.test_dot_against_exact_rational(1e8, F64)]),
    ("tree_tile_padding_index",
     "node[i] = base + i < n",
     "node[i] = base + i + 1 < n",
     [lambda: T.test_z0_is_the_plain_pairwise_sum(1000, F64)]),
    ("fp64_reference_deviation_sign",
     "dz[i] = (Z0[i] - (double)z0[i]) + Z1[i];",
     "dz[i] = ((double)z0[i] - Z0[i]) + Z1[i];",
     [lambda: B.test_fp32_against_fp64_reference("add")]),
    ("fp32_mirror_two_sum_lost_part",
     "T b_lost = b - b_virt;  /* what b lost in the rounding */",
     "T b_lost = b_virt - b;  /* what b lost in the rounding */",
     [lambda: E.test_two_sum_is_exact(F32)]),
    ("fast_two_sum_lost_part_sign",
     "r.z1 = b - bv;",
     "r.z1 = bv - b;",
     [lambda: CP.test_fast_two_sum_is_exact_when_ordered(F64)]),
    ("mpf1_keeps_p11",
     "z.z1 = p.z1 + (p01 + p10);\n    return z;\n}\n\n/* DPF1",
     "z.z1 = (p.z1 + x1 * y1) + (p01 + p10);\n    return z;\n}\n\n/* DPF1",
     [lambda: CP.test_mpf1_exact_cases(F64)]),
    ("mpf1_dropped_p10",
     "z.z1 = p.z1 + (p01 + p10);\n    return z;\n}\n\n/* DPF1",
     "z.z1 = p.z1 + p01;\n    return z;\n}\n\n/* DPF1",
     [lambda: CP.test_mpf1_bound_on_coupled_operands(F64)]),
    ("dpf1_divides_by_the_full_divisor",
     "z.z1 = c0 / y0;\n    return z;\n}\n\n/* One coupled",
     "z.z1 = c0 / (y0 + y1);\n    return z;\n}\n\n/* One coupled",
     [lambda: CP.test_dpf1_exact_cases(F64)]),
    ("dtf1_dotted_dividend_drops_y1",
     "return NM(div_tt)(x0, (T)0, y0, y1);",
     "return NM(div_tt)(x0, (T)0, y0, (T)0);",
     [lambda: B.test_div_with_dotted_dividend(F64), lambda: P.test_dtf1_example_with_dotted_dividend(F64)]),
    ("dpf1_dotted_dividend_drops_y1",
     ": yt ? NM(div_pp)(x0, (T)0, y0, y1)",
     ": yt ? NM(div_pp)(x0, (T)0, y0, (T)0)",
     [lambda: CP.test_dpf1_dotted_dividend_exact_cases(F64)]),
    ("dpf1_r1_sign",
     "T r1 = FMA(-z0, y1, x1);\n    T c0 = r0 + r1;\n    PAIR z;",
     "T r1 = FMA(z0, y1, x1);\n    T c0 = r0 + r1;\n    PAIR z;",
     [lambda: CP.test_dpf1_bound_on_coupled_operands(F64)]),
    ("dekker_chain_skips_renormalising",
     "if (mode == 2) z = NM(fast_two_sum)(z.z0, z.z1);",
     "if (mode == 3) z = NM(fast_two_sum)(z.z0, z.z1);",
     [CP.test_counting_ones_saturates_without_renormalising]),
    ("trsv_adds_the_product",
     "s = NM(sub_tt)(s.z0, s.z1, p.z0, p.z1);",
     "s = NM(add_tt)(s.z0, s.z1, p.z0, p.z1);",
     [lambda: A.test_jordan_block_logs_through_the_batched_solver("double")]),
    ("trsv_wrong_row_index",
     "int64_t a = ((int64_t)i * m + j) * nsys + k, b = (int64_t)j * nsys + k;",
     "int64_t a = ((int64_t)j * m + i) * nsys + k, b = (int64_t)j * nsys + k;",
     [lambda: A.test_exact_systems_are_solved_exactly(4, F64)]),
    ("quadratic_wrong_constant",
     "PAIR a4 = NM(mul_tt)((T)4, (T)0, a0[i], a1[i]);",
     "PAIR a4 = NM(mul_tt)((T)2, (T)0, a0[i], a1[i]);",
     [lambda: A.test_integer_roots_are_exact(F64)]),
    ("fma_error_sign",
     "T g = (b.z0 - z0) + b.z1;",
     "T g = (z0 - b.z0) + b.z1;",
     [lambda: A.test_fma_error_is_rounded_exactly(F64)]),
    ("fma_dropped_addend_low_part",
     "if (wt) t = t + w1;",
     "if (wt) t = t;",
     [lambda: A.test_fma_bound("ttt", F64)]),
]

# helper injected for the node-error mutant: ATF1 without err(x0 + y0)
PLAINISH = """
static PAIR NM(plainish_add)(T x0, T x1, T y0, T y1)
{
    PAIR z;
    z.z0 = x0 + y0;
    z.z1 = x1 + y1;
    return z;
}
"""


def build_mutant(tmp_path, original, planted):
    body = open(os.path.join(SRC, "tf_oracle_t.h")).read()
    top = open(os.path.join(SRC, "tf_oracle.c")).read()
    if original in body:
        assert body.count(original) == 1 or original == planted, "mutant anchor not unique"
        body = body.replace(original, planted, 1)
    else:
        assert top.count(original) == 1, "mutant anchor not found or not unique"
        top = top.replace(original, planted)
    if "plainish_add" in planted:
        anchor = "#define TF_TILE 256"
        body = body.replace(anchor, PLAINISH + anchor)
    d = tmp_path / "mut"
    d.mkdir()
    (d / "tf_oracle_t.h").write_text(body)
    (d / "tf_oracle.c").write_text(top)
    so = d / "libmut.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(so), str(d / "tf_oracle.c"), "-lm"], check=True)
    return str(so)


@pytest.mark.parametrize("name,original,planted,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, original, planted, pins):
    so = build_mutant(tmp_path, original, planted)
    caught = 0
    with oracle.use_library(so):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught += 1
    assert caught >= 1, "planted mistake %s passed every pin" % name


def test_unmutated_copy_passes(tmp_path):
    """Control: the same machinery with no edit passes the same pins."""
    so = build_mutant(tmp_path, "#define TF_TILE 256", "#define TF_TILE 256")
    with oracle.use_library(so):
        for _, _, _, pins in MUTANTS:
            for pin in pins:
                pin()
