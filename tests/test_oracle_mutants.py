"""The pins bite: plausible mistakes planted in copies of the oracle (on the CPU) each fail a pin.

Every mutant below is a one-token slip of the kind the pins are meant to catch: a sign, an index,
a swapped operand, a dropped term, an off-by-one tie or backlog rule.  Each mutant is compiled
from a modified copy of oracle/oracle.c into a temporary directory; the pin battery is then run
against it and at least one pin must fail.
"""
import subprocess

import pytest

import oracle.oracle as om
import test_oracle_golden as tg
import test_oracle_pins as tp
import golden_io

MUTANTS = {
    "flow_sign": ("(float)x - tau * u", "(float)x + tau * u"),
    "flow_components_swapped": ("const float u = flow[2 * p], v = flow[2 * p + 1];\n                for",
                                "const float v = flow[2 * p], u = flow[2 * p + 1];\n                for"),
    "bilinear_y1_index": ("int y1 = y0 + 1 < H ? y0 + 1 : H - 1;", "int y1 = y0;"),
    "bilinear_dropped_bottom_row": ("return gy * top + fy * bot;", "return gy * top + fy * top;"),
    "bilinear_x_weights_swapped": ("float top = gx * L[(size_t)y0 * W + x0] + fx * L[(size_t)y0 * W + x1];",
                                   "float top = fx * L[(size_t)y0 * W + x0] + gx * L[(size_t)y0 * W + x1];"),
    "blend_weights_swapped": ("V[k] = om * a + tau * b;", "V[k] = tau * a + om * b;"),
    "strict_positive_threshold": ("if (B - R >= cp)", "if (B - R > cp)"),
    "strict_negative_threshold": ("else if (B - R <= -cn)", "else if (B - R < -cn)"),
    "no_backlog_rule": ("const int backlog = pol > 0 ? (A >= Rn) : (A <= Rn);",
                        "const int backlog = 0;"),
    "time_drops_theta": ("const float phi = ((float)k + theta) / (float)S;",
                         "const float phi = (float)k / (float)S;"),
    "time_uses_next_subinterval": ("const float phi = ((float)k + theta) / (float)S;",
                                   "const float phi = ((float)k + 1.0f - theta) / (float)S;"),
    "polarity_bit_inverted": ("(uint64_t)(pol > 0 ? 1 : 0)", "(uint64_t)(pol > 0 ? 0 : 1)"),
    "sparse_selects_on_level": ("if (!(fabsf(A1 - A0) >= s->m)) continue;",
                                "if (!(fabsf(A1) >= s->m)) continue;"),
    "log_of_wrong_scale": ("(double)v / 255.0", "(double)v / 256.0"),
    "clamp_lower_bound_off": ("sy = fminf(fmaxf(sy, 0.0f), (float)(H - 1));",
                              "sy = fminf(fmaxf(sy, 0.5f), (float)(H - 1));"),
    "keeps_stale_reference": ("            s->lref[p] = R;\n", "            (void)R;\n"),
}


def _battery(stop_at_first=False):
    """Runs a fast subset of the pins; returns how many of them failed."""
    checks = []
    for path in golden_io.all_fixtures():
        checks.append(lambda p=path: tg.test_oracle_matches_hand_worked_fixture(None, p))
    checks.append(lambda: tp.test_p1_table_is_correctly_rounded_log(None))
    checks.append(lambda: tp.test_p3_basic_counts_and_times_closed_form(None, 0.2))
    checks.append(lambda: tp.test_p5_p12_zero_flow_is_linear_in_time(None))
    for m in (0, 1, 2):
        checks.append(lambda m=m: tp.test_p9_reference_bookkeeping(None, m))
    for args in [(0, 1, 11), (1, 2, 2), (0, 3, 3)]:
        checks.append(lambda a=args: tp.test_p7_translating_edge(None, *a, 1))
    checks.append(lambda: tp.test_p6_sparse_is_dense_restricted_to_selection(None))
    for m in ("dense", "sparse"):
        checks.append(lambda m=m: tp.test_p10_brute_force_8x8(None, m, 11))
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, RuntimeError, ValueError):
            failed += 1
            if stop_at_first:
                break
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(tmp_path, monkeypatch, name):
    src = open(om.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", *om.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    monkeypatch.setattr(om, "_lib", om.load_variant(str(lib)))
    assert _battery(stop_at_first=True) > 0, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_the_battery(oracle_mod):
    assert _battery() == 0
