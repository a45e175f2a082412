"""The pins of the memoryless mode, the difference-frame method, the accumulated frame and the
events/(pixel s) statistic bite: a one-token mistake planted in a copy of the oracle (on the CPU)
fails at least one of them."""
import subprocess

import pytest

import oracle.oracle as om
import golden_io
import test_oracle_golden as tg
import test_oracle_next as tn

MUTANTS = {
    "memoryless_non_strict_positive": ("if (D > cp) pol = 1;", "if (D >= cp) pol = 1;"),
    "memoryless_non_strict_negative": ("else if (D < -cn) pol = -1;", "else if (D <= -cn) pol = -1;"),
    "memoryless_time_at_subframe_start": ("const float phi = (float)(k + 1) / (float)S;",
                                          "const float phi = (float)k / (float)S;"),
    "memoryless_difference_to_interval_start": ("const float D = V[k + 1] - V[k];",
                                                "const float D = V[k + 1] - V[0];"),
    "difference_order_reversed": ("D1[i] = s->lut[s->prev[i]] - s->lut[s->prev2[i]];",
                                  "D1[i] = s->lut[s->prev2[i]] - s->lut[s->prev[i]];"),
    "difference_flow_sign": ("bil(D1, W, H, (float)x - tau * u", "bil(D1, W, H, (float)x + tau * u"),
    "difference_flow_components_swapped": (
        "const float u = flow[2 * p], v = flow[2 * p + 1];\n                    const float tau",
        "const float v = flow[2 * p], u = flow[2 * p + 1];\n                    const float tau"),
    "difference_state_not_rolled": ("        memcpy(s->prev2, s->prev, n);\n        memcpy",
                                     "        memcpy"),
    "difference_endpoint_is_first_frame": ("Dk = D2[p];", "Dk = D1[p];"),
    "difference_blend_weights_swapped": ("Dk = om * a + tau * b;", "Dk = tau * a + om * b;"),
    "accumulate_window_end_inclusive": ("if (t < t_begin || t >= t_end) continue;",
                                        "if (t < t_begin || t > t_end) continue;"),
    "accumulate_planes_swapped": ("counts[(pos ? 0 : 1) * plane", "counts[(pos ? 1 : 0) * plane"),
    "accumulate_ignores_epoch": ("const int64_t t = epoch + (int64_t)(k >> 25);",
                                 "const int64_t t = (int64_t)(k >> 25);"),
    "rate_sample_deviation": ("const double var = m2 - m1 * m1;",
                              "const double var = (m2 - m1 * m1) * (double)plane / (double)(plane - 1);"),
    "rate_counts_one_polarity": ("const uint64_t c = (uint64_t)counts[p] + (uint64_t)counts[plane + p];",
                                 "const uint64_t c = (uint64_t)counts[p];"),
    "rate_mean_not_per_second": ("*mean = m1 / seconds;", "*mean = m1;"),
}


def _battery(stop_at_first=False):
    checks = []
    for path in golden_io.next_fixtures():
        checks.append(lambda p=path: tg.test_oracle_matches_hand_worked_fixture(None, p))
    checks.append(lambda: tn.test_memoryless_brute_force_8x8(None, "dense", 11))
    checks.append(lambda: tn.test_memoryless_brute_force_8x8(None, "difference", 11))
    checks.append(lambda: tn.test_memoryless_brute_force_8x8(None, "basic", 1))
    for m in (om.BASIC, om.DIFFERENCE):
        checks.append(lambda m=m: tn.test_memoryless_at_most_one_event_per_subframe_on_the_grid(None, m))
        checks.append(lambda m=m: tn.test_memoryless_static_and_constant_inputs_emit_nothing(None, m))
    checks.append(lambda: tn.test_memoryless_dense_with_one_subinterval_is_basic(None))
    checks.append(lambda: tn.test_memoryless_and_reference_agree_below_two_thresholds(None))
    checks.append(lambda: tn.test_memoryless_time_reversal_flips_polarity(None))
    for args in [(True, 2, 2), (False, 4, 4), (True, 3, 6)]:
        checks.append(lambda a=args: tn.test_difference_translating_edge_closed_form(None, *a))
    checks.append(lambda: tn.test_difference_vertical_motion_uses_the_y_component(None))
    checks.append(lambda: tn.test_difference_first_interval_and_restart(None))
    checks.append(lambda: tn.test_accumulate_hand_example(None))
    checks.append(lambda: tn.test_accumulate_matches_loop_and_windows_partition(None))
    checks.append(lambda: tn.test_event_rate_hand_example(None))
    checks.append(lambda: tn.test_event_rate_is_the_population_statistic(None))
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, RuntimeError, ValueError, KeyError):
            failed += 1
            if stop_at_first:
                break
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(tmp_path, monkeypatch, name):
    src = open(om.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", *om.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    monkeypatch.setattr(om, "_lib", om.load_variant(str(lib)))
    assert _battery(stop_at_first=True) > 0, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_the_battery(oracle_mod):
    assert _battery() == 0
