"""The Lucas-Kanade pins bite: a one-token mistake planted in a copy of the oracle's flow
estimator (on the CPU) fails at least one of them.  Mistakes that only shift or rescale both
pyramids alike leave every flow unchanged (the estimate is invariant to them) and are not listed."""
import subprocess

import pytest

import oracle.oracle as om
import test_oracle_lk as tl

MUTANTS = {
    "residual_sign": ("const float d = i0 - bil_tap(&J[l], 0, u);",
                      "const float d = bil_tap(&J[l], 0, u) - i0;"),
    "residual_against_first_frame": ("const float d = i0 - bil_tap(&J[l], 0, u);",
                                     "const float d = i0 - bil_tap(&I[l], 0, u);"),
    "guess_not_doubled": ("gx = 2.0f * (gx + vx);", "gx = (gx + vx);"),
    "gradient_not_halved": ("return (img_at(im, x + 1, y) - img_at(im, x - 1, y)) * 0.5f;",
                            "return (img_at(im, x + 1, y) - img_at(im, x - 1, y)) * 1.0f;"),
    "cramer_sign": ("const float ex = (Gyy * bx - Gxy * by) / det;",
                    "const float ex = (Gyy * bx + Gxy * by) / det;"),
    "cramer_swapped_diagonal": ("const float ey = (Gxx * by - Gxy * bx) / det;",
                                "const float ey = (Gyy * by - Gxy * bx) / det;"),
    "normal_matrix_window_off_by_one": (
        "for (int dy = -r; dy <= r; ++dy) {\n            for (int dx = -r; dx <= r; ++dx) {\n"
        "                const or_tap t = tap_at(I[l].W, I[l].H, ux + (float)dx, uy + (float)dy);",
        "for (int dy = -r; dy < r; ++dy) {\n            for (int dx = -r; dx <= r; ++dx) {\n"
        "                const or_tap t = tap_at(I[l].W, I[l].H, ux + (float)dx, uy + (float)dy);"),
    "texture_test_dropped": ("if (!(trace >= P->min_trace * N) || !(det", "if (!(det"),
    "aperture_test_dropped": ("|| !(det >= P->min_ratio * trace * trace)) {", ") {"),
    "level_position_not_scaled": ("const float ux = (float)px * sc, uy = (float)py * sc;",
                                  "const float ux = (float)px, uy = (float)py;"),
    "integration_frames_swapped": ("oracle_lk_flow(s->prev, frame, W, H, &P, pts, np, fl, NULL);",
                                   "oracle_lk_flow(frame, s->prev, W, H, &P, pts, np, fl, NULL);"),
    "integration_wrong_pixels": (
        "if (s->cfg.method != OR_SPARSE || fabsf(s->L1[i] - s->L0[i]) >= s->m)",
        "if (s->cfg.method != OR_SPARSE || fabsf(s->L1[i] - s->L0[i]) < s->m)"),
}


def _battery(stop_at_first=False):
    checks = [
        lambda: tl.test_recovers_subpixel_and_pixel_translations(None, (-1.5, 0.75)),
        lambda: tl.test_recovers_subpixel_and_pixel_translations(None, (6.5, 4.25)),
        lambda: tl.test_large_motion_needs_the_pyramid(None),
        lambda: tl.test_static_scene_has_zero_flow(None),
        lambda: tl.test_textureless_and_edge_windows_are_rejected(None),
        lambda: tl.test_antisymmetry(None),
        lambda: tl.test_matches_independent_float64_implementation(None, 2, 4),
        lambda: tl.test_estimated_flow_drives_the_interpolation(None, om.SPARSE),
        lambda: tl.test_estimated_flow_drives_the_interpolation(None, om.DENSE),
    ]
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
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", *om.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    monkeypatch.setattr(om, "_lib", om.load_variant(str(lib)))
    monkeypatch.setattr(tl, "lk_flow", om.lk_flow)
    assert _battery(stop_at_first=True) > 0, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_the_battery(oracle_mod):
    assert _battery() == 0
