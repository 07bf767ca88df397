"""The pins catch plausible mistakes: each mutant copy of the oracle must fail one.

Each mutation below is a one-line change to a temporary copy of ``oracle/sco.c``
(the committed oracle is never touched): a flipped tie-break, a dropped term, a
wrong index.  The copy is compiled into a temporary library and the whole pin
suite runs against it in a child process; the test passes when some pin fails.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "insert_average_rounds_down": (
        "o[(size_t)p * C + c] = (uint8_t)((row[(size_t)x * C + c] + row[(size_t)xr * C + c] + 1) >> 1);",
        "o[(size_t)p * C + c] = (uint8_t)((row[(size_t)x * C + c] + row[(size_t)xr * C + c]) >> 1);"),
    "insert_left_neighbour": (
        "int xr = clampi(x + 1, 0, W - 1);",
        "int xr = clampi(x - 1, 0, W - 1);"),
    "origins_off_by_one": (
        "orig[(size_t)j * H + r] = idx[s];",
        "orig[(size_t)j * H + r] = idx[s < w - 1 ? s + 1 : s];"),
    "parent_tie_rightmost": (
        "if (best < 0 || m[(size_t)(i - 1) * W + p] < m[(size_t)(i - 1) * W + best]) best = p;",
        "if (best < 0 || m[(size_t)(i - 1) * W + p] <= m[(size_t)(i - 1) * W + best]) best = p;"),
    "last_row_tie_rightmost": (
        "if (m[(size_t)(H - 1) * W + j] < m[(size_t)(H - 1) * W + jstar]) jstar = j;",
        "if (m[(size_t)(H - 1) * W + j] <= m[(size_t)(H - 1) * W + jstar]) jstar = j;"),
    "energy_drops_y_term": ("s += absi(dx) + absi(dy);", "s += absi(dx);"),
    "energy_abs_of_sum": ("s += absi(dx) + absi(dy);", "s += absi(dx + dy);"),
    "energy_first_channel_only": (
        "for (int c = 0; c < C; ++c) {\n                int dx", "for (int c = 0; c < 1; ++c) {\n                int dx"),
    "energy_one_sided_up": ("int yu = clampi(y - 1, 0, H - 1)", "int yu = clampi(y, 0, H - 1)"),
    "dp_uses_row_above_energy": (
        "m[(size_t)i * W + j] = (int64_t)e[(size_t)i * W + j] +",
        "m[(size_t)i * W + j] = (int64_t)e[(size_t)(i - 1) * W + j] +"),
    "backtrack_reads_wrong_row": (
        "seam[i - 1] = seam[i] + (int)d[(size_t)i * W + seam[i]] - 1;",
        "seam[i - 1] = seam[i] + (int)d[(size_t)(i - 1) * W + seam[i]] - 1;"),
    "removal_deletes_right_neighbour": (
        "for (int x = seam[i]; x < W - 1; ++x)", "for (int x = seam[i] + 1; x < W - 1; ++x)"),
    "carve_energy_computed_once": (
        "if ((rc = sco_energy(img, H, w, C, pitch, e)) != SCO_OK) break;",
        "if (k == 0 && (rc = sco_energy(img, H, w, C, pitch, e)) != SCO_OK) break;"),
    "greedy_start_rightmost": (
        "if (e[(size_t)(H - 1) * W + j] < e[(size_t)(H - 1) * W + start]) start = j;",
        "if (e[(size_t)(H - 1) * W + j] <= e[(size_t)(H - 1) * W + start]) start = j;"),
    "brute_keeps_last_tie": ("if (!c->have || acc < c->best_cost) {", "if (!c->have || acc <= c->best_cost) {"),
    "forward_left_term_wrong_row": (
        "if (p == j - 1) v += pix_diff(img, pitch, C, i - 1, j, i, j - 1);",
        "if (p == j - 1) v += pix_diff(img, pitch, C, i, j, i, j - 1);"),
    "forward_side_terms_swapped": (
        "if (p == j - 1) v += pix_diff(img, pitch, C, i - 1, j, i, j - 1);",
        "if (p == j - 1) v += pix_diff(img, pitch, C, i - 1, j, i, j + 1);"),
    "forward_border_uncharged": (
        "int64_t cu = pix_diff(img, pitch, C, i, clampi(j - 1, 0, W - 1), i, clampi(j + 1, 0, W - 1));",
        "int64_t cu = (j > 0 && j < W - 1) ? pix_diff(img, pitch, C, i, j - 1, i, j + 1) : 0;"),
    "forward_first_row_zero": ("                m[j] = cu;\n", "                m[j] = 0;\n"),
    "forward_last_row_tie_rightmost": ("if (last[j] < last[jstar]) jstar = j;", "if (last[j] <= last[jstar]) jstar = j;"),
    "forward_backtrack_reads_wrong_row": (
        "seam[i - 1] = seam[i] - 1 + (int)d[(size_t)i * W + seam[i]];",
        "seam[i - 1] = seam[i] - 1 + (int)d[(size_t)(i - 1) * W + seam[i]];"),
    "forward_tie_rightmost": ("if (best < 0 || v < bestv) {", "if (best < 0 || v <= bestv) {"),
    "forward_carve_never_removes": (
        "if ((rc = sco_remove_seam(img, H, w, C, pitch, s)) != SCO_OK) break;\n        if (seams_out) memcpy(seams_out + (size_t)k * H, s, sizeof(int32_t) * (size_t)H);\n        if (costs_out) costs_out[k] = cost;\n    }\n    free(s);",
        "if (k < 0 && (rc = sco_remove_seam(img, H, w, C, pitch, s)) != SCO_OK) break;\n        if (seams_out) memcpy(seams_out + (size_t)k * H, s, sizeof(int32_t) * (size_t)H);\n        if (costs_out) costs_out[k] = cost;\n    }\n    free(s);"),
    "mask_bias_added": (
        "if (mask[(size_t)y * mpitch + x]) e[(size_t)y * W + x] -= B;",
        "if (mask[(size_t)y * mpitch + x]) e[(size_t)y * W + x] += B;"),
    "mask_bias_below_bound": (
        "return (int32_t)h * 510 * C + 1;", "return (int32_t)255 * C;"),
    "mask_not_shifted": (
        "if ((rc = sco_remove_seam(M, h, w, 1, mp, s)) != SCO_OK) break;", ""),
    "object_direction_inverted": (
        "return (c1 - c0 + 1) <= (r1 - r0 + 1) ? SCO_OBJ_VERTICAL : SCO_OBJ_HORIZONTAL;",
        "return (c1 - c0 + 1) >= (r1 - r0 + 1) ? SCO_OBJ_VERTICAL : SCO_OBJ_HORIZONTAL;"),
    "object_loop_stops_early": (
        "while (rc == SCO_OK && w > 1 && count_mask(M, h, w, mp) > 0)",
        "while (rc == SCO_OK && w > 1 && count_mask(M, h, w, mp) > 1)"),
    "object_restore_skipped_for_one_seam": (
        "if (rc == SCO_OK && restore && k > 0) {", "if (rc == SCO_OK && restore && k > 1) {"),
    "transpose_swaps_nothing": (
        "dst[(size_t)x * dpitch + (size_t)y * C + c] = src[(size_t)y * spitch + (size_t)x * C + c];",
        "dst[(size_t)x * dpitch + (size_t)y * C + c] = src[(size_t)(y % W) * spitch + (size_t)(x % H) * C + c];"),
}

CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, pins
o = oracle.Oracle({lib!r})
failed = []
for pin in pins.ALL_PINS:
    try:
        pin(o)
    except (AssertionError, ValueError) as ex:
        failed.append(pin.__name__)
print("FAILED_PINS", failed)
sys.exit(0 if failed else 3)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    with open(os.path.join(ROOT, "oracle", "sco.c")) as f:
        src = f.read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mpath = tmp_path / "sco_mut.c"
    mpath.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmut.so")
    oracle.compile_source(str(mpath), lib)
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, f"mutant {name} survived every pin (rc={r.returncode}):\n{r.stdout}\n{r.stderr}"
