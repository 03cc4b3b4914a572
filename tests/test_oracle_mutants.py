"""Sensitivity of the oracle's pins: plant plausible mistakes in a copy of the
oracle's C source (a dropped term, a wrong sign, a flipped comparison, a
transposed operand), build it on the CPU, and check that the pins of
test_oracle.py reject every one of them."""
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle as T
from tests import test_oracle_metrics as TM
from tests import test_oracle_regions as TR
from tests import test_oracle_danielsson as TD

MUTANTS = [
    ("tie rule reversed", "l_wins_tie = fl < fk;", "l_wins_tie = fl > fk;"),
    ("floor instead of first-win position", "return floor_div(num, den) + 1;",
     "return floor_div(num, den);"),
    ("intersection numerator sign", "- (int64_t)k * k + (int64_t)l * l",
     "+ (int64_t)k * k - (int64_t)l * l"),
    ("intersection numerator drops Dv[k]", "Dv[l] - Dv[k] - (int64_t)k * k",
     "Dv[l] - (int64_t)k * k"),
    ("intersection denominator not doubled", "int64_t den = 2 * (int64_t)(l - k);",
     "int64_t den = (int64_t)(l - k);"),
    ("upward sweep keeps the lower site on ties", "c->Dv[o] > db * db", "c->Dv[o] >= db * db"),
    ("odd step drops the +1", "c->Dv[o - W] + 2 * x + 1", "c->Dv[o - W] + 2 * x"),
    ("pop only on strict win", "if (s <= js[n - 1])", "if (s < js[n - 1])"),
    ("last pixel start dropped", "} else if (s <= W - 1) {", "} else if (s < W - 1) {"),
    ("brute force keeps the last tie", "if (best < 0 || d < best) {\n            best = d;\n            bestf = (int64_t)s[q].r * W + s[q].c;",
     "if (best < 0 || d <= best) {\n            best = d;\n            bestf = (int64_t)s[q].r * W + s[q].c;"),
    ("brute force transposes the site index", "bestf = (int64_t)s[q].r * W + s[q].c;\n        }\n    }\n    *D",
     "bestf = (int64_t)s[q].c * W + s[q].r;\n        }\n    }\n    *D"),
    ("fill uses j + k", "D[j] = (int32_t)(dv[k] + (int64_t)(j - k) * (j - k));",
     "D[j] = (int32_t)(dv[k] + (int64_t)(j - k) * (j + k));"),
    ("fill feature uses the pixel column", "F[j] = r[k] * W + k;", "F[j] = r[k] * W + j;"),
    ("floor division rounds towards zero", "if ((a % b != 0) && (a < 0))", "if ((a % b != 0) && (a > 0))"),
    ("polarity inverted", "return polarity ? !object : object;", "return polarity ? object : !object;"),
    ("contour test inverted for the upper neighbour",
     "if (r > 0 && !is_site(mask[(int64_t)(r - 1) * pitch + c], polarity)) keep = 1;",
     "if (r > 0 && is_site(mask[(int64_t)(r - 1) * pitch + c], polarity)) keep = 1;"),
    ("downward sweep carries the previous row, not the site row",
     "c->R[o] = c->R[o - W];\n", "c->R[o] = i - 1;\n"),
    ("sqrt in single precision", "(float)sqrt((double)D[q])", "sqrtf((float)D[q])"),
    ("basic row pass ignores the feature on ties",
     "if (best < 0 || d < best || (d == best && f < bestf)) {",
     "if (best < 0 || d < best) {"),
    ("city-block scans skip the upward column scan",
     "for (int32_t i = H - 2; i >= 0; --i) { /* upward */",
     "for (int32_t i = H - 2; i >= H; --i) { /* upward */"),
    ("city-block scans step by 2", "if (*c > up + 1) *c = up + 1;", "if (*c > up + 2) *c = up + 2;"),
    ("city-block scans skip the backward row scan",
     "for (int32_t j = W - 2; j >= 0; --j) /* backward */",
     "for (int32_t j = W - 2; j >= W; --j) /* backward */"),
    ("chessboard takes the smaller offset", ": (metric == 2) ? hi", ": (metric == 2) ? lo"),
    ("city-block squares the offsets", "(metric == 1) ? di + dj", "(metric == 1) ? di * di + dj * dj"),
    ("chamfer swaps the diagonal and straight costs", ": 4 * lo + 3 * (hi - lo);",
     ": 3 * lo + 4 * (hi - lo);"),
    ("chamfer forward scan skips the upper-right neighbour",
     "if (i > 0 && j + 1 < W) LOWER(i, j, AT(i - 1, j + 1) + 4);",
     "if (i > 0 && j + 1 < 0) LOWER(i, j, AT(i - 1, j + 1) + 4);"),
    ("chamfer backward diagonal step costs 3", "LOWER(i, j, AT(i + 1, j + 1) + 4);",
     "LOWER(i, j, AT(i + 1, j + 1) + 3);"),
    ("chamfer backward scan takes the rows top-down",
     "for (int32_t i = H - 1; i >= 0; --i) { /* backward: bottom-right to top-left */",
     "for (int32_t i = 0; i < H; ++i) { /* backward: bottom-right to top-left */"),
    ("regions drop the diagonal neighbours of the 8-neighbourhood",
     "if (connectivity == 4 && di != 0 && dj != 0) continue;", "if (di != 0 && dj != 0) continue;"),
    ("regions keep the diagonal neighbours in the 4-neighbourhood",
     "if (connectivity == 4 && di != 0 && dj != 0) continue;", "if (connectivity == 5) continue;"),
    ("regions label a component by the site it was reached from",
     "comp[nb] = (int32_t)start;", "comp[nb] = (int32_t)cur;"),
    ("regions label the pixel's own component, not its nearest site's",
     "labels[q] = F[q] < 0 ? -1 : comp[F[q]];", "labels[q] = F[q] < 0 ? -1 : (comp[q] >= 0 ? comp[q] : F[q]);"),
    ("regions search only upwards", "for (int32_t di = -1; di <= 1; ++di) {",
     "for (int32_t di = -1; di <= 0; ++di) {"),
    ("metric definition keeps the last of equally near sites",
     "if (best >= 0 && d >= best)", "if (best >= 0 && d > best)"),
    ("sampled metric definition swaps the pixel's row and column",
     "(int32_t)(o / b->W), (int32_t)(o % b->W),", "(int32_t)(o % b->W), (int32_t)(o / b->W),"),
    ("danielsson takes offers at equal distance", "    if (d[to] > nd) {", "    if (d[to] >= nd) {"),
    ("danielsson vertical step adds to dx",
     "for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i - 1, j), 1, 0);",
     "for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i - 1, j), 0, 1);"),
    ("danielsson first scan starts at the third row", "    for (int32_t i = 1; i < H; ++i) { /* first scan, downwards */",
     "    for (int32_t i = 2; i < H; ++i) { /* first scan, downwards */"),
    ("danielsson first scan sweeps the row back left to right",
     "        for (int32_t j = W - 2; j >= 0; --j) {\n            dan_offer(d, y, x, P(i, j), P(i - 1, j + 1), 1, 1);",
     "        for (int32_t j = 0; j <= W - 2; ++j) {\n            dan_offer(d, y, x, P(i, j), P(i - 1, j + 1), 1, 1);"),
    ("danielsson first scan drops the top-left offer",
     "            dan_offer(d, y, x, P(i, j), P(i, j - 1), 0, 1);\n            dan_offer(d, y, x, P(i, j), P(i - 1, j - 1), 1, 1);",
     "            dan_offer(d, y, x, P(i, j), P(i, j - 1), 0, 1);"),
    ("danielsson second scan takes the vertical step from above",
     "for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i + 1, j), 1, 0);",
     "for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i > 0 ? i - 1 : i + 1, j), 1, 0);"),
]


def _pins():
    yield T.test_example_mask_matches_initialisation, ()
    yield T.test_downward_sweep_matches_fig_eedt2, ()
    yield T.test_vertical_pass_matches_fig_eedt_b, ()
    for fn in ("brute", "brute_contour", "separable", "basic_rows"):
        yield T.test_final_matches_fig_eedt_c, (fn,)
    for fn in ("brute", "separable", "basic_rows"):
        yield T.test_single_site_matches_fig_euclidean, (fn,)
    yield T.test_propagation_row1_parabolas_and_kstar, ()
    yield T.test_envelope_trace_row1, ()
    yield T.test_all_oracle_forms_agree_on_small_masks, ()
    yield T.test_tiny_brute_force_by_enumeration, ()
    yield T.test_no_site_gives_sentinel, ()
    yield T.test_all_sites_zero_and_own_index, ()
    yield T.test_corner_site_closed_form, ()
    yield T.test_single_site_anywhere_separable, ()
    yield T.test_sites_in_one_row_reduce_to_1d, ()
    yield T.test_invariants_on_generated_masks, ()
    yield T.test_sqrt_epilogue, ()
    for pol in (0, 1):
        yield TM.test_cityblock_definition_matches_figure, (pol,)
        yield TM.test_chessboard_definition_matches_figure, (pol,)
    yield TM.test_cityblock_scans_vertical_stage_matches_figure, ()
    yield TM.test_cityblock_final_matches_figure_but_the_erratum, ()
    for seed in range(4):
        yield TM.test_cityblock_scans_equal_definition, (seed,)
    for metric in (1, 2):
        yield TM.test_metric_closed_forms_and_invariants, (metric,)
    for pol in (0, 1):
        yield TM.test_chamfer_definition_matches_figure, (pol,)
    yield TM.test_chamfer_forward_scan_matches_figure_but_the_erratum, ()
    yield TM.test_chamfer_final_matches_figure, ()
    for seed in range(4):
        yield TM.test_chamfer_scans_equal_definition, (seed,)
    yield TM.test_chamfer_bounds_against_euclidean, ()
    for metric in (1, 2, 3):
        yield TM.test_sampled_definition_equals_full_definition, (metric,)
    yield TR.test_diagonal_pair_is_one_object_in_8_and_two_in_4, ()
    yield TR.test_checkerboards, ()
    yield TR.test_full_empty_and_isolated_points, ()
    yield TR.test_paper_example_components, ()
    for seed in range(4):
        yield TR.test_regions_against_min_propagation, (seed,)
    yield TD.test_first_scan_matches_figure, ()
    yield TD.test_first_scan_top_left_offer_decides_a_cell, ()
    yield TD.test_final_matches_figure_but_the_erratum, ()
    for seed in range(3):
        yield TD.test_never_below_exact_and_consistent, (seed,)
    yield TD.test_single_sites_exact_and_one_row_propagates_nothing, ()
    yield TD.test_disconnected_region_is_missed, ()


def _failures(lib):
    failed = []
    with oracle.using(lib):
        for fn, args in _pins():
            try:
                fn(*args)
            except Exception:  # an assertion or a value error both reject
                failed.append(fn.__name__)
    return failed


def test_unmutated_source_passes_every_pin(tmp_path):
    so = tmp_path / "liboracle_clean.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread",
                           oracle.SRC, "-o", str(so), "-lm"])
    assert _failures(oracle.bind(str(so))) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(name, old, new, tmp_path):
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread",
                           str(mut), "-o", str(so), "-lm"])
    failed = _failures(oracle.bind(str(so)))
    assert failed, f"no pin rejects the planted mistake: {name}"
