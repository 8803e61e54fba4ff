"""Sensitivity of the oracle pins: plant a plausible mistake in a copy of
the oracle's C source (a dropped term, a wrong sign or index, a swapped
operand, a wrong tie rule), build it, and check that at least one pin in
test_oracle_pins fails.  CPU only; the planted copies live in a temporary
directory and never replace the real oracle."""
import os
import subprocess
import sys

import pytest

import oracle as O
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "tcdtw_oracle.c")

MUTANTS = [
    ("dtw: diagonal predecessor dropped",
     "if (i > 0 && j > 0) best = dmin(best, prev[j - 1]);", ";"),
    ("dtw: band test of the left predecessor off by one",
     "if (j > 0 && i - (j - 1) <= weff) best = dmin(best, cur[j - 1]);",
     "if (j > 0 && i - (j - 1) < weff) best = dmin(best, cur[j - 1]);"),
    ("point cost: absolute instead of squared difference",
     "s += d * d;", "s += fabs(d);"),
    ("dtw: row window one short", "jhi = imin(n - 1, i + weff);\n        double rowmin",
     "jhi = imin(n - 1, i + weff - 1);\n        double rowmin"),
    ("envelope: window one short", "ihi = imin(m - 1, j + weff);\n        for (int p = 0; p < D; ++p) {\n            double u",
     "ihi = imin(m - 1, j + weff - 1);\n        for (int p = 0; p < D; ++p) {\n            double u"),
    ("lb_mv: upper excess measured from the lower envelope",
     "if (x > u) lb += (x - u) * (x - u);", "if (x > u) lb += (x - l) * (x - l);"),
    ("lb_ad: max instead of min over the window",
     "best = dmin(best, point_cost(q + (size_t)i * D, c + (size_t)j * D, D));",
     "best = i == ilo ? point_cost(q + (size_t)i * D, c + (size_t)j * D, D) : dmax(best, point_cost(q + (size_t)i * D, c + (size_t)j * D, D));"),
    ("lb_ti: second branch of Eq. 7 with the wrong sign",
     "lo = dmax(Lp[j] - delta[i], delta[i] - Up[j]);", "lo = dmax(Lp[j] - delta[i], Up[j] - delta[i]);"),
    ("lb_ti: second branch of Eq. 7 dropped",
     "lo = dmax(Lp[j] - delta[i], delta[i] - Up[j]);", "lo = Lp[j] - delta[i];"),
    ("lb_ti: Eq. 8 subtracts the step",
     "hi = Up[j] + delta[i];", "hi = Up[j] - delta[i];"),
    ("lb_ti: top cell uses the previous candidate step",
     "lo = dmax(Lc[j - 1] - gamma[j], gamma[j] - Uc[j - 1]);",
     "lo = dmax(Lc[j - 1] - gamma[j - 1], gamma[j - 1] - Uc[j - 1]);"),
    ("lb_ti: query step indexed one row late",
     "delta[i] = point_dist(q + (size_t)(i - 1) * D, q + (size_t)i * D, D);",
     "delta[i] = i + 1 < m ? point_dist(q + (size_t)i * D, q + (size_t)(i + 1) * D, D) : 0.0;"),
    ("lb_ti: periodic rows not exact",
     "int exact_row = (i == 0) || (P > 0 && i % P == 0);", "int exact_row = (i == 0);"),
    ("lb_ti: column minimum without the clamp at zero",
     "colmin[j] = dmin(colmin[j], dmax(0.0, lo));", "colmin[j] = dmin(colmin[j], fabs(lo));"),
    ("lb_pc: the first cells merged instead of the last",
     "int b = rank < K - 1 ? rank : K - 1;", "int b = (M - 1 - rank) < K - 1 ? (M - 1 - rank) : K - 1;"),
    ("lb_pc: dimension 0 least significant in the cell key",
     "key = key * (uint64_t)Lv + (uint64_t)dgt;",
     "{ uint64_t pp = 1; for (int t = 0; t < p; ++t) pp *= (uint64_t)Lv; key += pp * (uint64_t)dgt; }"),
    ("lb_pc: Lv-1 segments per dimension",
     "float l = (b - a) / (float)Lv;", "float l = (b - a) / (float)(Lv > 1 ? Lv - 1 : 1);"),
    ("lb_pc: window of the group ends at its first position",
     "ihi = imin(m - 1, jlast + weff);", "ihi = imin(m - 1, jfirst + weff);"),
    ("lb_pc: largest instead of smallest box distance",
     "best = dmin(best, s);", "best = b == 0 ? s : dmax(best, s);"),
    ("knn: ties to the highest index", "if (d < best) { best = d; arg = k; }",
     "if (d <= best) { best = d; arg = k; }"),
    ("path gradient: factor 2 dropped", "gq[(size_t)i * D + p] += gbar * 2.0 * d;",
     "gq[(size_t)i * D + p] += gbar * d;"),
    ("path gradient: candidate sign flipped", "gc[(size_t)j * D + p] -= gbar * 2.0 * d;",
     "gc[(size_t)j * D + p] += gbar * 2.0 * d;"),
    ("path gradient: left step taken for up",
     "if (i > 0 && j - (i - 1) <= weff && CELL(i - 1, j) < bv) { bi = i - 1; bj = j; bv = CELL(i - 1, j); }",
     "if (i > 0 && j - (i - 1) <= weff && CELL(i - 1, j) < bv) { bi = i; bj = j - 1; bv = CELL(i - 1, j); }"),
]

PINS = [
    P.test_dtw_brute_force_small, P.test_dtw_golden_hand_example, P.test_dtw_closed_forms_and_symmetry,
    P.test_dtw_early_abandon_equivalence, P.test_lb_mv_golden, P.test_lb_mv_univariate_is_lb_keogh,
    P.test_lb_ti_golden, lambda: P.test_bounds_below_dtw_and_lb_ad(0), P.test_ti_cells_bracket_true_distance,
    P.test_lb_ti_special_cases, P.test_lb_pc_golden, P.test_lb_pc_special_cases, P.test_pc_boxes_cover_window_points,
    P.test_knn_exhaustive_matches_brute_force, lambda: P.test_cascade_equals_exhaustive(6),
    P.test_path_gradient_invariants,
]


def run_pins(lib_path):
    """Run every pin against the library at lib_path; exit 0 if all pass."""
    O._lib = None
    O.lib(lib_path)
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, OverflowError):
            sys.exit(1)
    sys.exit(0)


def _killed(lib_path):
    """True if some pin fails (or the planted copy crashes) -- in a child process."""
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_mutants as T; T.run_pins(%r)"
            % (here, os.path.dirname(here), lib_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300)
    return r.returncode != 0


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must be unique: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-I", os.path.dirname(SRC), "-o", str(so), str(mut), "-lm"], check=True)
    assert _killed(str(so)), "no pin caught: " + name


def test_unmodified_copy_passes_every_pin(tmp_path):
    """Control: the same harness on an unmodified copy reports no failure."""
    so = tmp_path / "libcontrol.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-I", os.path.dirname(SRC), "-o", str(so), SRC, "-lm"], check=True)
    assert not _killed(str(so))
