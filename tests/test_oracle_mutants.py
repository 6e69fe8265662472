"""Planted-mistake check of the oracle's pins (CPU only).

Each mutant is a copy of the oracle's C source with one plausible mistake
(a dropped term, a wrong sign, index or operand).  It is compiled into a
temporary library, swapped in, and the pin tests are re-run against it: at
least one of them must fail.  The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

import oracle
import test_oracle_hilbert as H
import test_oracle_update as U
import test_oracle_views as V

SRC = os.path.join(os.path.dirname(oracle.__file__), "dvl_oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("hilbert_invert_wrong_axis", "X[0] ^= P;                        /* invert */", "X[i] ^= P;"),
    ("hilbert_gray_fix_wrong_axis", "if (X[n - 1] & Q) t ^= Q - 1;", "if (X[0] & Q) t ^= Q - 1;"),
    ("hilbert_no_exchange", "X[i] ^= t;\n            }", "(void)t;\n            }"),
    ("hilbert_bit_order", "h = (h << 1) | ((X[i] >> j) & 1u);", "h = (h << 1) | ((X[2 - i] >> j) & 1u);"),
    ("centroid_offset_dropped", "((uint32_t)1 << level[h]) >> 1", "((uint32_t)1 << level[h])"),
    ("grid_bits_off_by_one", "while (((int64_t)1 << b) < extent) ++b;", "while (((int64_t)1 << b) <= extent) ++b;"),
    ("sort_ties_reversed", "if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;",
     "if (p->idx != q->idx) return p->idx < q->idx ? 1 : -1;"),
    ("quantiser_sign", "*b = (float)(-(double)lo * (double)sf);", "*b = (float)((double)lo * (double)sf);"),
    ("quantiser_no_clamp", "if (fl > (double)(n_tf - 1)) return n_tf - 1;", ""),
    ("variation_sum", "    return hi - lo;\n}\n\n/* Eq. 3", "    return hi + lo;\n}\n\n/* Eq. 3"),
    ("vmax_range_off_by_one", "for (int32_t a = i; a <= j; ++a) {", "for (int32_t a = i; a < j; ++a) {"),
    ("vmax_no_fallback", "vmax = ora_vmax_tf(ORA_VMAX_TF_BOUND, M, n_tf, alpha, im, jm);", "vmax = 0.0;"),
    ("level_scale_dropped", "(p->level_scale == 3 ? 3 : 1) * lev", "(p->level_scale == 3 ? 3 : 1) * 0"),
    ("exponent_dropped", "double f = pow(r * scale, p->exponent);", "double f = r * scale;"),
    ("min_importance_dropped", "return f > p->min_importance ? f : p->min_importance;", "return f;"),
    ("ratio_inverted", "double r = vmax > 0.0 ? v / vmax : 0.0;", "double r = v > 0.0 ? vmax / v : 0.0;"),
    ("neumaier_sign", "if (fabs(sum) >= fabs(f[h])) comp += (sum - t) + f[h];",
     "if (fabs(sum) >= fabs(f[h])) comp += (sum - t) - f[h];"),
    ("prefix_inclusive_for_xf1", "double xf1 = (E[h] * (double)W) / F;", "double xf1 = (E[h + 1] * (double)W) / F;"),
    ("projection_floor_for_upper", "double hi_b = ceil(xf2) - 1.0;", "double hi_b = floor(xf2);"),
    ("min_compare_flipped", "if (x < out->vmin[o]) out->vmin[o] = x;", "if (x > out->vmin[o]) out->vmin[o] = x;"),
    ("mean_divides_by_count_plus_one", "out->sum[o] / (double)out->count[k];", "out->sum[o] / (double)(out->count[k] + 1);"),
    ("height_from_max_not_mean", "ora_tf_index((float)out->mean[o], s[m], b[m], n_tf);",
     "ora_tf_index(out->vmax[o], s[m], b[m], n_tf);"),
    ("degenerate_not_handled", "for (int64_t h = 0; h < n; ++h) f[h] = 1.0;", ";"),
    ("histogram_last_cell_dropped", "for (int64_t h = first[bin]; h <= (int64_t)last[bin]; ++h) {",
     "for (int64_t h = first[bin]; h < (int64_t)last[bin]; ++h) {"),
    ("histogram_window_reversed", "ora_quantiser(n_buckets, lo, hi, &s, &b);", "ora_quantiser(n_buckets, hi, lo, &s, &b);"),
    ("raster_round_not_floor", "int32_t r = (int32_t)floorf(t);", "int32_t r = (int32_t)floorf(t + 0.5f);"),
    ("raster_next_height_ignored", "int32_t r1 = b + 1 < n_bins ? ora_row(y[b + 1], n_rows) : r0;",
     "int32_t r1 = r0;"),
    ("raster_bars_from_one", "            lo = 0;\n            hi = r0;", "            lo = 1;\n            hi = r0;"),
]


def _pins():
    """The pin tests, as zero-argument callables."""
    cases = []
    for ex in U._golden():
        cases.append(lambda ex=ex: U.test_hand_examples(oracle, ex))
    cases += [
        lambda: H.test_bijection_and_unit_steps(oracle, 3),
        lambda: H.test_aligned_subcubes_are_contiguous(oracle, 4),
        lambda: H.test_representative_point_does_not_change_order(oracle, 0),
        lambda: H.test_amr_cells_cover_contiguous_ranges(oracle, 0),
        lambda: H.test_sort_matches_stable_library_sort(oracle),
        lambda: H.test_grid_bits(oracle, ([56], [0], [0], [3]), 6),
        lambda: H.test_grid_bits(oracle, ([57], [0], [0], [0]), 6),
        lambda: U.test_uniform_variation_single_level_is_linear(oracle),
        lambda: U.test_uniform_variation_amr_widths(oracle, 2.0, 2),
        lambda: U.test_single_field_has_no_variation(oracle),
        lambda: U.test_zero_total_width_falls_back_to_linear(oracle),
        lambda: U.test_prefix_matches_correctly_rounded_sums(oracle),
        lambda: U.test_quantiser_exact_window(oracle),
        lambda: U.test_quantiser_matches_exact_floor_away_from_edges(oracle),
        lambda: U.test_vmax_range_literal(oracle),
        lambda: U.test_vmax_range_is_not_an_upper_bound(oracle),
        lambda: U.test_structural_invariants(oracle, 12, 257, 2.0, 0.025),
        lambda: V.test_histogram_hand_example(oracle),
        lambda: V.test_histogram_counts_sum_to_bin_sizes_with_straddles(oracle),
        lambda: V.test_histogram_matches_numpy_away_from_bucket_edges(oracle),
        lambda: V.test_histogram_values_outside_the_window_go_to_the_end_buckets(oracle),
        lambda: V.test_raster_constant_line_is_one_row(oracle),
        lambda: V.test_raster_hand_example(oracle),
        lambda: V.test_raster_invariants(oracle, 0),
    ]
    for s in range(24):
        cases.append(lambda s=s: U.test_against_exact_rational_bruteforce(oracle, s))
    return cases


def run_pins_against(so_path: str) -> int:
    """Run the pin battery against the library at ``so_path``; returns the
    index of the first failing pin, or -1 if all pass."""
    oracle.use_library(oracle.bind(so_path))
    for k, pin in enumerate(_pins()):
        try:
            pin()
        except AssertionError:
            return k
        except pytest.skip.Exception:
            continue
        except (ValueError, MemoryError, OverflowError):
            return k
    return -1


def _run_child(so: str):
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_mutants as T; "
            "k = T.run_pins_against(%r); print('first failing pin', k); sys.exit(0 if k < 0 else 3)"
            % (here, os.path.dirname(here), so))
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)


def test_unmodified_oracle_passes_the_battery():
    """Control: the same child-process harness reports success on the real oracle."""
    r = _run_child(oracle.build(force=False))
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, mut, tmp_path):
    import shutil
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation site for {name} not found exactly once"
    d = str(tmp_path)
    with open(os.path.join(d, "dvl_oracle.c"), "w") as fh:
        fh.write(src.replace(orig, mut))
    shutil.copy(os.path.join(os.path.dirname(SRC), "dvl_oracle.h"), d)
    so = os.path.join(d, f"mut_{name}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-w",
                           "-o", so, os.path.join(d, "dvl_oracle.c"), "-lm"])
    r = _run_child(so)
    # exit 3: a pin failed; a crash (negative code) also means the mistake was caught
    assert r.returncode != 0, f"no pin caught the planted mistake {name}: {r.stdout}{r.stderr[-2000:]}"
