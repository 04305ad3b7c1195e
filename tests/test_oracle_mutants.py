"""Plant plausible mistakes in copies of the oracle and check that the pins catch each.

Each mutant is the oracle's C source with one edit (a dropped term, a wrong
sign, index, rounding, constant or transposed operand).  The pins of
``test_oracle.py`` run against the mutant build; at least one must fail.
"""
import os
import tempfile

import pytest

import oracle
import oracle.oracle as oracle_front
import test_oracle as pins

MUTANTS = {
    "read index off by one": ("acc[t] += x_u8(x, pitch, c, t + s);", "acc[t] += x_u8(x, pitch, c, t + s + 1);"),
    "round down instead of half up": ("floor(delay_samples + 0.5)", "floor(delay_samples)"),
    "dropped reference-frequency term": ("1.0 / (f * f) - 1.0 / (f_high * f_high)", "1.0 / (f * f)"),
    "inverse instead of inverse square": ("1.0 / (f * f) - 1.0 / (f_high * f_high)", "1.0 / f - 1.0 / f_high"),
    "channel frequencies ascending": ("f_high - (double)c * chan_bw", "f_high - (double)(c + 1) * chan_bw"),
    "first channel dropped": ("for (int c = 0; c < n_chan; ++c) {\n        int64_t s", "for (int c = 1; c < n_chan; ++c) {\n        int64_t s"),
    "DM index off by one": ("dm_start + (double)d * dm_step", "dm_start + (double)(d + 1) * dm_step"),
    "time sampling multiplied": ("((dm * ORACLE_KDM) * k) / t_samp", "((dm * ORACLE_KDM) * k) * (1e-4 / t_samp) / t_samp"),
    "constant as printed with Eq. 1 in MHz ms": ("#define ORACLE_KDM 4.148808e3", "#define ORACLE_KDM 4.1488e3"),
    "nibbles swapped": ("return (t & 1) ? (b >> 4) : (b & 15);", "return (t & 1) ? (b & 15) : (b >> 4);"),
    "adjoint reads transposed table": ("int64_t s = shift[(int64_t)d * n_chan + c];\n      const float *yr", "int64_t s = shift[(int64_t)c * n_dm + d];\n      const float *yr"),
    "adjoint delays the wrong way": ("gr[t + s] += (double)yr[t];", "gr[t + (n_samp - n_out - s)] += (double)yr[t];"),
    "f32 forward drops last channel": ("for (int c = 0; c < n_chan; ++c) {\n      const float *row", "for (int c = 0; c < n_chan - 1; ++c) {\n      const float *row"),
    "16-bit bytes swapped": ("return (int64_t)p[0] | ((int64_t)p[1] << 8);", "return (int64_t)p[1] | ((int64_t)p[0] << 8);"),
    "16-bit sample stride of one byte": ("const uint8_t *p = x + (int64_t)c * pitch_bytes + 2 * t;", "const uint8_t *p = x + (int64_t)c * pitch_bytes + t;"),
    "16-bit high byte dropped": ("return (int64_t)p[0] | ((int64_t)p[1] << 8);", "return (int64_t)p[0];"),
    "bin drops its last sample": ("for (int i = 0; i < factor; ++i) {\n        const int64_t t = j * factor + i;", "for (int i = 0; i < factor - 1; ++i) {\n        const int64_t t = j * factor + i;"),
    "bin windows overlap": ("const int64_t t = j * factor + i;", "const int64_t t = j + i;"),
    "bin keeps the partial last bin": ("const int64_t n_bins = n_samp / factor;\n  if (out_pitch < n_bins) return -1;\n#pragma omp parallel for schedule(static)\n  for (int c = 0; c < n_chan; ++c) {", "const int64_t n_bins = (n_samp + factor - 1) / factor;\n  if (out_pitch < n_bins) return -1;\n#pragma omp parallel for schedule(static)\n  for (int c = 0; c < n_chan; ++c) {"),
    "bin averages instead of sums": ("      out[(int64_t)c * out_pitch + j] = acc;\n    }\n  }", "      out[(int64_t)c * out_pitch + j] = acc / factor;\n    }\n  }"),
    "f32 bin skips first sample": ("for (int i = 0; i < factor; ++i) acc += (double)x[(int64_t)c * pitch + j * factor + i];", "for (int i = 1; i < factor; ++i) acc += (double)x[(int64_t)c * pitch + j * factor + i];"),
    "corner turn packs output nibbles high first": ("(uint8_t)(v0 | (v1 << 4));", "(uint8_t)(v1 | (v0 << 4));"),
    "corner turn reads input nibbles high first": ("const int v0 = (c % 2) ? (b0 >> 4) : (b0 & 15);", "const int v0 = (c % 2) ? (b0 & 15) : (b0 >> 4);"),
    "corner turn reads the next spectrum": ("out[(int64_t)c * out_pitch + t * es + b] = in[t * in_pitch + (int64_t)c * es + b];", "out[(int64_t)c * out_pitch + t * es + b] = in[(t + 1 < n_samp ? t + 1 : t) * in_pitch + (int64_t)c * es + b];"),
    "corner turn reverses element bytes": ("out[(int64_t)c * out_pitch + t * es + b] = in[t * in_pitch + (int64_t)c * es + b];", "out[(int64_t)c * out_pitch + t * es + b] = in[t * in_pitch + (int64_t)c * es + (es - 1 - b)];"),
    "normalised by channel count": ("out[(int64_t)r * n_out + t] = (float)acc[t];", "out[(int64_t)r * n_out + t] = (float)(acc[t] / n_chan);"),
    "32-bit top byte dropped": ("((int64_t)p[2] << 16) | ((int64_t)p[3] << 24);", "((int64_t)p[2] << 16);"),
    "32-bit sample stride of two bytes": ("const uint8_t *p = x + (int64_t)c * pitch_bytes + 4 * t;", "const uint8_t *p = x + (int64_t)c * pitch_bytes + 2 * t;"),
    "32-bit bytes 1 and 2 swapped": ("(int64_t)p[0] | ((int64_t)p[1] << 8) | ((int64_t)p[2] << 16)", "(int64_t)p[0] | ((int64_t)p[2] << 8) | ((int64_t)p[1] << 16)"),
    "abs sum counts each term twice": ("a[t] += fabs((double)row[t]);", "a[t] += 2.0 * fabs((double)row[t]);"),
    "abs sum without the absolute value": ("a[t] += fabs((double)row[t]);", "a[t] += (double)row[t];"),
    "abs sum over the unshifted window": ("a[t] += fabs((double)row[t]);", "a[t] += fabs((double)x[(int64_t)c * pitch + t]);"),
    "abs sum not cleared per row": ("    if (a)\n      for (int64_t t = 0; t < n_out; ++t) a[t] = 0.0;\n", ""),
}

PIN_CALLS = [
    ("hand delays", pins.test_shift_hand_derived_delays, ()),
    ("plan max small", pins.test_shift_plan_max, ("small",)),
    ("plan max lowfreq", pins.test_shift_plan_max, ("lowfreq_u4",)),
    ("monotone", pins.test_shift_special_cases_and_monotone, ("small",)),
    ("exact rational", pins.test_shift_matches_exact_rational, ("small",)),
    ("eq4 slope", pins.test_shift_against_narrow_band_form, ("grad_f32",)),
    ("literal u8", pins.test_forward_equals_literal_eq3, ("u8",)),
    ("literal u4", pins.test_forward_equals_literal_eq3, ("u4",)),
    ("literal f32", pins.test_forward_equals_literal_eq3, ("f32",)),
    ("literal u16", pins.test_forward_equals_literal_eq3, ("u16",)),
    ("u16 little-endian", pins.test_forward_u16_little_endian_samples, ()),
    ("u16 == u8", pins.test_forward_u16_small_values_equal_u8, ()),
    ("literal u32", pins.test_forward_equals_literal_eq3, ("u32",)),
    ("u32 little-endian", pins.test_forward_u32_little_endian_samples_and_u16_agreement, ()),
    ("dm0", pins.test_forward_dm0_is_channel_sum, ()),
    ("pulse", pins.test_forward_injected_pulse, ()),
    ("u4 == u8 == f32", pins.test_forward_u4_equals_u8_equals_f32, ()),
    ("dense", pins.test_forward_and_adjoint_against_dense_matrix, ()),
    ("dense abs sum", pins.test_forward_f32_abs_sum_against_dense_matrix, ()),
    ("dot exact", pins.test_adjoint_exact_dot_test_small_integers, ()),
    ("unread zero", pins.test_adjoint_unread_entries_are_zero, ()),
    ("bin reshape u8", pins.test_bin_equals_reshape_sum, ("u8",)),
    ("bin reshape f32", pins.test_bin_equals_reshape_sum, ("f32",)),
    ("bin identity", pins.test_bin_factor_one_identity_constant_and_impulse, ()),
    ("bin compose", pins.test_bin_factors_compose, ()),
    ("binned dm0", pins.test_binned_forward_dm0_is_sum_of_unbinned_dm0, ()),
    ("binned whole-bin delays", pins.test_binned_forward_with_delays_in_whole_bins, ()),
    ("corner turn u8", pins.test_corner_turn_is_numpy_transpose, ("u8",)),
    ("corner turn u16", pins.test_corner_turn_is_numpy_transpose, ("u16",)),
    ("corner turn u4", pins.test_corner_turn_u4_nibble_orders, ()),
    ("corner turn round trip", pins.test_corner_turn_round_trip_and_forward, ()),
]


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d
    oracle_front.use_library(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, workdir):
    old, new = MUTANTS[name]
    src = oracle_front.source()
    assert src.count(old) == 1, "mutation site not unique: " + name
    lib = oracle_front.compile_source(src.replace(old, new), os.path.join(workdir, "m%d.so" % abs(hash(name))))
    oracle_front.use_library(lib)
    caught = []
    try:
        for label, fn, args in PIN_CALLS:
            try:
                fn(*args)
            except (AssertionError, ValueError):
                caught.append(label)
                break
    finally:
        oracle_front.use_library(None)
    assert caught, "no pin caught the mutant: " + name
