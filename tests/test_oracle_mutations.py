"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/fh_oracle.c (a
dropped term, a flipped sign, swapped operands, an off-by-one, a wrong
rounding, the accumulated row step, wrong tie / exclusion / separation
rules), builds it with the oracle's own flags, routes the oracle through it,
and runs the pins of tests/test_oracle.py and tests/test_oracle_geometry.py
against it: at least one pin must fail for every mutant, and every pin must
pass on the unmutated source.  The pins compare the oracle with the paper's
geometry, closed forms, invariants and an independent cell-major
evaluation, never with itself, so a pin that catches a mutant shows that the
mistake would not have gone unseen.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle as T
import test_oracle_geometry as TG

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "fh_oracle.c")).read()

MUTANTS = [
    ("dropped b0 term", "return x - b0 * QI - (int64_t)kf * (QI / 2);", "return x - (int64_t)kf * (QI / 2);"),
    ("half-width sign", "return x - b0 * QI - (int64_t)kf * (QI / 2);", "return x - b0 * QI + (int64_t)kf * (QI / 2);"),
    ("Doppler sign", "double d = 1.0 + ((vi[0] * nhat[0]", "double d = 1.0 - ((vi[0] * nhat[0]"),
    ("swapped velocity components", "(vi[0] * nhat[0] + vi[1] * nhat[1])", "(vi[1] * nhat[0] + vi[0] * nhat[1])"),
    ("D instead of 1/D", "r[i] = 1.0 / d;", "r[i] = d;"),
    ("reference time dropped", "tau[i] = t[i] - t0;", "tau[i] = t[i];"),
    ("spin-down sign", "int64_t L = edge[p] - shift;", "int64_t L = edge[p] + shift;"),
    ("row spin-down without fdot0", "double fs = fdot0 + (double)s * dfdot;", "double fs = (double)s * dfdot;"),
    ("accumulated row step", "double fs = fdot0 + (double)s * dfdot;\n    return llrint((fs * tau) * S);",
     "return llrint((fdot0 * tau) * S) + (int64_t)s * llrint((dfdot * tau) * S);"),
    ("stripe one bin wider", "lab < L + width", "lab <= L + width"),
    ("ceil for the centre", "return (int64_t)floor(x);", "return (int64_t)ceil(x);"),
    ("weights ignored", "row[b] += wi;", "row[b] += 1.0;"),
    ("value order reversed", "if (v != bv) return v > bv;", "if (v != bv) return v < bv;"),
    ("bin tie reversed", "if (b != bb) return b < bb;", "if (b != bb) return b > bb;"),
    ("row tie reversed", "return s < bs;", "return s > bs;"),
    ("exclusion off by one", "if (d <= excl) continue;", "if (d < excl) continue;"),
    ("separation off by one", "if (d < sep) found2 = 0;", "if (d <= sep) found2 = 0;"),
]


def _geometry_pin():
    """The full-grid stripe-edge pin of test_oracle_geometry on 4000 pairs."""
    pm, grid, rng = TG._batch_geometry(20_000, seed=8333)
    nhat = TG.synth.sky_uniform(1, rng)[0]
    peaks = rng.integers(0, pm.n_peaks, size=4000)
    rows = rng.integers(0, grid.ns, size=4000).astype(np.int32)
    L = oracle.left_edges(pm, grid, nhat, peaks, rows)
    e_q, _ = TG._exact_edges(pm, grid, nhat, peaks, rows)
    d = [float(int(a) - b) for a, b in zip(L, e_q)]
    assert min(d) >= -1.5 - 1e-3 and max(d) <= 0.5 + 1e-3
    bad, _ = TG._first_bin_mismatches(L, e_q)
    assert bad == 0


def _candidate_pins():
    for case in T._load_candidate_cases():
        T.test_candidates_hand_built(case)


PINS = [
    ("single peak K_f 1", lambda: T.test_single_peak_is_a_line_of_kf_bins(1)),
    ("single peak K_f 10", lambda: T.test_single_peak_is_a_line_of_kf_bins(10)),
    ("vertical stripe at tau 0", T.test_zero_tau_gives_vertical_stripe),
    ("closed form without Doppler", T.test_no_doppler_closed_form),
    ("row count invariant", T.test_row_count_invariant_without_clipping),
    ("time reversal", T.test_time_reversal_symmetry),
    ("noiseless injection", lambda: T.test_noiseless_injection_peaks_at_n_fft(1)),
    ("cell-major brute force K_f 10", lambda: T.test_brute_force_cell_major_matches(10, 0)),
    ("cell-major brute force K_f 2", lambda: T.test_brute_force_cell_major_matches(2, 1)),
    ("float geometry", T.test_float_geometry_cross_check),
    ("weights per FFT", T.test_unit_weights_equal_counts_and_weights_are_per_fft),
    ("hand-built candidate maps", _candidate_pins),
    ("full-grid edge geometry", _geometry_pin),
]


def _build(src, tmp_path, name):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(src)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), "-lm"], check=True)
    return str(so)


def _failing_pins(path):
    failed = []
    with oracle._library(path):
        for name, pin in PINS:
            try:
                pin()
            except AssertionError:
                failed.append(name)
    return failed


def test_every_pin_passes_on_the_oracle_source(tmp_path):
    assert _failing_pins(_build(SRC, tmp_path, "unmutated")) == []


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_mutant_fails_a_pin(tmp_path, mutant):
    name, old, new = mutant
    assert SRC.count(old) >= 1, "mutation site not found: " + name
    failed = _failing_pins(_build(SRC.replace(old, new), tmp_path, "mutant"))
    assert failed, "no pin catches: " + name
