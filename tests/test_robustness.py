"""Detection runs of Section 5 (Tables 1-2 analogue) on the FP64 oracle, and pins of the
ordinary cross-ambiguity function of Eq. (11) the runs compare against."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_robustness  # noqa: E402


def test_caf11_tone_closed_form():
    # s = r delayed by d and shifted by f bins, |r| = 1 everywhere: the lag products of
    # delay d are e^{j 2 pi f i / N} for i >= d (0 before), so A[d][f] = N - d exactly
    # (up to rounding) and A[d][f + m] = sum_{i >= d} W^{m i}, a geometric sum.
    n, d, f = 256, 7, 5
    ph = np.exp(2j * np.pi * np.arange(n) * 0.137)
    r = synth.c64(ph)
    s = synth.c64(synth.delayed(r.astype(np.complex128), d) * np.exp(2j * np.pi * f * np.arange(n) / n))
    A = oracle.caf11(s, r, 0, 16, 0, 16)
    # |z| = 1 up to the complex64 rounding of the inputs (a few 1e-8 per sample)
    assert abs(A[d, f] - (n - d)) < 1e-6 * n
    m = 3
    w = np.exp(-2j * np.pi * m / n)
    geo = (w ** d - w ** n) / (1 - w)
    assert abs(A[d, f + m] - geo) < 1e-6 * n


def test_caf11_parseval_and_window():
    # every bin of a row: sum_p |A[l][p]|^2 = N sum_i |z_l[i]|^2 (Parseval); a window of
    # bins starting at a negative p0 picks the same values mod N
    n = 128
    s, r = synth.random_pair(n, seed=11)
    A = oracle.caf11(s, r, 3, 4, 0, n)
    for j in range(4):
        z = s.astype(np.complex128) * np.conj(synth.delayed(r.astype(np.complex128), 3 + j))
        assert abs(np.sum(np.abs(A[j]) ** 2) - n * np.sum(np.abs(z) ** 2)) < 1e-9 * n * np.sum(np.abs(z) ** 2)
    B = oracle.caf11(s, r, 3, 4, -10, 20)
    np.testing.assert_array_equal(B, A[:, (np.arange(-10, 10)) % n])


def test_object_margin_scoring():
    # two objects on a flat floor of 1: one at 4 (12.04 dB above), one at 0.5 (below)
    A = np.ones((20, 20))
    A[5, 5] = 4.0
    A[15, 12] = 0.5
    m = synth.object_margin(A, [(5, 5), (15, 12)])
    assert m["detected"] == 1 and m["objects"] == 2
    assert abs(m["margin_db"] - 20 * np.log10(1 / 0.5)) < 1e-12
    assert abs(m["object_db"][0] - 20 * np.log10(4.0)) < 1e-12
    # cells within +-3 of an object are not part of the floor
    A[7, 8] = 100.0
    assert synth.object_margin(A, [(5, 5), (15, 12)])["detected"] == 1


def test_golden_covers_every_scene_and_noise():
    g = make_robustness.parse()
    for scene in synth.ROBUST_SCENES:
        objs = synth.scene_objects(scene, synth.ROBUST_WINDOW[3])
        for noise in synth.ROBUST_NOISES:
            for surf in make_robustness.SURFACES:
                det, nobj, margin, levels = g[(scene, noise, surf)]
                assert nobj == len(objs) == len(levels)
                assert det == sum(v > 0 for v in levels)
                assert abs(margin - max(-v for v in levels)) < 1e-3


@pytest.mark.parametrize("scene", list(synth.ROBUST_SCENES))
def test_golden_outcomes_from_the_oracle(scene):
    # the stored outcomes are what the oracle's surfaces give (detection exactly, levels to
    # the stored digits)
    g = make_robustness.parse()
    for noise in synth.ROBUST_NOISES:
        res = make_robustness.outcomes(scene, noise)
        for surf in make_robustness.SURFACES:
            det, nobj, margin, levels = g[(scene, noise, surf)]
            m = res[surf]
            assert m["detected"] == det and m["objects"] == nobj, (scene, noise, surf)
            assert abs(m["margin_db"] - margin) < 2e-4
            np.testing.assert_allclose(m["object_db"], levels, atol=2e-4)
