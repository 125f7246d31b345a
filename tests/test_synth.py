"""Seeded input generators: determinism and the stated signal statistics."""
import hashlib

import numpy as np
import pytest

import synth


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_generators_are_deterministic():
    assert _digest(synth.config1()) == _digest(synth.config1())
    a = synth.config2()
    b = synth.config2()
    assert _digest(a["s"], a["r"]) == _digest(b["s"], b["r"])
    c = synth.config4(4)
    d = synth.config4(4)
    assert [_digest(x["s"], x["r"]) for x in c] == [_digest(x["s"], x["r"]) for x in d]


def test_reference_statistics():
    cfg = synth.config2()
    r = cfg["r"].astype(np.complex128)
    n = cfg["n"]
    assert r.dtype == np.complex128 and cfg["r"].dtype == np.complex64
    assert abs(np.mean(r.real ** 2 + r.imag ** 2) / 2.0 - 1.0) < 1e-5
    assert abs(np.mean(r.real ** 2) - 1.0) < 0.1 and abs(np.mean(r.imag ** 2) - 1.0) < 0.1
    spec = np.abs(np.fft.fft(r)) ** 2
    k = np.abs(np.fft.fftfreq(n, 1.0 / n))
    assert spec[k > 0.1 * n + 1].sum() < 1e-6 * spec.sum()


def test_exact_quadrant_tone():
    x = synth.config1()[0]
    assert x[16].real == 0.0 and x[48].real == 0.0
    assert x[0].imag == 0.0 and x[32].imag == 0.0


def test_config_shapes():
    c3 = synth.config3()
    assert c3["s"].shape == (65536,) and c3["n_tau"] == 1024 and c3["n_dop"] == 512
    c5 = synth.config5()
    r = c5["r"]
    assert np.all(np.abs(r.real) >= 0.05) and np.all(np.abs(r.imag) >= 0.05)
    assert c5["w"].shape == (256, 256)
    cp = synth.config4()
    assert len(cp) == 64
    for c in cp:
        assert 1024 <= c["n"] <= 32768 and 128 <= c["n_tau"] <= 512
        assert c["n_dop"] == 2 * (c["n"] // 16)


def test_eps_contaminated_mixture_statistics():
    rng = np.random.default_rng(5)
    x = synth.eps_contaminated(rng, 400000, 0.9, 0.25, 10.0)
    # per part: variance eps sigma1^2 + (1 - eps) sigma2^2, and the share of |part| > 2
    # (beyond 8 sigma1) is about the heavy-tail probability times P(|N(0, 100)| > 2)
    var = 0.9 * 0.25 ** 2 + 0.1 * 100.0
    assert np.var(x.real) == pytest.approx(var, rel=0.03)
    assert np.var(x.imag) == pytest.approx(var, rel=0.03)
    frac = np.mean(np.abs(x.real) > 2.0)
    assert frac == pytest.approx(0.1 * 0.8415, rel=0.05)


def test_robustness_pairs_are_seeded():
    for scene in synth.ROBUST_SCENES:
        for noise in synth.ROBUST_NOISES:
            s1, r1 = synth.robustness_pair(scene, noise, n=1024)
            s2, r2 = synth.robustness_pair(scene, noise, n=1024)
            assert s1.dtype == np.complex64 and np.array_equal(s1, s2) and np.array_equal(r1, r2)
