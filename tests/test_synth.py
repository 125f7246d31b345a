"""Seeded input generators: determinism and the stated signal statistics."""
import hashlib

import numpy as np

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
