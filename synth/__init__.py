"""Seeded synthetic inputs shaped like the paper's passive-radar workload.

This module holds no arithmetic of the method (no additive operator, no twiddle-sign
logic, no NDFT): it only draws seeded signals, and both the GPU tests and the oracle
tests consume what it returns. Every generator works in FP64 and returns complex64
(the dtype the library takes); the oracle reads those complex64 values upcast exactly.

Signal model (Section 5 of the paper, Eqs. (15)-(16)): the surveillance channel is a
sum of delayed, Doppler-shifted copies of the reference plus noise,
``s[i] = sum_m a_m r[i - tau_m] e^{j 2 pi f_m i / N} + noise``, with r[m < 0] = 0.
The paper's stereo-FM reference (Eqs. (13)-(14)) leaves its modulation index and
channel statistics unstated, so the reference here is low-pass filtered complex
Gaussian noise of 0.2 f_s two-sided bandwidth (an FM-broadcast-like spectrum), scaled
to unit variance per real part.

Seeds: ``numpy.random.default_rng([1402, 532, config, sub])``.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = (1402, 532)


def rng_for(config: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE[0], SEED_BASE[1], int(config), int(sub)])


def exp_bins(k: int, n: int) -> np.ndarray:
    """e^{j 2 pi k i / n} for i in [0, n), exponent reduced as an integer mod n, with
    exact 0/+-1 components where 4 (k i mod n) is a multiple of n."""
    i = np.arange(n, dtype=np.int64)
    m = (int(k) * i) % n
    th = 2.0 * np.pi * m.astype(np.float64) / n
    out = np.cos(th) + 1j * np.sin(th)
    quad = (4 * m) % n == 0
    exact = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])
    out[quad] = exact[(4 * m[quad]) // n]
    return out


def complex_gaussian(rng: np.random.Generator, shape, sigma: float = 1.0) -> np.ndarray:
    """Real parts drawn first, then imaginary parts; N(0, sigma^2) per part."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return sigma * (re + 1j * im)


def lowpass_reference(rng: np.random.Generator, n: int, frac: float = 0.1) -> np.ndarray:
    """Complex Gaussian noise, brick-wall filtered to |k| <= floor(frac * n) bins and
    scaled to unit variance per real part (FP64)."""
    w = complex_gaussian(rng, n)
    W = np.fft.fft(w)
    k = np.fft.fftfreq(n, d=1.0 / n)
    W[np.abs(k) > math.floor(frac * n)] = 0.0
    x = np.fft.ifft(W)
    x = x / math.sqrt(np.mean(x.real ** 2 + x.imag ** 2) / 2.0)
    return x


def delayed(x: np.ndarray, tau: int) -> np.ndarray:
    """x[i - tau] with zeros before the start of the record (linear, not circular)."""
    out = np.zeros_like(x)
    if tau < x.shape[0]:
        out[tau:] = x[: x.shape[0] - tau]
    return out


def surveillance(ref: np.ndarray, rng: np.random.Generator, targets, clutter,
                 noise_db: float = -20.0) -> np.ndarray:
    """Eq. (16)-style scene. targets: [(delay, doppler_bin, amp_db)], clutter:
    [(delay, amp_db)]; dB levels are amplitude levels relative to the unit-variance
    reference; noise power is noise_db relative to the reference power E|r|^2 = 2."""
    n = ref.shape[0]
    s = np.zeros(n, np.complex128)
    for tau, dop, amp_db in targets:
        s += 10.0 ** (amp_db / 20.0) * delayed(ref, tau) * exp_bins(dop, n)
    for tau, amp_db in clutter:
        s += 10.0 ** (amp_db / 20.0) * delayed(ref, tau)
    sigma = math.sqrt(10.0 ** (noise_db / 10.0))  # per part: 2 sigma^2 = 0.01 * 2
    s += complex_gaussian(rng, n, sigma)
    return s


def c64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex64)


# ----------------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------------

def config1():
    """Single NDFT, N = 64: row 0 = e^{j 2 pi 7 n / 64} (exact quadrant values), rows
    1..16 i.i.d. complex Gaussian, unit variance per part. Returns complex64 [17][64]."""
    n = 64
    x = np.zeros((17, n), np.complex128)
    x[0] = exp_bins(7, n)
    x[1:] = complex_gaussian(rng_for(1, 1), (16, n))
    return c64(x)


def config1_numpy_tone():
    """The same tone from numpy.exp (components ~1e-16 instead of exact zeros)."""
    n = 64
    return np.exp(2j * np.pi * 7 * np.arange(n) / n)


def radar_pair(n: int, config: int, target=(37, 12, -10.0),
               clutter=((0, 0.0), (5, 0.0), (11, 0.0)), noise_db: float = -20.0):
    """(surveillance, reference) complex64 for the single-CPI radar workloads."""
    rng = rng_for(config, 0)
    r = lowpass_reference(rng, n)
    s = surveillance(r, rng, [target], list(clutter), noise_db)
    return c64(s), c64(r)


def config2():
    """N = 4096, delays 0..255, all 4096 Doppler bins (p0 = 0)."""
    s, r = radar_pair(4096, 2)
    return dict(s=s, r=r, n=4096, tau0=0, n_tau=256, p0=0, n_dop=4096)


def config3():
    """N = 65536, delays 0..1023, Doppler bins p in [-256, 256)."""
    s, r = radar_pair(65536, 3)
    return dict(s=s, r=r, n=65536, tau0=0, n_tau=1024, p0=-256, n_dop=512)


def config4(n_cpi: int = 64):
    """Batch of CPIs of uneven length: N log-uniform in [1024, 32768], delay counts
    uniform in [128, 512], Doppler bins [-floor(N/16), floor(N/16)), 1-4 targets with
    random delay, Doppler and -20..-5 dB amplitude, clutter 0/5/11 at 0 dB."""
    rng = rng_for(4, 0)
    cpis = []
    for _ in range(n_cpi):
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(32768)))))
        n_tau = int(rng.integers(128, 513))
        half = n // 16
        n_tgt = int(rng.integers(1, 5))
        tg = []
        for _t in range(n_tgt):
            tg.append((int(rng.integers(0, n_tau)), int(rng.integers(-half, half)),
                       float(rng.uniform(-20.0, -5.0))))
        r = lowpass_reference(rng, n)
        s = surveillance(r, rng, tg, [(0, 0.0), (5, 0.0), (11, 0.0)], -20.0)
        cpis.append(dict(s=c64(s), r=c64(r), n=n, tau0=0, n_tau=n_tau, p0=-half,
                         n_dop=2 * half, targets=tg))
    return cpis


def config5():
    """Differentiation workload: N = 8192, 256 delays x 256 Doppler bins (p in
    [-128, 128)), reference parts pushed to |part| >= 0.05, weights U[0, 1)."""
    n = 8192
    rng = rng_for(5, 0)
    r = lowpass_reference(rng, n)
    r = np.sign(r.real) * np.maximum(np.abs(r.real), 0.05) + 1j * (
        np.sign(r.imag) * np.maximum(np.abs(r.imag), 0.05))
    s = surveillance(r, rng, [(37, 12, -10.0)], [(0, 0.0), (5, 0.0), (11, 0.0)], -20.0)
    w = rng_for(5, 2).uniform(0.0, 1.0, (256, 256))
    return dict(s=c64(s), r=c64(r), n=n, tau0=0, n_tau=256, p0=-128, n_dop=256, w=w)


def random_pair(n: int, seed: int, zeros: float = 0.0, integer: bool = False):
    """Generic test inputs: complex Gaussian (or small integers), with a fraction of
    exact zero parts. Returns complex64 (s, r)."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 100, int(seed)])
    if integer:
        s = rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)
        r = rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)
    else:
        s = complex_gaussian(rng, n)
        r = complex_gaussian(rng, n)
    if zeros > 0:
        for a in (s, r):
            mr = rng.uniform(size=n) < zeros
            mi = rng.uniform(size=n) < zeros
            a.real[mr] = 0.0
            a.imag[mi] = 0.0
    return c64(s), c64(r)


def dyadic_pair(n: int, seed: int):
    """Inputs whose parts are drawn from four separated sets of powers of two: Re s in
    {+-2, +-4}, Im s = +-1/4, Re r = +-1, Im r = +-1/2 (random signs). Every value is a
    multiple of 1/4 and no two magnitudes of different parts coincide, so sums of their
    magnitudes never tie and any FP32 sum of such terms below 2^22 is exact. Returns
    complex64 (s, r)."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 101, int(seed)])
    sg = lambda: rng.choice([-1.0, 1.0], n)  # noqa: E731
    s = sg() * rng.choice([2.0, 4.0], n) + 1j * sg() * 0.25
    r = sg() * 1.0 + 1j * sg() * 0.5
    return c64(s), c64(r)


def sparse_pair(n: int, seed: int, count: int = 48, positions=()):
    """A surveillance record with only `count` non-zero samples (complex Gaussian), at the
    given positions plus random distinct others, against a dense complex Gaussian
    reference: every delay row then holds at most `count` non-zero lag terms, so a single
    wrong sign operand moves an output by a large fraction of its l1 scale. Returns
    complex64 (s, r)."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 102, int(seed)])
    pos = sorted({int(p) % n for p in positions})
    taken = set(pos)
    rest = [int(k) for k in rng.permutation(n) if int(k) not in taken]
    pos = pos + rest[: max(0, count - len(pos))]
    s = np.zeros(n, np.complex128)
    s[pos] = complex_gaussian(rng, len(pos))
    r = complex_gaussian(rng, n)
    return c64(s), c64(r)


# ----------------------------------------------------------------------------------
# Robustness scenes: targets and clutter under AWGN or eps-contaminated Gaussian noise
# ----------------------------------------------------------------------------------

def eps_contaminated(rng: np.random.Generator, shape, eps: float, sigma1: float,
                     sigma2: float) -> np.ndarray:
    """Complex noise whose real and imaginary parts are drawn independently from
    N(0, sigma1^2) with probability eps and from N(0, sigma2^2) (the heavy tail) otherwise."""
    shape = (shape,) if isinstance(shape, int) else tuple(shape)
    pick = rng.uniform(size=(2,) + shape) < eps
    g = rng.standard_normal((2,) + shape)
    parts = np.where(pick, sigma1 * g, sigma2 * g)
    return parts[0] + 1j * parts[1]


# scene -> (targets [(delay, doppler_bin, amp_db)], clutter [(delay, amp_db)]); amplitudes
# relative to the unit-variance reference, clutter at zero Doppler
ROBUST_SCENES = {
    "2 targets 1 clutter": ([(37, 11, -6.0), (80, -23, -8.0)], [(5, 0.0)]),
    "4 targets 2 clutters": ([(37, 11, -6.0), (80, -23, -8.0), (20, 40, -6.0), (101, -7, -10.0)],
                             [(5, 0.0), (12, -3.0)]),
    "1 target 3 clutters": ([(64, 17, -6.0)], [(3, 0.0), (9, -3.0), (15, -6.0)]),
}
# noise -> ("awgn", noise_db) or ("eps", eps, sigma1, sigma2): the four noise cases of
# each scene in the paper's detection tables (AWGN at 3 dB and 6 dB SNR, i.e. noise power
# 3 / 6 dB below the reference power, and the two contaminated mixtures)
ROBUST_NOISES = {
    "awgn 3 dB": ("awgn", -3.0),
    "awgn 6 dB": ("awgn", -6.0),
    "eps 0.9 / 0.25 / 10": ("eps", 0.9, 0.25, 10.0),
    "eps 0.8 / 0.5 / 20": ("eps", 0.8, 0.5, 20.0),
}
# surface window of the detection runs: N = 8192, delays 0..127, Doppler bins -64..63
ROBUST_WINDOW = (8192, 0, 128, -64, 128)


def robustness_pair(scene: str, noise: str, n: int = 8192, seed: int = 0):
    """(surveillance, reference) complex64 for one scene and noise of the robustness runs:
    low-pass reference (noise free), delayed / Doppler-shifted copies for the objects."""
    rng = rng_for(6, seed)
    r = lowpass_reference(rng, n)
    targets, clutter = ROBUST_SCENES[scene]
    s = surveillance(r, rng, targets, clutter, noise_db=-300.0)
    kind = ROBUST_NOISES[noise]
    if kind[0] == "awgn":
        s = s + complex_gaussian(rng, n, math.sqrt(10.0 ** (kind[1] / 10.0)))
    else:
        s = s + eps_contaminated(rng, n, *kind[1:])
    return c64(s), c64(r)


def scene_objects(scene: str, p0: int):
    """(delay row, bin column) of every target and clutter object of a scene on a surface
    whose first Doppler column is bin p0 (delay rows from 0)."""
    targets, clutter = ROBUST_SCENES[scene]
    return [(d, q - p0) for d, q, _ in targets] + [(d, -p0) for d, _ in clutter]


def object_margin(A, objects, guard: int = 3):
    """Detection on a surface magnitude (the side-lobe floor of the detection tables):
    floor = the largest |A| farther than +-guard cells (delay and Doppler) from every
    object; an object is detected when its own cell stands above the floor. margin_db =
    20 log10(floor / weakest object), below 0 when every object is detected.
    Scoring of the scenes only: no arithmetic of the method."""
    mag = np.abs(np.asarray(A))
    mask = np.ones(mag.shape, bool)
    for l, q in objects:
        mask[max(0, l - guard):l + guard + 1, max(0, q - guard):q + guard + 1] = False
    floor = float(mag[mask].max())
    vals = [float(mag[l, q]) for l, q in objects]
    return {"detected": int(sum(v > floor for v in vals)), "objects": len(objects),
            "margin_db": 20.0 * math.log10(floor / max(min(vals), 1e-30)),
            "object_db": [20.0 * math.log10(max(v, 1e-30) / floor) for v in vals]}
