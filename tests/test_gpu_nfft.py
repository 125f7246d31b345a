"""GPU NFFT (ndft_nfft, Section 3) against the oracle's recursion, in both readings of
Eq. (10): every butterfly's twiddle product by Eq. (6), and the printed equation (ordinary
twiddle products, the operator in the length-1 sums).

Every intermediate's sign decides a jump of the result, so the comparison is with the
oracle's FP32 evaluation of the same recursion (oracle.nfft32 / nfft32_outer), bit for
bit; the FP64 recursion is checked to a tolerance. Lengths 1 .. 8192 (every power of two
in between is a distinct pass count) in LDS, rows of 2^14 .. 2^20 samples (the top levels
as passes over global memory), Gaussian and small-integer data with zeros, a batch larger
than the grid (rows looped by the work-groups), and the Section 3 tone example.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_0532_amd as m

    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192])
@pytest.mark.parametrize("kind", ["gauss", "int_zeros"])
def test_nfft_bit_exact_vs_fp32_recursion(nd, orc, n, kind):
    rng = np.random.default_rng(n + (0 if kind == "gauss" else 1))
    if kind == "gauss":
        x = (rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))).astype(np.complex64)
    else:
        x = (rng.integers(-3, 4, (5, n)) + 1j * rng.integers(-3, 4, (5, n))).astype(np.complex64)
        x[rng.uniform(size=(5, n)) < 0.2] = 0
    print("nfft n", n, kind, flush=True)
    X = nd.nfft(dev(x)).cpu().numpy()
    np.testing.assert_array_equal(X, orc.nfft32(x))
    if kind == "gauss":
        X64 = orc.nfft(x)
        assert np.max(np.abs(X - X64)) <= 1e-5 * np.abs(X64).max()


def test_nfft_many_rows(nd, orc):
    rng = np.random.default_rng(9)
    x = (rng.standard_normal((5000, 1024)) + 1j * rng.standard_normal((5000, 1024))).astype(np.complex64)
    X = nd.nfft(dev(x)).cpu().numpy()
    rows = np.array([0, 1, 2047, 2048, 4999])
    np.testing.assert_array_equal(X[rows], orc.nfft32(x[rows]))


def test_nfft_tone_example(nd, orc):
    # Section 3 example (its figure): x[n] = e^{j 2 pi 7 n / 64}, N = 64, peak at k = 7
    x = synth.config1()[:1]
    X = nd.nfft(dev(x)).cpu().numpy()[0]
    np.testing.assert_array_equal(X, orc.nfft32(x)[0])
    assert int(np.argmax(np.abs(X))) == 7


def test_nfft_rejects_bad_lengths(nd):
    for n in (3, 12, 24576):
        with pytest.raises(RuntimeError, match="INVAL"):
            nd.nfft(torch.zeros((2, n), dtype=torch.complex64, device="cuda"))


@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 512, 4096, 8192])
@pytest.mark.parametrize("kind", ["gauss", "int_zeros"])
def test_nfft_printed_reading_bit_exact(nd, orc, n, kind):
    rng = np.random.default_rng(n + 200 + (0 if kind == "gauss" else 1))
    if kind == "gauss":
        x = (rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))).astype(np.complex64)
    else:
        x = (rng.integers(-3, 4, (4, n)) + 1j * rng.integers(-3, 4, (4, n))).astype(np.complex64)
        x[rng.uniform(size=(4, n)) < 0.2] = 0
    print("nfft printed reading n", n, kind, flush=True)
    X = nd.nfft(dev(x), reading=nd.NFFT_PRINTED).cpu().numpy()
    np.testing.assert_array_equal(X, orc.nfft32_outer(x))
    X64 = orc.nfft_outer(x)
    assert np.max(np.abs(X - X64)) <= 1e-5 * max(1.0, np.abs(X64).max())


@pytest.mark.parametrize("reading", [0, 1])
@pytest.mark.parametrize("n,batch", [(1 << 14, 3), (1 << 15, 2), (1 << 16, 2), (1 << 17, 2), (1 << 20, 1)])
def test_nfft_long_rows_bit_exact(nd, orc, reading, n, batch):
    rng = np.random.default_rng(n + reading)
    x = (rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n))).astype(np.complex64)
    x[:, :: 97] = 0
    print("nfft long rows n", n, "batch", batch, "reading", reading, flush=True)
    X = nd.nfft(dev(x), reading=reading).cpu().numpy()
    ref = orc.nfft32_outer(x) if reading else orc.nfft32(x)
    np.testing.assert_array_equal(X, ref)
