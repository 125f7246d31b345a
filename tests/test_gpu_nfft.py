"""GPU NFFT (ndft_nfft, Section 3) against the oracle's recursion.

Every intermediate's sign decides a jump of the result, so the comparison is with the
oracle's FP32 evaluation of the same recursion (oracle.nfft32), bit for bit; the FP64
recursion is checked to a tolerance. Lengths 1 .. 8192 (every power of two in between
is a distinct pass count), Gaussian and small-integer data with zeros, a batch larger
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
    for n in (3, 12, 16384):
        with pytest.raises(RuntimeError, match="INVAL"):
            nd.nfft(torch.zeros((2, n), dtype=torch.complex64, device="cuda"))
