"""GPU parity of the whole-row decimated DFT for transform length 512 (N a multiple of
512, at most 1024 bins, enough delay rows): the Eq. (12b) surface (lag products), the FP32
sign-split form of Eq. (12a) (its twiddle half: the exact lag signs) and the FP32 form of
Eq. (12c) (signs of the ordinary lag product), each against the FP64 oracle on sampled
delay rows. The shapes cover a ragged last group of transforms (M not a multiple of 16),
a single group, the largest bin window, one bin, bins starting at 0 and wrapping past N,
delay rows near the end of the record (mostly zero lag products), and more rows than the
work-groups (taken in XCD order) cover in one pass. The sign halves read the sign codes of
the twiddle-sign kernel and add its partial planes themselves.
Tolerance: l1-relative per output <= 1e-5 (FP32)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_0532_amd as m

    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0)), "non-zero output where the exact result is 0"
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


# n, tau0, n_tau, p0, n_dop, data
SHAPES = [
    (20480, 0, 128, -512, 1024, "gauss"),     # M = 40: groups 16, 16, 8; every bin window slot
    (8704, 0, 130, 0, 777, "int_zeros"),      # M = 17: one full group and one of a single phase
    (8192, 7990, 192, 4000, 1, "gauss"),      # delays up to N - 10, one bin near N/2
    (4096, 3, 300, -200, 400, "int_zeros"),   # M = 8: a single partial group
    (16384, 1, 256, 16000, 700, "gauss"),     # bins wrapping past N
    (12288, 0, 520, -100, 200, "int_zeros"),  # 520 rows over 512 work-groups in XCD order
]


def data(shape):
    n, kind = shape[0], shape[5]
    if kind == "gauss":
        return synth.random_pair(n, seed=n + 51, zeros=0.02)
    return synth.random_pair(n, seed=n + 52, zeros=0.2, integer=True)


def rows_of(n_tau):
    rng = np.random.default_rng(n_tau)
    return np.unique(np.concatenate([[0, 1, n_tau // 2, n_tau - 1], rng.integers(0, n_tau, 4)]))


def fftd_plan(nd):
    for k in range(nd.plan_count(nd.FP32)):
        if nd.plan_name(nd.FP32, k).startswith("fp32s_fftd"):
            return k
    raise AssertionError("no FP32 FFT plan")


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_{s[2]}x{s[4]}" for s in SHAPES])
def test_caf12b_whole_row_kernel(nd, orc, shape):
    n, tau0, n_tau, p0, n_dop, _ = shape
    s, r = data(shape)
    rows = rows_of(n_tau)
    print("dft512 caf12b", shape, flush=True)
    A = nd.caf12b(dev(s), dev(r), tau0, n_tau, p0, n_dop).cpu().numpy()
    Ao, sc = orc.caf12b(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    assert rel_err(A[rows], Ao, sc) <= TOL


# the sign-split form's twiddle-sign half walks sign runs; its plan is admitted where the
# largest base b of the window has 256 b <= N (a handful of runs per 256-sample chunk)
SPLIT_SHAPES = [
    (20480, 0, 128, -80, 160, "gauss"),       # M = 40
    (8704, 0, 130, 0, 34, "int_zeros"),       # M = 17, bins from 0 (bin 0 summed apart)
    (8192, 7990, 192, -16, 32, "gauss"),      # delays near the end of the record
    (16384, 1, 256, 16320, 128, "gauss"),     # bins wrapping past N
    (10240, 0, 600, -40, 80, "gauss"),        # M = 20; 600 rows over 512 work-groups in XCD order
]


@pytest.mark.parametrize("shape", SPLIT_SHAPES, ids=[f"n{s[0]}_{s[2]}x{s[4]}" for s in SPLIT_SHAPES])
def test_fp32_signsplit_fft_half(nd, orc, shape):
    n, tau0, n_tau, p0, n_dop, _ = shape
    s, r = data(shape)
    rows = rows_of(n_tau)
    print("dft512 caf fp32 fft half", shape, flush=True)
    nd.set_plan(nd.FP32, fftd_plan(nd), 0)
    try:
        A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=nd.FP32).cpu().numpy()
        C = nd.caf12c(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=nd.FP32).cpu().numpy()
    finally:
        nd.set_plan(nd.FP32, -1, 0)
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    assert rel_err(A[rows], Ao, sc) <= TOL
    Co, scc = orc.caf12c(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    assert rel_err(C[rows], Co, scc) <= TOL


def test_whole_row_kernel_deterministic(nd):
    s, r = synth.random_pair(20480, seed=77)
    a = nd.caf12b(dev(s), dev(r), 0, 200, -300, 600)
    b = nd.caf12b(dev(s), dev(r), 0, 200, -300, 600)
    assert torch.equal(a, b)
