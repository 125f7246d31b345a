"""GPU parity of the Eq. (12b) surface (ndft_caf12b) against the FP64 oracle.

Eq. (12b): the lag product of Eq. (6), then the ordinary DFT. The kernel decimates
each row (N = M L, L the largest power of two dividing N up to 512: length-L FFTs, then
M terms per bin), so the shapes cover every transform length 1 .. 512 (every radix
sequence), one and several work-groups per delay (with a ragged last group), odd
lengths (L = 1: the plain sum), ragged delay and bin windows and exact zeros, plus the
N = 65536 surface on sampled rows. FP32: l1-relative error per output <= 1e-5 against
the l1 mass of the real products (the oracle's scale); outputs whose scale is 0 exactly 0.
"""
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


def log(*a):
    print(*a, flush=True)


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0)), "non-zero output where the exact result is 0"
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


# n, tau0, n_tau, p0, n_dop, data
SHAPES = [
    (2, 0, 2, 0, 2, "gauss"),
    (4, 0, 4, -2, 4, "int_zeros"),
    (8, 1, 7, 0, 8, "gauss"),
    (16, 0, 16, -8, 16, "gauss"),
    (32, 3, 20, 5, 27, "int_zeros"),
    (64, 0, 64, -32, 64, "gauss"),
    (128, 0, 100, -64, 128, "gauss"),
    (256, 0, 256, 0, 256, "int_zeros"),
    (4096, 3, 300, -200, 400, "gauss"),     # L = 512, one group of 8 phases
    (12288, 0, 40, -256, 512, "gauss"),     # 24 phases: groups of 16 and a ragged 8
    (5120, 2, 33, -100, 200, "int_zeros"),  # L = 512, M = 10
    (999, 0, 130, -50, 101, "gauss"),       # odd: L = 1
    (1002, 7, 64, 0, 1002, "int_zeros"),    # L = 2, every bin
    (65540, 0, 3, -2, 5, "gauss"),          # L = 4, M = 16385: nine groups
    (17, 0, 17, 0, 17, "int_zeros"),
    (40000, 5, 20, -300, 600, "gauss"),     # L = 64, M = 625
]

_ORACLE = {}


def case(orc, shape):
    if shape not in _ORACLE:
        n, tau0, n_tau, p0, n_dop, kind = shape
        if kind == "gauss":
            s, r = synth.random_pair(n, seed=n + 15, zeros=0.02)
        else:
            s, r = synth.random_pair(n, seed=n + 16, zeros=0.2, integer=True)
        Ao, sc = orc.caf12b(s, r, tau0, n_tau, p0, n_dop)
        _ORACLE[shape] = (s, r, Ao, sc)
    return _ORACLE[shape]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_{s[5]}" for s in SHAPES])
def test_caf12b_vs_oracle(nd, orc, shape):
    n, tau0, n_tau, p0, n_dop, kind = shape
    s, r, Ao, sc = case(orc, shape)
    log("caf12b shape", shape)
    A = nd.caf12b(dev(s), dev(r), tau0, n_tau, p0, n_dop).cpu().numpy()
    e = rel_err(A, Ao, sc)
    log("caf12b max l1-relative error", e)
    assert e <= TOL


def test_caf12b_n65536_sampled_rows(nd, orc):
    c = synth.config3()
    rng = np.random.default_rng(35)
    rows = np.unique(np.concatenate([[0, 5, 37, 1023], rng.integers(0, c["n_tau"], 4)]))
    log("caf12b N = 65536 rows", rows.tolist())
    A = nd.caf12b(dev(c["s"]), dev(c["r"]), c["tau0"], c["n_tau"], c["p0"], c["n_dop"]).cpu().numpy()
    Ao, sc = orc.caf12b(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"], rows=rows)
    e = rel_err(A[rows], Ao, sc)
    log("caf12b N = 65536 sampled max l1-relative error", e)
    assert e <= TOL
    # the strongest cells of the surface are the clutter and target cells of the workload
    mag = np.abs(A)
    assert mag[0].argmax() == 256  # zero Doppler at zero delay (direct path)


def test_caf12b_zero_surveillance_is_exactly_zero(nd):
    s = np.zeros(4096, np.complex64)
    _, r = synth.random_pair(4096, seed=4)
    A = nd.caf12b(dev(s), dev(r), 0, 64, -32, 64)
    assert torch.count_nonzero(A).item() == 0


def test_caf12b_fp32_only(nd):
    s, r = synth.random_pair(256, seed=3)
    for prec in (1, 2):
        with pytest.raises(RuntimeError, match="UNSUPPORTED"):
            nd.caf12b(dev(s), dev(r), 0, 8, -4, 8, prec=prec)


def test_caf12b_deterministic_and_reuses_workspace(nd):
    s, r = synth.random_pair(16384, seed=10)
    a = nd.caf12b(dev(s), dev(r), 0, 100, -256, 512)
    ws = torch.full((nd.caf12b_workspace_bytes(16384, 0, 100, -256, 512),), 255, dtype=torch.uint8,
                    device="cuda")
    b = nd.caf12b(dev(s), dev(r), 0, 100, -256, 512, ws=ws)
    assert torch.equal(a, b)
