"""The fast exact transform (plan fp32x_fast_exact, N a power of two from 8 to 4096) against
the FP64 oracle: Eq. (7) rows (ndft_forward), Eq. (12a) and Eq. (12c) surfaces, every bin
and bin windows, Gaussian and integer data with exact zeros, more rows than work-groups.

The transform regroups the terms of Eq. (7) (folds over the power-of-two divisors of the
bin index, cyclic correlations over the odd residues, FFTs), so it is held to the FP32
tolerance of the other FP32 forms: (|dRe| + |dIm|) / scale <= 1e-5 per output, exact zeros
where the scale is 0.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
NAME = "fp32x_fast_exact"


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_0532_amd as m

    yield m
    m.set_plan(0, -1, 0)


@pytest.fixture
def fast(nd):
    names = [nd.plan_name(0, k) for k in range(nd.plan_count(0))]
    nd.set_plan(0, names.index(NAME), 0)
    yield
    nd.set_plan(0, -1, 0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0)), "non-zero output where the exact result is 0"
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


def rows(n, batch, seed, integer=False):
    rng = np.random.default_rng(seed)
    if integer:
        x = rng.integers(-3, 4, (batch, n)) + 1j * rng.integers(-3, 4, (batch, n))
    else:
        x = rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n))
        x.real[rng.uniform(size=x.shape) < 0.1] = 0.0
    return x.astype(np.complex64)


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("integer", [False, True])
def test_forward_every_bin(nd, orc, fast, n, integer):
    x = rows(n, 3, n + integer, integer)
    log("fast forward n", n, "integer", integer)
    X = nd.forward(dev(x), prec=0).cpu().numpy()
    Xo, sc = orc.ndft(x.astype(np.complex128))
    e = rel_err(X, Xo, sc)
    log("max l1-relative error", e)
    assert e <= TOL


@pytest.mark.parametrize("n,k0,kc", [(64, -5, 11), (1024, 1000, 100), (4096, -2048, 4096), (256, 255, 1)])
def test_forward_windows(nd, orc, fast, n, k0, kc):
    x = rows(n, 4, 7 * n)
    log("fast forward window", n, k0, kc)
    X = nd.forward(dev(x), k0=k0, k_count=kc, prec=0).cpu().numpy()
    Xo, sc = orc.ndft(x.astype(np.complex128), k0=k0, k_count=kc)
    assert rel_err(X, Xo, sc) <= TOL


def test_forward_more_rows_than_work_groups(nd, orc, fast):
    # 600 rows of 1024: four work-groups per compute unit at most, so rows loop
    x = rows(1024, 600, 11)
    x[17] = 0  # a zero row: exactly zero output
    X = nd.forward(dev(x), prec=0).cpu().numpy()
    pick = [0, 17, 255, 256, 511, 599]
    Xo, sc = orc.ndft(x[pick].astype(np.complex128))
    assert rel_err(X[pick], Xo, sc) <= TOL
    assert np.all(X[17] == 0)


@pytest.mark.parametrize(
    "shape",
    [(8, 0, 8, -3, 8), (64, 0, 64, 0, 64), (512, 3, 100, -200, 400), (1024, 0, 40, 0, 1024),
     (4096, 0, 12, 0, 4096), (4096, 4000, 96, -2048, 4096)],
)
@pytest.mark.parametrize("kind", ["gauss", "int_zeros"])
def test_caf_fast(nd, orc, fast, shape, kind):
    n, tau0, n_tau, p0, n_dop = shape
    if kind == "gauss":
        s, r = synth.random_pair(n, seed=n + 5, zeros=0.02)
    else:
        s, r = synth.random_pair(n, seed=n + 6, zeros=0.2, integer=True)
    log("fast caf", shape, kind)
    A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=0).cpu().numpy()
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop)
    e = rel_err(A, Ao, sc)
    log("max l1-relative error", e)
    assert e <= TOL


def test_caf_fast_is_built_in_for_config2(nd):
    plan, ks = nd.get_plan(0, 4096, 256, 0, 4096)
    assert nd.plan_name(0, plan) == NAME


def test_caf_fast_zero_and_negation(nd, fast):
    s, r = synth.random_pair(2048, seed=9, zeros=0.05)
    A = nd.caf(dev(np.zeros_like(s)), dev(r), 0, 30, -100, 300, prec=0).cpu().numpy()
    assert np.all(A == 0)
    A = nd.caf(dev(s), dev(r), 0, 30, -100, 300, prec=0).cpu().numpy()
    An = nd.caf(dev(-s), dev(r), 0, 30, -100, 300, prec=0).cpu().numpy()
    # every step is odd in z (sums, products with fixed tables, FFTs): exactly -A
    np.testing.assert_array_equal(An, -A)


@pytest.mark.parametrize("shape", [(64, 0, 64, 0, 64), (1024, 5, 60, -512, 1024), (4096, 100, 40, 0, 4096)])
@pytest.mark.parametrize("kind", ["gauss", "int_zeros"])
def test_caf12c_fast(nd, orc, fast, shape, kind):
    # Eq. (12c): the ordinary lag product s conj(r) (FP64, exact signs), then the operator
    # of Eq. (6) with the twiddles: the same transform on those rows
    n, tau0, n_tau, p0, n_dop = shape
    if kind == "gauss":
        s, r = synth.random_pair(n, seed=n + 15, zeros=0.02)
    else:
        s, r = synth.random_pair(n, seed=n + 16, zeros=0.2, integer=True)
    log("fast caf12c", shape, kind)
    A = nd.caf12c(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=0).cpu().numpy()
    Ao, sc = orc.caf12c(s, r, tau0, n_tau, p0, n_dop)
    e = rel_err(A, Ao, sc)
    log("max l1-relative error", e)
    assert e <= TOL


def test_caf12c_fast_is_built_in_for_wide_windows(nd):
    # the Eq. (12c) surface takes the fast transform where the sign-split walk would be
    # long: the built-in call equals the forced one bit for bit
    s, r = synth.random_pair(4096, seed=77, zeros=0.02)
    A = nd.caf12c(dev(s), dev(r), 0, 64, 0, 4096, prec=0).cpu().numpy()
    names = [nd.plan_name(0, k) for k in range(nd.plan_count(0))]
    nd.set_plan(0, names.index(NAME), 0)
    try:
        Af = nd.caf12c(dev(s), dev(r), 0, 64, 0, 4096, prec=0).cpu().numpy()
    finally:
        nd.set_plan(0, -1, 0)
    np.testing.assert_array_equal(A, Af)


def test_fast_tables_cache(nd, orc, fast):
    # the first call of a length fills the device's slot and reads it, later calls read
    # it; clearing and filling again gives the same bits (the capture of an uncached
    # length, which makes the tables in the workspace, is checked with the graph replays)
    x = rows(2048, 5, 91)
    nd.fast_tables_cached(reset=True)
    X1 = nd.forward(dev(x), prec=0).cpu().numpy()
    assert nd.fast_tables_cached() >> 11 & 1
    X2 = nd.forward(dev(x), prec=0).cpu().numpy()
    np.testing.assert_array_equal(X1, X2)
    nd.fast_tables_cached(reset=True)
    X3 = nd.forward(dev(x), prec=0).cpu().numpy()
    np.testing.assert_array_equal(X1, X3)
    Xo, sc = orc.ndft(x.astype(np.complex128))
    assert rel_err(X1, Xo, sc) <= TOL
