"""Sign operands of the hot path itself, bit for bit.

The sign-split plans evaluate every cell as T + D (the identity of Eq. (1)-(2) applied to
the four real operators of Eq. (6)): T = sum_i csgn(W^{ip}) z_l[i] takes its twiddle signs
from the crossing walk of the lag kernel, D = sum_i W^{ip} csgn(z_l[i]) takes its lag
signs from the 2-bit code words that kernel writes for the matrix cores (or, in the FP32
plan, from the FFT kernel's own exact-sign fill). ndft_dbg_split runs the plan's lag kernel
exactly as the surface call does and returns the decoded code words and T alone, so:

* lag signs: the decoded code words equal the oracle's exact lag signs (Eq. (2) case
  analysis on exact sums) for every delay and sample, on the N = 65536 radar workload,
  on cancelling data and on ties;
* twiddle signs: on dyadic data (every value a multiple of 1/4, every lag component
  non-zero) all FP32 sums of the lag kernel are exact, so T must equal the oracle's
  sum_i csgn(W^{ip}) z_l[i] bit for bit; one wrong twiddle sign moves it by at least 1/4;
* the D half: A - T must equal sum_i W^{ip} csgn(z_l[i]) (oracle twiddles and signs)
  to within 0.5 in |dRe| + |dIm|, while one wrong lag sign moves it by at least 1
  (|W| = 1 and a sign changes by 1 or 2);
* sparse surveillance records (impulses): each delay row holds at most 48 non-zero lag
  terms, so one wrong sign operand anywhere is an l1-relative error of order 1e-2, far
  above the tolerances; run for every plan at the N = 65536 and N = 4096 workload shapes.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-4, 2: 1e-4}
SPLIT_PREFIX = ("bf16x2s_", "bf16x2g_", "fp8s_", "fp32s_")


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_0532_amd as m

    yield m
    for p in (0, 1, 2):
        m.set_plan(p, -1, 0)


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


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def oracle_lag_rows(orc, s, r, delays, lin=False, want_z=True):
    """(z [len(delays)][n] complex128 or None, signs [len(delays)][n][2] int8) from the
    oracle, rows in parallel threads (the C oracle releases the interpreter lock)."""
    fn = orc.lag_row_lin if lin else orc.lag_row
    n = s.shape[0]
    z = np.zeros((len(delays), n), np.complex128) if want_z else None
    sg = np.zeros((len(delays), n, 2), np.int8)

    def one(k):
        zk, sg[k] = fn(s, r, int(delays[k]))
        if want_z:
            z[k] = zk

    with cf.ThreadPoolExecutor(workers()) as ex:
        list(ex.map(one, range(len(delays))))
    return z, sg


def split_plans(nd):
    out = []
    for p in (0, 1, 2):
        for k in range(nd.plan_count(p)):
            if nd.plan_name(p, k).startswith(SPLIT_PREFIX):
                out.append((p, k))
    return out


def all_plans():
    import paper_1402_0532_amd as m

    try:
        return [(p, k) for p in (0, 1, 2) for k in range(m.plan_count(p))]
    except Exception:  # no library: the module fixture skips
        return [(0, 0)]


def all_split_plans():
    import paper_1402_0532_amd as m

    try:
        return split_plans(m)
    except Exception:
        return [(1, 0)]


def bins(n, p0, n_dop):
    return (p0 + np.arange(n_dop)) % n


def twiddle_sign_matrix(orc, n, p0, n_dop):
    """(Sr, Si) float64 [n_dop][n]: the oracle's exact twiddle signs."""
    S = orc.twiddle_signs(n, p0, n_dop)
    return S[:, :, 0].astype(np.float64), S[:, :, 1].astype(np.float64)


def oracle_T(orc, z, sg, n, p0, n_dop):
    """T[l][q] = sum_i csgn(W^{i p_q}) z_l[i], and at p_q = 0 mod n the whole cell
    sum_i z_l[i] + csgn(z_l[i]); exact in FP64 for dyadic data."""
    Sr, Si = twiddle_sign_matrix(orc, n, p0, n_dop)
    zr, zi = z.real.T.copy(), z.imag.T.copy()  # [n][rows]
    T = (Sr @ zr - Si @ zi) + 1j * (Sr @ zi + Si @ zr)  # [n_dop][rows]
    T = T.T.copy()
    q0 = np.nonzero(bins(n, p0, n_dop) == 0)[0]
    if q0.size:
        d0 = sg[:, :, 0].sum(axis=1).astype(np.float64) + 1j * sg[:, :, 1].sum(axis=1).astype(np.float64)
        T[:, q0[0]] = z.sum(axis=1) + d0
    return T


def oracle_D(orc, sg, n, p0, n_dop):
    """D[l][q] = sum_i W^{i p_q} csgn(z_l[i]) with the oracle's twiddles (exact at the
    quadrant points); column p_q = 0 mod n set to 0 (that bin is summed whole in T)."""
    wt = np.array([orc.twiddle(m, n) for m in range(n)])
    ps = bins(n, p0, n_dop)
    i = np.arange(n, dtype=np.int64)
    sig = (sg[:, :, 0].astype(np.float64) + 1j * sg[:, :, 1].astype(np.float64)).T  # [n][rows]
    D = np.zeros((n_dop, sg.shape[0]), np.complex128)
    for q0 in range(0, n_dop, 64):
        F = wt[(ps[q0:q0 + 64, None] * i[None, :]) % n]
        D[q0:q0 + 64] = F @ sig
    D = D.T.copy()
    D[:, ps == 0] = 0
    return D


# ------------------------------------------------------------------------------------
# lag signs: the code words of the lag kernel
# ------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cfg3():
    return synth.config3()


@pytest.fixture(scope="module")
def cfg3_signs(orc, cfg3):
    c = cfg3
    log("oracle lag signs of all", c["n_tau"], "delays at N =", c["n"])
    _, sg = oracle_lag_rows(orc, c["s"], c["r"], np.arange(c["tau0"], c["tau0"] + c["n_tau"]), want_z=False)
    return sg


@pytest.mark.parametrize("prec", [1, 2, 0])
def test_lag_codes_config3_every_delay(nd, cfg3, cfg3_signs, prec):
    c = cfg3
    plan, _ = nd.get_plan(prec, c["n"], c["n_tau"], c["p0"], c["n_dop"])
    log("lag codes config3 prec", prec, "plan", nd.plan_name(prec, plan))
    assert nd.plan_name(prec, plan).startswith(SPLIT_PREFIX)
    lg, _ = nd.dbg_split(dev(c["s"]), dev(c["r"]), c["tau0"], c["n_tau"], c["p0"], c["n_dop"], prec=prec,
                         T=False)
    lg = lg.cpu().numpy()
    bad = np.argwhere(lg != cfg3_signs)
    assert bad.size == 0, ("first mismatches (delay, sample, part)", bad[:8].tolist())


def test_lag_codes_config3_eq12c_every_delay(nd, orc, cfg3):
    c = cfg3
    _, sg = oracle_lag_rows(orc, c["s"], c["r"], np.arange(c["tau0"], c["tau0"] + c["n_tau"]), lin=True,
                            want_z=False)
    lg, _ = nd.dbg_split(dev(c["s"]), dev(c["r"]), c["tau0"], c["n_tau"], c["p0"], c["n_dop"], prec=1,
                         lin=True, T=False)
    lg = lg.cpu().numpy()
    bad = np.argwhere(lg != sg)
    assert bad.size == 0, ("first mismatches (delay, sample, part)", bad[:8].tolist())


def cancel_pair(n, seed):
    """Lag products whose FP32 value cancels to 0 while the exact value is +-1/2 or 0:
    s = (2^24, -2^24) against r = (1, 1/2), among small integers and zeros."""
    rng = np.random.default_rng(seed)
    s = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex64)
    r = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex64)
    big = rng.uniform(size=n) < 0.3
    s[big] = np.complex64(2.0 ** 24 - 2.0 ** 24 * 1j) * rng.choice([1, -1], big.sum())
    r[big] = np.complex64(1.0 + 0.5j)
    return s, r


def tie_pair(n, seed):
    """Exact ties and one-ulp differences between |s_r| + |r_r| and |s_i| + |r_i|, with
    denormal and zero parts."""
    rng = np.random.default_rng(seed)
    base = rng.integers(1, 5, n).astype(np.float32)
    eps = np.spacing(np.float32(4.0))
    s = (base + 1j * (base + rng.integers(-1, 2, n) * eps)).astype(np.complex64)
    r = (rng.integers(1, 3, n) * np.sign(rng.standard_normal(n))
         + 1j * rng.integers(1, 3, n) * np.sign(rng.standard_normal(n))).astype(np.complex64)
    tiny = rng.uniform(size=n) < 0.05
    s.real[tiny] = np.float32(1e-40)
    r.imag[rng.uniform(size=n) < 0.05] = 0.0
    return s, r


@pytest.mark.parametrize("prec,plan", all_split_plans())
@pytest.mark.parametrize("kind", ["cancel", "ties"])
@pytest.mark.parametrize("lin", [False, True])
def test_lag_codes_hard_data_every_plan(nd, orc, prec, plan, kind, lin):
    n, tau0, n_tau, p0, n_dop = 8192, 3, 70, -33, 66
    s, r = cancel_pair(n, 31) if kind == "cancel" else tie_pair(n, 32)
    _, sg = oracle_lag_rows(orc, s, r, np.arange(tau0, tau0 + n_tau), lin=lin, want_z=False)
    nd.set_plan(prec, plan, 0)
    log("lag codes", kind, "lin", lin, "plan", nd.plan_name(prec, plan))
    try:
        lg, _ = nd.dbg_split(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec, lin=lin, T=False)
    finally:
        nd.set_plan(prec, -1, 0)
    lg = lg.cpu().numpy()
    bad = np.argwhere(lg != sg)
    assert bad.size == 0, ("first mismatches (delay, sample, part)", bad[:8].tolist())


# ------------------------------------------------------------------------------------
# twiddle signs: T bit for bit on dyadic data
# ------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def dyadic65536(orc):
    n, tau0, n_tau, p0, n_dop = 65536, 0, 1024, -256, 512
    s, r = synth.dyadic_pair(n, 1)
    rng = np.random.default_rng(41)
    rows = np.unique(np.concatenate([[0, 1, 15, 16, 255, 256, 1023], rng.integers(0, n_tau, 41)]))
    out = {}
    for lin in (False, True):
        z, sg = oracle_lag_rows(orc, s, r, tau0 + rows, lin=lin)
        # every lag component at i >= d is non-zero (the data are built for it); the
        # zero-padded head of each row is exactly zero
        for k, d in enumerate(tau0 + rows):
            assert np.all(sg[k, d:] != 0) and np.all(sg[k, :d] == 0)
        out[lin] = oracle_T(orc, z, sg, n, p0, n_dop)
    return (s, r, n, tau0, n_tau, p0, n_dop, rows), out


@pytest.mark.parametrize("prec", [1, 2, 0])
@pytest.mark.parametrize("lin", [False, True])
def test_twiddle_signs_T_exact_n65536(nd, dyadic65536, prec, lin):
    (s, r, n, tau0, n_tau, p0, n_dop, rows), Tref = dyadic65536
    plan, _ = nd.get_plan(prec, n, n_tau, p0, n_dop)
    log("T exact N = 65536 prec", prec, "lin", lin, "plan", nd.plan_name(prec, plan))
    _, T = nd.dbg_split(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec, lin=lin, lag=False)
    T = T.cpu().numpy()[rows].astype(np.complex128)
    diff = np.argwhere(T != Tref[lin])
    assert diff.size == 0, ("first mismatches (row index, bin)", diff[:8].tolist(),
                            T[tuple(diff[0])] if diff.size else None, Tref[lin][tuple(diff[0])] if diff.size else None)


@pytest.mark.parametrize("prec,plan", all_split_plans())
def test_twiddle_signs_T_exact_every_plan(nd, orc, prec, plan):
    # a wide Doppler window (many crossings per chunk), odd delay offset, ragged tiles
    n, tau0, n_tau, p0, n_dop = 8192, 5, 77, -1000, 2001
    s, r = synth.dyadic_pair(n, 2)
    z, sg = oracle_lag_rows(orc, s, r, np.arange(tau0, tau0 + n_tau))
    Tref = oracle_T(orc, z, sg, n, p0, n_dop)
    nd.set_plan(prec, plan, 0)
    log("T exact N = 8192 plan", nd.plan_name(prec, plan))
    try:
        _, T = nd.dbg_split(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec, lag=False)
    finally:
        nd.set_plan(prec, -1, 0)
    T = T.cpu().numpy().astype(np.complex128)
    diff = np.argwhere(T != Tref)
    assert diff.size == 0, ("first mismatches (delay, bin)", diff[:8].tolist())


# ------------------------------------------------------------------------------------
# the D half: A - T against the twiddles times the exact lag signs
# ------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cfg3_D(orc, cfg3, cfg3_signs):
    c = cfg3
    rng = np.random.default_rng(43)
    rows = np.unique(np.concatenate([[0, 5, 11, 37, 1023], rng.integers(0, c["n_tau"], 27)]))
    D = oracle_D(orc, cfg3_signs[rows], c["n"], c["p0"], c["n_dop"])
    return rows, D


@pytest.mark.parametrize("prec", [1, 2, 0])
def test_D_half_config3(nd, cfg3, cfg3_D, prec):
    c = cfg3
    rows, Dref = cfg3_D
    S, R = dev(c["s"]), dev(c["r"])
    A = nd.caf(S, R, c["tau0"], c["n_tau"], c["p0"], c["n_dop"], prec=prec).cpu().numpy()
    _, T = nd.dbg_split(S, R, c["tau0"], c["n_tau"], c["p0"], c["n_dop"], prec=prec, lag=False)
    T = T.cpu().numpy()
    D = A[rows].astype(np.complex128) - T[rows].astype(np.complex128)
    err = np.abs(D.real - Dref.real) + np.abs(D.imag - Dref.imag)
    log("D half config3 prec", prec, "max |dRe| + |dIm|", float(err.max()))
    assert float(err.max()) < 0.5


# ------------------------------------------------------------------------------------
# impulses: sparse surveillance records, every plan
# ------------------------------------------------------------------------------------
# sample positions at chunk and stage edges and at the quadrant points of low bins
EDGES = (0, 1, 31, 32, 63, 64, 127, 128, 255, 256, 257, 511, 512, 4095, 4096, 8191, 8192, 16383, 16384,
         16385, 32767, 32768, 49152, 65535)


@pytest.fixture(scope="module")
def sparse65536(orc):
    n, tau0, n_tau, p0, n_dop = 65536, 0, 1024, -256, 512
    s, r = synth.sparse_pair(n, 5, 48, EDGES)
    rows = np.array([0, 1, 2, 63, 64, 255, 256, 511, 700, 1000, 1022, 1023])
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    return (s, r, n, tau0, n_tau, p0, n_dop, rows), Ao, sc


@pytest.mark.parametrize("prec,plan", all_split_plans())
def test_impulses_n65536_every_split_plan(nd, sparse65536, prec, plan):
    (s, r, n, tau0, n_tau, p0, n_dop, rows), Ao, sc = sparse65536
    nd.set_plan(prec, plan, 0)
    log("impulses N = 65536 plan", nd.plan_name(prec, plan))
    try:
        A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec).cpu().numpy()
    finally:
        nd.set_plan(prec, -1, 0)
    e = rel_err(A[rows], Ao, sc)
    log("  max l1-relative error", e)
    assert e <= TOL[prec]


@pytest.fixture(scope="module")
def sparse4096(orc):
    n, tau0, n_tau, p0, n_dop = 4096, 0, 256, 0, 4096
    s, r = synth.sparse_pair(n, 6, 48, (0, 1, 255, 256, 1023, 1024, 2048, 3072, 4095))
    rows = np.array([0, 1, 5, 11, 37, 128, 200, 254, 255])
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    return (s, r, n, tau0, n_tau, p0, n_dop, rows), Ao, sc


@pytest.mark.parametrize("prec,plan", all_plans())
def test_impulses_n4096_all_bins_every_plan(nd, sparse4096, prec, plan):
    (s, r, n, tau0, n_tau, p0, n_dop, rows), Ao, sc = sparse4096
    nd.set_plan(prec, plan, 0)
    log("impulses N = 4096 all bins plan", nd.plan_name(prec, plan))
    try:
        A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec).cpu().numpy()
    finally:
        nd.set_plan(prec, -1, 0)
    e = rel_err(A[rows], Ao, sc)
    log("  max l1-relative error", e)
    assert e <= TOL[prec]


# ------------------------------------------------------------------------------------
# rounding of the twiddle-sign half on DC-heavy rows at the largest admitted base
# ------------------------------------------------------------------------------------
def dc_pair(n, seed):
    """Records whose lag products keep one sign and nearly one value along each row (a
    strong constant plus 1% noise per part): the prefix sums the crossing walk reads grow
    linearly along the row while T itself stays small, the hardest case for its rounding."""
    rng = np.random.default_rng(seed)
    s = (1.0 + 0.01 * rng.standard_normal(n)) + 1j * (0.7 + 0.01 * rng.standard_normal(n))
    r = (0.9 + 0.01 * rng.standard_normal(n)) - 1j * (0.6 + 0.01 * rng.standard_normal(n))
    return synth.c64(s), synth.c64(r)


@pytest.fixture(scope="module")
def dc65536(orc):
    # bins -256..255: the largest base 256 has 256 b = N, the limit where the built-in
    # choice still takes the sign-split plans
    n, tau0, n_tau, p0, n_dop = 65536, 0, 64, -256, 512
    s, r = dc_pair(n, 61)
    rows = np.array([0, 1, 17, 40, 63])
    z, sg = oracle_lag_rows(orc, s, r, tau0 + rows)
    T = oracle_T(orc, z, sg, n, p0, n_dop)
    A, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    return (s, r, n, tau0, n_tau, p0, n_dop, rows), T, A, sc


@pytest.fixture(scope="module")
def dc16384(orc):
    # bins -256..255 at N = 16384: 64 b = N, the limit where the built-in choice still takes
    # the FP32 sign-split plan (8 sign changes per part and 256-sample chunk at b = 256)
    n, tau0, n_tau, p0, n_dop = 16384, 0, 128, -256, 512
    s, r = dc_pair(n, 62)
    rows = np.array([0, 1, 33, 90, 127])
    z, sg = oracle_lag_rows(orc, s, r, tau0 + rows)
    T = oracle_T(orc, z, sg, n, p0, n_dop)
    A, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    return (s, r, n, tau0, n_tau, p0, n_dop, rows), T, A, sc


def test_twiddle_sign_half_rounding_dc_rows_fp32_limit(nd, dc16384):
    (s, r, n, tau0, n_tau, p0, n_dop, rows), Tref, Aref, sc = dc16384
    plan, _ = nd.get_plan(0, n, n_tau, p0, n_dop)
    name = nd.plan_name(0, plan)
    assert name.startswith("fp32s_"), name
    _, T = nd.dbg_split(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=0, lag=False)
    eT = rel_err(T.cpu().numpy()[rows], Tref, sc)
    A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=0).cpu().numpy()
    eA = rel_err(A[rows], Aref, sc)
    log("DC rows at the FP32 plan's limit, plan", name, "T half l1-relative error", eT, "whole cell", eA)
    assert eT <= 5e-6
    assert eA <= TOL[0]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_twiddle_sign_half_rounding_dc_rows(nd, dc65536, prec):
    (s, r, n, tau0, n_tau, p0, n_dop, rows), Tref, Aref, sc = dc65536
    plan, _ = nd.get_plan(prec, n, n_tau, p0, n_dop)
    name = nd.plan_name(prec, plan)
    assert name.startswith(SPLIT_PREFIX), name
    _, T = nd.dbg_split(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec, lag=False)
    eT = rel_err(T.cpu().numpy()[rows], Tref, sc)
    A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec).cpu().numpy()
    eA = rel_err(A[rows], Aref, sc)
    log("DC rows, plan", name, "T half l1-relative error", eT, "whole cell", eA)
    # the twiddle-sign half alone within half the FP32 budget; the cell within the form's
    assert eT <= 5e-6
    assert eA <= TOL[prec]
