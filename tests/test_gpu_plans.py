"""Every tile plan of every precision against the FP64 oracle (Eq. (12a)).

The library picks one plan per shape; the autotuner may pick any other, so each plan is
forced here (ndft_set_plan, with split-K counts) over shapes that reach its code paths:
powers of two and odd lengths, N = 2 mod 4, a length whose twiddle table cannot be made
exact at the quadrant points (integer sign path), ragged delay and bin tiles, ragged
sample chunks, exact zeros and lag products whose FP32 value cancels to 0 while the exact
value does not (the exact-sign repair of the register-lag kernels), base sets of one
tile multiple plus base 0 (which those kernels sum on the vector units), and batches.
Tolerance as in test_gpu_parity (l1-relative per output; exact zeros where the scale is 0).
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-4, 2: 1e-4}


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


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0)), "non-zero output where the exact result is 0"
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


def cancel_pair(n, seed):
    """Samples whose lag products often round to 0 in FP32 (exact value +-1/2 or 0):
    s = (2^24, -2^24) with r = (1, 1/2) at lag 0, plus integer and zero samples."""
    rng = np.random.default_rng(seed)
    s = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex64)
    r = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex64)
    big = rng.uniform(size=n) < 0.3
    s[big] = np.complex64(2.0 ** 24 - 2.0 ** 24 * 1j) * rng.choice([1, -1], big.sum())
    r[big] = np.complex64(1.0 + 0.5j)
    return s, r


# n, tau0, n_tau, p0, n_dop, ksplit, data
SHAPES = [
    (4096, 3, 300, -200, 400, 0, "gauss"),     # power of two, ragged tiles
    (999, 0, 130, -50, 101, 3, "gauss"),       # odd length, three chunks
    (1002, 7, 64, 0, 1002, 0, "int_zeros"),    # N = 2 mod 4, all bins
    (65540, 0, 3, -2, 5, 2, "gauss"),          # quadrant points off the table grid
    (1200, 0, 40, -30, 64, 5, "cancel"),       # FP32 cancellation, zeros
    (17, 0, 17, 0, 17, 0, "int_zeros"),        # shorter than one stage
    (4096, 5, 200, -128, 256, 0, "gauss"),     # 129 bases: base 0 apart for 64/128-row tiles
    (1200, 0, 40, -96, 192, 5, "cancel"),      # 97 bases: base 0 apart for 96-row tiles
    (2048, 0, 50, 10, 90, 0, "gauss"),         # no base 0 in the window
    (8192, 2, 70, -33, 66, 3, "int_zeros"),    # sign runs crossing chunk edges, exact zeros
]

_ORACLE = {}


def case(orc, shape):
    if shape not in _ORACLE:
        n, tau0, n_tau, p0, n_dop, _, kind = shape
        if kind == "gauss":
            s, r = synth.random_pair(n, seed=n + 1, zeros=0.02)
        elif kind == "int_zeros":
            s, r = synth.random_pair(n, seed=n + 2, zeros=0.2, integer=True)
        else:
            s, r = cancel_pair(n, n)
        Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop)
        _ORACLE[shape] = (s, r, Ao, sc)
    return _ORACLE[shape]


def plans():
    import paper_1402_0532_amd as m

    try:
        return [(p, k) for p in (0, 1, 2) for k in range(m.plan_count(p))]
    except Exception:  # no library: the module fixture skips
        return [(0, 0)]


@pytest.mark.parametrize("prec,plan", plans())
@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_{s[6]}" for s in SHAPES])
def test_plan_vs_oracle(nd, orc, prec, plan, shape):
    n, tau0, n_tau, p0, n_dop, ks, kind = shape
    s, r, Ao, sc = case(orc, shape)
    nd.set_plan(prec, plan, ks)
    print("plan", nd.plan_name(prec, plan), "shape", shape, flush=True)
    try:
        A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=prec).cpu().numpy()
    finally:
        nd.set_plan(prec, -1, 0)
    assert rel_err(A, Ao, sc) <= TOL[prec]


@pytest.mark.parametrize("prec,plan", [pk for pk in plans() if pk[0] != 2])
def test_plan_batched_vs_oracle(nd, orc, prec, plan):
    shapes = [(1, 0, 1, 0, 1), (999, 2, 90, -5, 11), (4096, 0, 129, 7, 257), (1002, 10, 50, -100, 200),
              (65540, 0, 2, -1, 3)]
    cpis = []
    for k, (n, tau0, n_tau, p0, n_dop) in enumerate(shapes):
        if k == 3:
            s, r = cancel_pair(n, 7)
        else:
            s, r = synth.random_pair(n, seed=400 + k, zeros=0.03)
        cpis.append(dict(s=s, r=r, n=n, tau0=tau0, n_tau=n_tau, p0=p0, n_dop=n_dop))
    surv, ref, descs, olen = nd.pack_batch(cpis)
    nd.set_plan(prec, plan, 0)
    try:
        bp = nd.BatchPlan(descs, prec, chunk=1024)
        print("batched plan", bp.plan_name, flush=True)
        out = torch.empty(olen, dtype=torch.complex64, device="cuda")
        bp.run(dev(surv), dev(ref), out)
        res = out.cpu().numpy()
    finally:
        nd.set_plan(prec, -1, 0)
    for c, d in zip(cpis, descs):
        A = res[d["out_off"]: d["out_off"] + d["n_tau"] * d["n_dop"]].reshape(d["n_tau"], d["n_dop"])
        Ao, sc = orc.caf(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
        assert rel_err(A, Ao, sc) <= TOL[prec], (c["n"], c["tau0"])
