"""GPU adjoint (ndft_caf_backward) against the FP64 oracle gradient and finite differences.

Gradient convention: grad = dL/dRe + j dL/dIm for a real loss L. Derivative rule at every
operator node: d(x (x) y)/dx = sign(y) (almost everywhere). Tolerance metric per element:
(|dRe| + |dIm|) / scale, with scale the l1 mass of the terms that reach the element,
sum over contributing delays and bins of 2(|G_r| + |G_i|). FP32 <= 1e-5, split-BF16 <= 1e-4.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-4}


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_0532_amd as m

    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def grad_scales(G, n, tau0):
    """l1 mass reaching grad_r[m] (delays with m + d < n) and grad_s[i] (i - d >= 0)."""
    n_tau = G.shape[0]
    row = 2 * (np.abs(G.real) + np.abs(G.imag)).sum(axis=1)  # per delay
    sr = np.zeros(n)
    ss = np.zeros(n)
    for l in range(n_tau):
        d = tau0 + l
        sr[: n - d] += row[l]
        ss[d:] += row[l]
    return sr, ss


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0))
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


SHAPES = [(1, 0, 1, 0, 1), (7, 1, 4, -3, 7), (64, 0, 16, -8, 16), (300, 5, 40, -20, 41),
          (1000, 0, 100, 17, 64), (4096, 3, 70, -100, 200)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_backward_matches_oracle_gradient(nd, orc, prec, shape):
    n, tau0, n_tau, p0, n_dop = shape
    s, r = synth.random_pair(n, seed=200 + n, zeros=0.05)
    rng = np.random.default_rng(n)
    G = (rng.standard_normal((n_tau, n_dop)) + 1j * rng.standard_normal((n_tau, n_dop))).astype(np.complex64)
    print("backward", shape, prec, flush=True)
    gr, gs = nd.caf_backward(dev(s), dev(r), tau0, n_tau, p0, n_dop, dev(G), prec=prec)
    gro, gso = orc.caf_grad(s, r, tau0, n_tau, p0, n_dop, G)
    sr, ss = grad_scales(G.astype(np.complex128), n, tau0)
    assert rel_err(gr.cpu().numpy(), gro, sr) <= TOL[prec]
    assert rel_err(gs.cpu().numpy(), gso, ss) <= TOL[prec]


@pytest.fixture(scope="module")
def cfg5(orc):
    c = synth.config5()
    A, _ = orc.caf(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    G = (2.0 * c["w"] * A)
    gro, gso = orc.caf_grad(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"], G)
    return c, A, G, gro, gso


@pytest.mark.parametrize("prec", [0, 1])
def test_config5_gradient_vs_oracle(nd, cfg5, prec):
    c, A, G, gro, gso = cfg5
    args = (c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    s = dev(c["s"]).requires_grad_(True)
    r = dev(c["r"]).requires_grad_(True)
    w = dev(c["w"].astype(np.float32))
    Ag = nd.NDFTCaf.apply(s, r, *args, prec)
    loss = (w * (Ag.real ** 2 + Ag.imag ** 2)).sum()
    loss.backward()
    sr, ss = grad_scales(G, c["n"], c["tau0"])
    er = rel_err(r.grad.cpu().numpy(), gro, sr)
    es = rel_err(s.grad.cpu().numpy(), gso, ss)
    print("config5 gradient l1-relative error prec", prec, "ref", er, "surv", es, flush=True)
    assert er <= TOL[prec] and es <= TOL[prec]


def test_config5_gradient_vs_finite_differences(nd, orc, cfg5):
    # central differences (h = 1e-4, FP64) of the literal loss at every real coordinate of
    # r (2N of them), skipping those whose +-h step can move a lag-product component across
    # zero (the loss jumps there: Eq. (6) applied to the lag product and the twiddle)
    c, A, G, gro, gso = cfg5
    n, h = c["n"], 1e-4
    coords = np.arange(2 * n)
    fd = orc.caf_loss_fd(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"], c["w"], coords, h)
    args = (c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    gr, _ = nd.caf_backward(dev(c["s"]), dev(c["r"]), *args, dev((2.0 * c["w"] * A).astype(np.complex64)),
                            prec=0, need_grad_s=False)
    gr = gr.cpu().numpy().astype(np.complex128)
    ana = np.where(coords % 2 == 0, gr[coords // 2].real, gr[coords // 2].imag)
    # r[m] moves the lag products z_l[m + d] of every delay d; a step of h in one part of
    # r[m] moves each component of s (x) conj(r) by at most h (the operator's slope is +-1
    # in each operand away from 0), so a component within 2h of zero may change sign
    near = np.zeros(n, bool)
    for l in range(c["n_tau"]):
        d = c["tau0"] + l
        z, _ = orc.lag_row(c["s"], c["r"], d)
        zz = z[d:]
        near[: n - d] |= (np.abs(zz.real) <= 2 * h) | (np.abs(zz.imag) <= 2 * h)
    r64 = c["r"].astype(np.complex128)
    near |= (np.abs(r64.real) <= 2 * h) | (np.abs(r64.imag) <= 2 * h)  # an operand crossing 0
    keep = ~near[coords // 2]
    assert keep.mean() >= 0.9, keep.mean()
    sr, _ = grad_scales(G, n, c["tau0"])
    err = np.abs(ana - fd) / sr[coords // 2]
    print("config5 GPU gradient vs FD on %d of %d coordinates, max l1-relative error %.3g"
          % (keep.sum(), 2 * n, float(err[keep].max())), flush=True)
    assert np.all(err[keep] <= 1e-5)


def test_backward_deterministic(nd):
    s, r = synth.random_pair(2048, seed=3)
    G = dev((np.ones((64, 100)) * (1 + 2j)).astype(np.complex64))
    a = nd.caf_backward(dev(s), dev(r), 0, 64, -50, 100, G)
    b = nd.caf_backward(dev(s), dev(r), 0, 64, -50, 100, G)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
