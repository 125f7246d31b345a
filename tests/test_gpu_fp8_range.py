"""The FP8 form's data range: the combined FP8 kernel carries the data as four e4m3 terms
of z 2^-e, with the exponent e taken on the device from the largest |re| + |im| of the
inputs (and carried by the sign operands and the MFMA block scales), so inputs of any
magnitude up to 2^29 keep the form's accuracy, tiny inputs included; beyond, the
surface is NaN. Forward NDFT (Eq. (7)) and wide-window surfaces (Eq. (12a)) against the
FP64 oracle, l1-relative per output <= 1e-4; the batched FP8 kernel on scaled CPIs."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


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


SCALES = [1e-7, 1e-3, 1.0, 300.0, 1e5, 3e7]


@pytest.mark.parametrize("scale", SCALES)
def test_fp8_forward_any_magnitude(nd, orc, scale):
    rng = np.random.default_rng(int(np.log10(scale) + 10))
    x = (scale * (rng.standard_normal((6, 1000)) + 1j * rng.standard_normal((6, 1000)))).astype(np.complex64)
    x[:, ::17] = 0
    print("fp8 forward scale", scale, flush=True)
    X = nd.forward(dev(x), prec=nd.FP8).cpu().numpy()
    Xo, sc = orc.ndft(x.astype(np.complex128))
    assert rel_err(X, Xo, sc) <= TOL


@pytest.mark.parametrize("scale", SCALES)
def test_fp8_wide_window_surface_any_magnitude(nd, orc, scale):
    # all 4096 bins: the built-in FP8 choice is the combined kernel
    n, tau0, n_tau, p0, n_dop = 4096, 0, 40, 0, 4096
    s, r = synth.random_pair(n, seed=int(np.log10(scale) + 30), zeros=0.02)
    s = (s * scale).astype(np.complex64)
    r = (r * np.sqrt(scale)).astype(np.complex64)
    plan, _ = nd.get_plan(nd.FP8, n, n_tau, p0, n_dop)
    print("fp8 surface scale", scale, "plan", nd.plan_name(nd.FP8, plan), flush=True)
    assert not nd.plan_name(nd.FP8, plan).startswith("fp8s_")
    A = nd.caf(dev(s), dev(r), tau0, n_tau, p0, n_dop, prec=nd.FP8).cpu().numpy()
    rows = np.array([0, 1, 20, 39])
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop, rows=rows)
    assert rel_err(A[rows], Ao, sc) <= TOL


def test_fp8_beyond_range_is_nan_not_wrong(nd):
    x = np.full((2, 256), 2.0 ** 30 + 0j, np.complex64)
    X = nd.forward(dev(x), prec=nd.FP8).cpu().numpy()
    assert np.all(np.isnan(X.real) | np.isnan(X.imag))


def test_fp8_batched_scaled_cpis(nd, orc):
    cpis = []
    for k, (n, tau0, n_tau, p0, n_dop, scale) in enumerate(
            [(999, 2, 90, -5, 11, 1e4), (4096, 0, 129, 7, 257, 1e-4), (1002, 10, 50, -100, 200, 1e6)]):
        s, r = synth.random_pair(n, seed=500 + k, zeros=0.03)
        cpis.append(dict(s=(s * scale).astype(np.complex64), r=r, n=n, tau0=tau0, n_tau=n_tau, p0=p0, n_dop=n_dop))
    surv, ref, descs, olen = nd.pack_batch(cpis)
    plan = nd.BatchPlan(descs, prec=nd.FP8)
    out = torch.zeros(olen, dtype=torch.complex64, device="cuda")
    plan.run(dev(surv), dev(ref), out)
    out = out.cpu().numpy()
    for c, d in zip(cpis, descs):
        A = out[d["out_off"]:d["out_off"] + d["n_tau"] * d["n_dop"]].reshape(d["n_tau"], d["n_dop"])
        Ao, sc = orc.caf(c["s"], c["r"], d["tau0"], d["n_tau"], d["p0"], d["n_dop"])
        assert rel_err(A, Ao, sc) <= TOL, d
