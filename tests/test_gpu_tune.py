"""The autotuner (tune.autotune_caf, tune.autotune_batch) run end to end on small shapes:
it times every tile plan (and split-K counts or chunk sizes), applies the fastest, and the
surfaces computed with the tuned choice still match the FP64 oracle (Eq. (12a); FP32 <=
1e-5, split-BF16 <= 1e-4). The tuning cache goes to a temporary file."""
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


@pytest.fixture(autouse=True)
def tune_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("NDFT_TUNE_CACHE", str(tmp_path / "tune.json"))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(got, ref, scale):
    got = np.asarray(got, np.complex128)
    err = np.abs(got.real - ref.real) + np.abs(got.imag - ref.imag)
    zero = scale == 0
    assert not np.any(zero & (err != 0))
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_autotune_caf_then_oracle(nd, orc, prec):
    from paper_1402_0532_amd import tune

    n, tau0, n_tau, p0, n_dop = 4096, 3, 150, -64, 128
    s, r = synth.random_pair(n, seed=81, zeros=0.02)
    S, R = dev(s), dev(r)
    try:
        best = tune.autotune_caf(S, R, tau0, n_tau, p0, n_dop, prec=prec, reps=2, use_cache=False)
        print("autotune_caf prec", prec, best, flush=True)
        assert best["tried"] >= 2 and best["name"] == nd.plan_name(prec, best["plan"])
        plan, ks = nd.get_plan(prec, n, n_tau, p0, n_dop)
        assert plan == best["plan"]
        A = nd.caf(S, R, tau0, n_tau, p0, n_dop, prec=prec).cpu().numpy()
        # a second call takes the stored choice from the cache
        again = tune.autotune_caf(S, R, tau0, n_tau, p0, n_dop, prec=prec, reps=2, use_cache=True)
        assert again["plan"] == best["plan"]
    finally:
        tune.reset(prec)
    Ao, sc = orc.caf(s, r, tau0, n_tau, p0, n_dop)
    assert rel_err(A, Ao, sc) <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_batch_then_oracle(nd, orc, prec):
    from paper_1402_0532_amd import tune

    shapes = [(999, 2, 90, -5, 11), (4096, 0, 129, 7, 257), (1002, 10, 50, -100, 200), (3000, 0, 64, -32, 64)]
    cpis = []
    for k, (n, tau0, n_tau, p0, n_dop) in enumerate(shapes):
        s, r = synth.random_pair(n, seed=90 + k, zeros=0.03)
        cpis.append(dict(s=s, r=r, n=n, tau0=tau0, n_tau=n_tau, p0=p0, n_dop=n_dop))
    surv, ref, descs, olen = nd.pack_batch(cpis)
    Sp, Rp = dev(surv), dev(ref)
    out = torch.zeros(olen, dtype=torch.complex64, device="cuda")
    try:
        bp, rec = tune.autotune_batch(descs, Sp, Rp, out, prec=prec, reps=1, chunks=(1024, 4096))
        print("autotune_batch prec", prec, rec, flush=True)
        assert rec["tried"] >= 2 and bp.batch.plan == rec["plan"]
        out.zero_()
        bp.run(Sp, Rp, out)
        torch.cuda.synchronize()
    finally:
        tune.reset(prec)
    got = out.cpu().numpy()
    for c, d in zip(cpis, descs):
        A = got[d["out_off"]:d["out_off"] + d["n_tau"] * d["n_dop"]].reshape(d["n_tau"], d["n_dop"])
        Ao, sc = orc.caf(c["s"], c["r"], d["tau0"], d["n_tau"], d["p0"], d["n_dop"])
        assert rel_err(A, Ao, sc) <= TOL[prec], d
