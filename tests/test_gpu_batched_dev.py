"""Batched surfaces from device-resident CPI descriptors (ndft_caf_batched_dev): a planning
kernel lays out the workspace on the device, so nothing is prepared on the host.

Checks: every CPI against the FP64 oracle (Eq. (12a); FP32 <= 1e-5, split-BF16 and FP8
<= 1e-4), bit-identical to the host-prepared batch with the same plan and chunk, a
workspace that only fits with a larger chunk (the planner doubles it), the device-side
errors (an invalid descriptor, a workspace too small for one chunk per surface: status
set, outputs untouched), and hipGraph capture with the descriptors changed on the device
between replays (each replay against the eager call and the oracle).
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
    assert not np.any(zero & (err != 0))
    return float(np.max(np.where(zero, 0.0, err / np.where(zero, 1.0, scale)), initial=0.0))


SHAPES = [(1, 0, 1, 0, 1), (37, 2, 9, -5, 11), (300, 0, 129, 7, 257), (1000, 10, 50, -100, 200),
          (4100, 0, 64, -256, 512), (777, 3, 200, 0, 777), (2048, 0, 130, -64, 128), (9000, 5, 40, -600, 1200)]


def batch():
    cpis = []
    for k, (n, tau0, n_tau, p0, n_dop) in enumerate(SHAPES):
        s, r = synth.random_pair(n, seed=700 + k, zeros=0.03 if k % 2 else 0.0, integer=(k == 5))
        cpis.append(dict(s=s, r=r, n=n, tau0=tau0, n_tau=n_tau, p0=p0, n_dop=n_dop))
    return cpis


def split_out(out, descs):
    return [out[d["out_off"]: d["out_off"] + d["n_tau"] * d["n_dop"]].reshape(d["n_tau"], d["n_dop"])
            for d in descs]


def host_ws_bytes(nd, descs, prec):
    from paper_1402_0532_amd import _lib

    arr = (_lib.NdftCpi * len(descs))()
    for k, d in enumerate(descs):
        for f in nd.CPI_FIELDS:
            setattr(arr[k], f, int(d[f]))
    return int(_lib.load().ndft_caf_batched_workspace(arr, len(descs), prec, 0))


def check_vs_oracle(orc, cpis, descs, out, prec):
    for c, d, A in zip(cpis, descs, split_out(out, descs)):
        Ao, sc = orc.caf(c["s"], c["r"], d["tau0"], d["n_tau"], d["p0"], d["n_dop"])
        e = rel_err(A, Ao, sc)
        assert e <= TOL[prec], (d, e)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dev_batch_vs_oracle(nd, orc, prec):
    cpis = batch()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    table = nd.cpi_table(descs)
    ws = torch.empty(host_ws_bytes(nd, descs, prec), dtype=torch.uint8, device="cuda")
    out = torch.full((olen,), float("nan"), dtype=torch.complex64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    print("dev batch prec", prec, "ws", ws.numel(), flush=True)
    nd.caf_batched_dev(dev(surv), dev(ref), out, table, prec=prec, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    check_vs_oracle(orc, cpis, descs, out.cpu().numpy(), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_dev_batch_equals_prepared_batch(nd, prec):
    cpis = batch()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    # the prepared batch with the plan the device form takes (its built-in choice); the
    # workspace bound keeps the device planner at the default chunk
    table = nd.cpi_table(descs)
    ws = torch.empty(nd.caf_batched_dev_workspace_bytes(len(descs), max(d["n"] for d in descs),
                                                        max(d["n_tau"] for d in descs),
                                                        max(d["n_dop"] for d in descs), prec),
                     dtype=torch.uint8, device="cuda")
    a = torch.zeros(olen, dtype=torch.complex64, device="cuda")
    nd.caf_batched_dev(dev(surv), dev(ref), a, table, prec=prec, ws=ws)
    torch.cuda.synchronize()
    hdr_plan = int(ws[12:16].view(torch.int32).item()) - 100 * prec  # plan_id of the header
    nd.set_plan(prec, hdr_plan, 0)
    try:
        plan = nd.BatchPlan(descs, prec)
        assert plan.batch.plan == hdr_plan
        b = torch.zeros(olen, dtype=torch.complex64, device="cuda")
        plan.run(dev(surv), dev(ref), b)
        torch.cuda.synchronize()
    finally:
        nd.set_plan(prec, -1, 0)
    assert torch.equal(a, b)


def host_ws_bytes_plan(nd, descs, prec, plan, chunk):
    from paper_1402_0532_amd import _lib

    nd.set_plan(prec, plan, 0)
    try:
        arr = (_lib.NdftCpi * len(descs))()
        for k, d in enumerate(descs):
            for f in nd.CPI_FIELDS:
                setattr(arr[k], f, int(d[f]))
        return int(_lib.load().ndft_caf_batched_workspace(arr, len(descs), prec, chunk))
    finally:
        nd.set_plan(prec, -1, 0)


def test_dev_batch_small_workspace_doubles_the_chunk(nd, orc):
    cpis = batch()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    S, R = dev(surv), dev(ref)
    out = torch.zeros(olen, dtype=torch.complex64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    big = torch.empty(host_ws_bytes(nd, descs, 0) * 4, dtype=torch.uint8, device="cuda")
    nd.caf_batched_dev(S, R, out, nd.cpi_table(descs), prec=0, ws=big)
    torch.cuda.synchronize()
    plan = int(big[12:16].view(torch.int32).item())  # plan_id of the header (FP32: the plan)
    # the device plan's layout at twice the default chunk: smaller than at the default,
    # so the planner has to double the chunk once to fit
    need2 = host_ws_bytes_plan(nd, descs, 0, plan, 8192)
    need1 = host_ws_bytes_plan(nd, descs, 0, plan, 4096)
    assert need2 < need1
    ws = torch.empty(need2, dtype=torch.uint8, device="cuda")
    out.zero_()
    nd.caf_batched_dev(S, R, out, nd.cpi_table(descs), prec=0, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    check_vs_oracle(orc, cpis, descs, out.cpu().numpy(), 0)


def test_dev_batch_device_side_errors_leave_outputs(nd):
    cpis = batch()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    ws = torch.empty(host_ws_bytes(nd, descs, 1), dtype=torch.uint8, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    sentinel = torch.full((olen,), 7.0 + 3.0j, dtype=torch.complex64, device="cuda")
    bad = [dict(d) for d in descs]
    bad[3]["tau0"] = bad[3]["n"]  # delays past the record
    out = sentinel.clone()
    nd.caf_batched_dev(dev(surv), dev(ref), out, nd.cpi_table(bad), prec=1, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 1  # NDFT_E_INVAL
    assert torch.equal(out, sentinel)
    # the tables fit but not the samples and partial sums, even at one chunk per surface
    from paper_1402_0532_amd import _lib

    tiny = torch.empty(64 << 10, dtype=torch.uint8, device="cuda")
    out = sentinel.clone()
    nd.caf_batched_dev(dev(surv), dev(ref), out, nd.cpi_table(descs), prec=1, ws=tiny, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 3  # NDFT_E_WORKSPACE
    assert torch.equal(out, sentinel)
    # host-side rejections: nothing enqueued
    with pytest.raises(RuntimeError, match="WORKSPACE"):
        nd.caf_batched_dev(dev(surv), dev(ref), out, nd.cpi_table(descs), prec=1,
                           ws=torch.empty(256, dtype=torch.uint8, device="cuda"))
    assert _lib.load().ndft_caf_batched_dev_workspace(0, 100, 10, 10, 0) == 0


def test_dev_batch_graph_replay_with_new_descriptors(nd, orc):
    cpis = batch()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    s_pool, r_pool = dev(surv), dev(ref)
    # a second geometry over the same pools: other delays and Doppler windows, each
    # surface no larger than before (the output layout is kept)
    alt = []
    for d in descs:
        e = dict(d)
        e["tau0"] = 0
        e["p0"] = d["p0"] + 3
        alt.append(e)
    table = nd.cpi_table(descs)
    table_alt = nd.cpi_table(alt)
    max_n = max(d["n"] for d in descs)
    ws_bytes = nd.caf_batched_dev_workspace_bytes(len(descs), max_n, max(d["n_tau"] for d in descs),
                                                  max(d["n_dop"] for d in descs), 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    live = table.clone()  # the descriptor table the graph reads
    out = torch.zeros(olen, dtype=torch.complex64, device="cuda")
    eager = {}
    for key, t in (("a", table), ("b", table_alt)):
        e = torch.zeros(olen, dtype=torch.complex64, device="cuda")
        nd.caf_batched_dev(s_pool, r_pool, e, t, prec=1, ws=ws)
        eager[key] = e
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        nd.caf_batched_dev(s_pool, r_pool, out, live, prec=1, ws=ws)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        nd.caf_batched_dev(s_pool, r_pool, out, live, prec=1, ws=ws)
    for rep, key in enumerate(["a", "b", "b", "a", "b"]):
        live.copy_(table if key == "a" else table_alt)  # descriptors changed on the device
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda") * 2  # unrelated eager work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager[key]), (rep, key)
        del junk
    check_vs_oracle(orc, cpis, alt, eager["b"].cpu().numpy(), 1)
