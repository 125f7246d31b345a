"""Benchmark: NDFT cross-ambiguity surface cells/s on one MI355X.

Workload (the N = 65536 radar CPI): surveillance/reference of 65536 complex64 samples
(low-pass Gaussian reference, one target at delay 37 / Doppler 12 bins at -10 dB, clutter
at delays 0/5/11, -20 dB noise), delays 0..1023, Doppler bins -256..255:
1024 x 512 = 524288 surface cells per step. A step is one ndft_caf call (contraction +
ordered split-K reduction) with inputs already resident in HBM.

Prints ONE JSON line. `value` is cells/s of the reported form (default: split-BF16);
`forms` gives every form with its speed-up over the plain FP32 path (the FP32 sign-split
contraction on the FP32 matrix cores, its fastest tile plan) and over the FP32 form with
the twiddle half as an FFT; `roofline` is for the dominant kernel: the contraction
(algorithmic flops 16 N per cell) or, for the sign-split plans, the matrix kernel of the
twiddle x lag-sign half (8 N per cell), over its event-timed duration; for the FFT form the
timed kernel's own bound (vector-unit flops of the decimated FFT) is given under `forms`;
`cpu_baseline` times the FP64 oracle on a bounded sample of the same surface's rows.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16x2": 2500.0, "fp8": 5000.0}  # dense MFMA peaks, MI355X
# Vector-unit peaks from the unit counts and the clock: 256 CUs x 4 SIMDs x 16 lanes at
# 2.4 GHz issue 39.3 T lane operations/s; an FP32 FMA is 2 flops, so 78.6 TFLOP/s for
# unpacked FP32 (the library is built without packed FP32 instructions; the published
# 157.3 TFLOP/s counts packed FMAs).
VALU_LANE_TOPS = 39.3216
VALU_FP32_TFLOPS = 2.0 * VALU_LANE_TOPS
# every source of the library: a recorded figure is tied to the exact build it came from
KERNEL_SOURCES = sorted("paper_1402_0532_amd/csrc/" + f for f in os.listdir(os.path.join(ROOT, "paper_1402_0532_amd", "csrc"))
                        if f.endswith((".hip", ".hpp")))
TRAFFIC_FILE = "profiles/contract_traffic_caf_n65536.txt"
SPLIT_PLAN_PREFIXES = ("bf16x2s_", "bf16x2g_", "fp8s_", "fp32s_")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(form: str, half: str = "d_half"):
    """HBM bytes per contraction launch measured with rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, calibrated on a copy kernel), if recorded for the current kernel source."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    key = "traffic_bytes_per_launch_" + form + ("_t_half" if half == "t_half" else "")
    return float(rec[key]) if key in rec else None


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def fft_flops_per_row(n: int, n_dop: int) -> float:
    """Vector-unit flops of the decimated DFT of one length-n row at n_dop bins: n = M L
    with L the largest power of two dividing n (at most 512): M complex FFTs of length L
    (5 L log2 L flops each, the usual radix-2 count) and M complex multiply-adds (8 flops)
    per requested bin."""
    L = 1
    while L < 512 and n % (2 * L) == 0:
        L *= 2
    M = n // L
    return 5.0 * L * math.log2(L) * M + 8.0 * M * n_dop if L > 1 else 8.0 * n * n_dop


def fast_flops_per_row(n: int) -> float:
    """Flops of the fast exact transform of one length-n row (n a power of two, every bin):
    per correlation length L = 2^l >= 64 its lg - l + 1 pairs of two length-L/4 sequences,
    each transformed forward and back (5 Q log2 Q flops a complex FFT) and multiplied by the
    spectra (two complex products and a sum: 14 flops an entry); the direct correlations of
    lengths 2 .. 32 (8 flops a term); the FFT of the signs (5 n log2 n); the folds and the
    sums into T (2 flops an entry and level)."""
    lg = int(round(math.log2(n)))
    f = 5.0 * n * lg + 2.0 * n * lg * 2
    for l in range(1, lg + 1):
        b, half = lg - l + 1, 2 ** (l - 1)
        if l <= 5:
            f += 8.0 * b * half * half
        else:
            q = half // 2
            f += 2 * (2 * b) * 5.0 * q * math.log2(q) + 14.0 * b * half
    return f


def tsum_ops(n: int, n_tau: int, p0: int, n_dop: int) -> float:
    """Operations of the twiddle-sign half (lsum_kernel) for one surface: per delay and
    sample the Eq. (6) lag product at the paper's count for one complex operator (4 sign,
    8 abs, 6 add: 18) and 2 adds of the prefix sums; per delay, base b and part (real,
    imaginary) 2 b sign changes of csgn(W^{bk}) over the n samples, each a +-2 P term
    (2 ops: real and imaginary)."""
    bases = {min((p0 + q) % n, n - (p0 + q) % n) for q in range(n_dop)}
    crossings = sum(4 * b for b in bases)  # both parts
    return float(n_tau) * (20.0 * n + 2.0 * crossings)


def time_caf(nd, torch, s, r, geo, prec, steps, warmup, event_kernel=True):
    """(ms per call, event-timed main-kernel ms per launch) of ndft_caf on one stream."""
    n, tau0, n_tau, p0, n_dop = geo
    ws = torch.empty(max(1, nd.caf_workspace_bytes(n, tau0, n_tau, p0, n_dop, prec)), dtype=torch.uint8,
                     device=s.device)
    out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device)
    for _ in range(warmup):
        nd.caf(s, r, tau0, n_tau, p0, n_dop, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    nd.prof_read()
    nd.prof_read(1)
    nd.prof_enable(event_kernel)
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(steps):
        nd.caf(s, r, tau0, n_tau, p0, n_dop, prec, out=out, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    nd.prof_enable(False)
    k_ms, k_cnt = nd.prof_read()
    nd.prof_read(1)
    return e0.elapsed_time(e1) / steps, (k_ms / k_cnt if k_cnt else None), out


def bench_batched(nd, tune, synth, torch, args):
    """64 CPIs of uneven length in one persistent launch, replayed from a hipGraph."""
    import numpy as np

    cpis = synth.config4()
    surv, ref, descs, olen = nd.pack_batch(cpis)
    cells = sum(c["n_tau"] * c["n_dop"] for c in cpis)
    flops = sum(16.0 * c["n"] * c["n_tau"] * c["n_dop"] for c in cpis)
    s_pool = torch.from_numpy(surv).cuda()
    r_pool = torch.from_numpy(ref).cuda()
    out = torch.empty(olen, dtype=torch.complex64, device="cuda")
    res = {"workload": "64 CPIs, N log-uniform in [1024, 32768], 128-512 delays, Doppler +-N/16",
           "cells": cells, "algorithmic_flops": flops}
    for form in ("fp32", "bf16x2"):
        prec = nd.PRECISIONS[form]
        if not args.no_batch_autotune:
            bp, rec = tune.autotune_batch(descs, s_pool, r_pool, out, prec)
        else:
            bp, rec = nd.BatchPlan(descs, prec), None
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            bp.run(s_pool, r_pool, out)
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=st):
            bp.run(s_pool, r_pool, out)
        g.replay()
        torch.cuda.synchronize()
        reps = max(3, args.steps // 4)
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[form] = {"ms_per_batch": ms, "cells_per_s": cells / (ms * 1e-3),
                     "algorithmic_tflops": flops / (ms * 1e-3) / 1e12, "plan": bp.plan_name,
                     "items": int(bp.batch.n_items),
                     "autotune": rec}
        del g, bp
    res["speedup_bf16x2_vs_fp32"] = res["fp32"]["ms_per_batch"] / res["bf16x2"]["ms_per_batch"]
    tune.reset()
    # the same batch with the CPI descriptors in device memory (no host preparation), its
    # planning kernel inside the replayed graph
    from paper_1402_0532_amd import _lib

    lib = _lib.load()
    arr = (_lib.NdftCpi * len(descs))()
    for k, d in enumerate(descs):
        for f in nd.CPI_FIELDS:
            setattr(arr[k], f, int(d[f]))
    table = nd.cpi_table(descs)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    res["device_descriptors"] = {}
    for form in ("fp32", "bf16x2"):
        prec = nd.PRECISIONS[form]
        # a workspace that fits the layout of any plan at the default chunk
        need = 0
        for p in range(nd.plan_count(prec)):
            nd.set_plan(prec, p, 0)
            need = max(need, int(lib.ndft_caf_batched_workspace(arr, len(descs), prec, 0)))
        nd.set_plan(prec, -1, 0)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        run = lambda: nd.caf_batched_dev(s_pool, r_pool, out, table, prec=prec, ws=ws)
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            run()
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=st):
            run()
        g.replay()
        torch.cuda.synchronize()
        reps = max(3, args.steps // 4)
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        lib.ndft_caf_batched_dev_status(nd._ptr(ws), nd._ptr(status), nd._stream_handle())
        torch.cuda.synchronize()
        plan_id = int(ws[12:16].view(torch.int32).item())
        res["device_descriptors"][form] = {
            "ms_per_batch": ms, "cells_per_s": cells / (ms * 1e-3), "algorithmic_tflops": flops / (ms * 1e-3) / 1e12,
            "plan": nd.plan_name(prec, plan_id - 100 * prec), "status": int(status.item())}
        del g, ws
    return res


def bench_config2(nd, synth, torch, args):
    """The plain-FP32 workload of the radar model at N = 4096: 256 delays x all 4096 Doppler
    bins (1048576 cells). Every base bin up to N / 2 is needed, so the library takes its
    wide-window kernels (in FP32 the fast exact transform, N being a power of two); each
    form's main kernel is event-timed against its dense peak (16 N algorithmic flops per
    cell; 8 N for a sign-split matrix half), the fast transform against the vector units'
    FP32 peak with its own flop count."""
    import numpy as np

    c = synth.config2()
    geo = (c["n"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    cells = c["n_tau"] * c["n_dop"]
    flops = 16.0 * c["n"] * cells
    s = torch.from_numpy(c["s"]).cuda()
    r = torch.from_numpy(c["r"]).cuda()
    rows = np.array([0, 5, 11, 37, 255])
    ref = None
    if not args.no_cpu_baseline:
        import oracle

        ref = oracle.caf(c["s"], c["r"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"], rows=rows)
    res = {"workload": "caf_n4096_tau256_dop4096", "cells": cells, "algorithmic_flops": flops}
    for form in ("fp32", "bf16x2", "fp8"):
        prec = nd.PRECISIONS[form]
        ms, kern, out = time_caf(nd, torch, s, r, geo, prec, max(5, args.steps), max(3, args.warmup // 10))
        plan, ks = nd.get_plan(prec, c["n"], c["n_tau"], c["p0"], c["n_dop"])
        pname = nd.plan_name(prec, plan)
        if pname.startswith("fp32x_fast"):
            # the fast exact transform: its own flops against the vector units' FP32 peak
            kflops, peak, bound = fast_flops_per_row(c["n"]) * c["n_tau"], VALU_FP32_TFLOPS, "alu"
        else:
            kflops = flops / 2 if pname.startswith(SPLIT_PLAN_PREFIXES) else flops
            peak, bound = PEAK_TFLOPS[form], "mfma"
        tf = kflops / (kern * 1e-3) / 1e12
        res[form] = {"ms_per_surface": ms, "cells_per_s": cells / (ms * 1e-3), "plan": pname, "ksplit": ks,
                     "main_kernel_ms": kern, "main_kernel_tflops": tf, "bound": bound,
                     "frac_of_peak": tf / peak,
                     "algorithmic_tflops_whole_call": flops / (ms * 1e-3) / 1e12}
        if ref is not None:
            g = out.cpu().numpy()[rows].astype(np.complex128)
            Ao, sc = ref
            err = (np.abs(g.real - Ao.real) + np.abs(g.imag - Ao.imag)) / np.where(sc > 0, sc, 1)
            res[form]["max_l1_rel_err_vs_oracle"] = float(err.max())
            res[form]["err_rows_checked"] = int(len(rows))
    for form in ("bf16x2", "fp8"):
        res[form]["speedup_vs_fp32"] = res["fp32"]["ms_per_surface"] / res[form]["ms_per_surface"]
    return res


def bench_adjoint(nd, synth, torch, args):
    """Hand adjoint of the N=8192, 256 x 256 surface (loss sum w |A|^2)."""
    c = synth.config5()
    s = torch.from_numpy(c["s"]).cuda()
    r = torch.from_numpy(c["r"]).cuda()
    w = torch.from_numpy(c["w"].astype("float32")).cuda()
    a = (c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    n, cells = c["n"], c["n_tau"] * c["n_dop"]
    fwd_flops = 16.0 * n * cells  # N complex operator products per cell
    bwd_flops = 8.0 * n * cells   # the adjoint contraction gz = S^H G (ternary S)
    res = {"workload": "N=8192, 256 delays x 256 Doppler bins, loss sum w|A|^2",
           "forward_algorithmic_flops": fwd_flops, "backward_contraction_flops": bwd_flops}
    for form in ("fp32", "bf16x2"):
        prec = nd.PRECISIONS[form]
        A = nd.caf(s, r, *a, prec)
        G = (2.0 * w * A).contiguous()
        nd.caf_backward(s, r, *a, G, prec)
        torch.cuda.synchronize()
        reps = max(5, args.steps)
        nd.prof_read()
        nd.prof_read(1)
        nd.prof_enable(True)
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(reps):
            nd.caf_backward(s, r, *a, G, prec)
        e1.record()
        torch.cuda.synchronize()
        nd.prof_enable(False)
        kb_ms, kb_n = nd.prof_read()
        nd.prof_read(1)
        ms_b = e0.elapsed_time(e1) / reps
        ms_f, kf_ms, _ = time_caf(nd, torch, s, r, (n,) + a, prec, reps, 3)
        kb = kb_ms / max(kb_n, 1)
        plan, _ = nd.get_plan(prec, n, c["n_tau"], c["p0"], c["n_dop"])
        pname = nd.plan_name(prec, plan)
        if pname.startswith("fp32s_"):
            # the FP32 sign-split plan: its timed kernel is the FFT of the twiddle half, priced
            # by the FFT's flops against the vector units (the dense count does not apply)
            kf_flops, kf_peak = fft_flops_per_row(n, c["n_dop"]) * c["n_tau"], VALU_FP32_TFLOPS
        else:
            kf_flops = fwd_flops / 2 if pname.startswith(SPLIT_PLAN_PREFIXES) else fwd_flops
            kf_peak = PEAK_TFLOPS[form]
        res[form] = {"backward_ms": ms_b, "forward_ms": ms_f, "forward_plan": pname,
                     "forward_main_kernel_ms": kf_ms,
                     "forward_frac_of_peak": kf_flops / (kf_ms * 1e-3) / 1e12 / kf_peak,
                     "forward_algorithmic_tflops_whole_call": fwd_flops / (ms_f * 1e-3) / 1e12,
                     "backward_contraction_kernel_ms": kb,
                     "backward_contraction_frac_of_peak": bwd_flops / (kb * 1e-3) / 1e12 / PEAK_TFLOPS[form],
                     "backward_whole_call_frac_of_peak": bwd_flops / (ms_b * 1e-3) / 1e12 / PEAK_TFLOPS[form]}
    res["speedup_bf16x2_vs_fp32_backward"] = res["fp32"]["backward_ms"] / res["bf16x2"]["backward_ms"]
    return res


def bench_other_surfaces(nd, synth, torch, args):
    """The Eq. (12b) surface (Eq. (6) lag product, then the ordinary DFT: decimated FFTs,
    FP32) and the Eq. (12c) surface (ordinary lag product, then the Eq. (6) operator:
    the sign-split kernels) on the same N=65536 workload."""
    import numpy as np

    c = synth.config3()
    a = (c["tau0"], c["n_tau"], c["p0"], c["n_dop"])
    s = torch.from_numpy(c["s"]).cuda()
    r = torch.from_numpy(c["r"]).cuda()
    cells = c["n_tau"] * c["n_dop"]
    rows = np.array([0, 37, 511, 1023])
    out_all = {}
    for eq, fn, wsfn, forms in (("caf12b", nd.caf12b, nd.caf12b_workspace_bytes, ("fp32",)),
                                ("caf12c", nd.caf12c, nd.caf12c_workspace_bytes, ("fp32", "bf16x2", "fp8"))):
        res = {"workload": "%s_n65536_tau1024_dop512" % eq}
        ref = None
        if not args.no_cpu_baseline:
            import oracle

            ref = getattr(oracle, eq)(c["s"], c["r"], *a, rows=rows)
        for form in forms:
            prec = nd.PRECISIONS[form]
            ws = torch.empty(max(1, wsfn(c["n"], *a, prec)), dtype=torch.uint8, device="cuda")
            out = torch.empty((c["n_tau"], c["n_dop"]), dtype=torch.complex64, device="cuda")
            for _ in range(args.warmup):
                fn(s, r, *a, prec, out=out, ws=ws)
            torch.cuda.synchronize()
            reps = max(5, args.steps)
            e0, e1 = _events(torch)
            e0.record()
            for _ in range(reps):
                fn(s, r, *a, prec, out=out, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[form] = {"ms_per_surface": ms, "cells_per_s": cells / (ms * 1e-3)}
            if ref is not None:
                g = out.cpu().numpy()[rows].astype(np.complex128)
                Ao, sc = ref
                err = (np.abs(g.real - Ao.real) + np.abs(g.imag - Ao.imag)) / np.where(sc > 0, sc, 1)
                res[form]["max_l1_rel_err_vs_oracle"] = float(err.max())
                res[form]["err_rows_checked"] = int(len(rows))
            del ws
        out_all[eq] = res
    return out_all


def bench_nfft(nd, torch, args):
    """Batched NFFT (Section 3), both readings of Eq. (10): 32 Mi points as 4096 rows of
    N = 8192 (one row per work-group), as 131072 rows of N = 256 (32 rows per work-group),
    and as 32 rows of N = 2^20 (the top levels over global memory)."""
    res = {}
    lib = nd._lib.load()
    for rows, n in ((4096, 8192), (131072, 256), (32, 1 << 20)):
        g = torch.Generator(device="cuda").manual_seed(5)
        x = torch.complex(torch.randn(rows, n, device="cuda", generator=g),
                          torch.randn(rows, n, device="cuda", generator=g))
        out = torch.empty_like(x)
        wsb = int(lib.ndft_nfft_workspace(rows, n))
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
        for reading, name in ((0, "every_butterfly"), (1, "printed")):
            run = lambda: nd._lib.check(lib.ndft_nfft(nd._ptr(x), nd._ptr(out), rows, n, reading,
                                                      nd._ptr(ws) if wsb else None, wsb, nd._stream_handle()))
            for _ in range(max(3, args.warmup // 10)):
                run()
            torch.cuda.synchronize()
            reps = max(5, args.steps)
            e0, e1 = _events(torch)
            e0.record()
            for _ in range(reps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            # read the rows, write the transforms (complex64); long rows: each top level
            # reads and writes the rows once more
            levels = max(0, int(math.log2(n)) - 13)
            hbm = 16.0 * rows * n * (1 + levels)
            res["%d x N=%d %s" % (rows, n, name)] = {
                "ms": ms, "transforms_per_s": rows / (ms * 1e-3), "hbm_gb_per_s": hbm / (ms * 1e-3) / 1e9,
                "hbm_frac_of_8tbs": hbm / (ms * 1e-3) / 8e12}
        del x, out, ws
    return res


def bench_forward(nd, torch, args):
    """The NDFT of Eq. (7) on a batch (1024 rows of N = 4096, every bin) in FP32: the
    built-in choice (the fast exact transform) against the FP32 contraction forced through
    the plan table, and both against the oracle on two rows."""
    import numpy as np

    rows, n = 1024, 4096
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.complex(torch.randn(rows, n, device="cuda", generator=g),
                      torch.randn(rows, n, device="cuda", generator=g))
    res = {"workload": "forward_b1024_n4096_all_bins", "outputs": rows * n,
           "algorithmic_flops": 16.0 * n * rows * n}
    names = [nd.plan_name(0, k) for k in range(nd.plan_count(0))]
    pick = [0, rows - 1]
    ref = None
    if not args.no_cpu_baseline:
        import oracle

        ref = oracle.ndft(x[pick].cpu().numpy().astype(np.complex128))
    for label, plan in (("fast", -1), ("contraction", names.index("fp32_b96_l128_w12_ks8"))):
        nd.set_plan(0, plan, 0)
        try:
            out = nd.forward(x, prec=0)
            for _ in range(max(3, args.warmup // 10)):
                out = nd.forward(x, prec=0)
            torch.cuda.synchronize()
            reps = max(5, args.steps) if label == "fast" else 3
            e0, e1 = _events(torch)
            e0.record()
            for _ in range(reps):
                out = nd.forward(x, prec=0)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            p, _ = nd.get_plan(0, n, rows, 0, n)
            res[label] = {"ms": ms, "outputs_per_s": rows * n / (ms * 1e-3), "plan": nd.plan_name(0, p)}
            if ref is not None:
                got = out[pick].cpu().numpy().astype(np.complex128)
                Xo, sc = ref
                err = (np.abs(got.real - Xo.real) + np.abs(got.imag - Xo.imag)) / np.where(sc > 0, sc, 1)
                res[label]["max_l1_rel_err_vs_oracle"] = float(err.max())
        finally:
            nd.set_plan(0, -1, 0)
    res["fast"]["flops_own"] = fast_flops_per_row(n) * rows
    res["fast"]["frac_of_fp32_vector_peak"] = res["fast"]["flops_own"] / (res["fast"]["ms"] * 1e-3) / 1e12 / VALU_FP32_TFLOPS
    res["speedup_fast_vs_contraction"] = res["contraction"]["ms"] / res["fast"]["ms"]
    return res


def bench_robustness(nd, synth, torch, args):
    """Targets and clutter under AWGN and eps-contaminated Gaussian noise (noise-free
    reference): the Eq. (12a) and (12b) surfaces (this library) against the ordinary
    cross-ambiguity function of Eq. (11) (numpy FFT of the lag products, comparison only),
    scored by synth.object_margin (side-lobe floor beyond +-3 cells of every object)."""
    import numpy as np

    n, tau0, n_tau, p0, n_dop = synth.ROBUST_WINDOW
    res = {"workload": "N=%d, delays %d..%d, Doppler bins %d..%d; objects per scene; margin_db = "
                       "20 log10(max off-object |A| / weakest object |A|), guard +-3 cells"
                       % (n, tau0, tau0 + n_tau - 1, p0, p0 + n_dop - 1)}
    bins = (p0 + np.arange(n_dop)) % n
    for scene in synth.ROBUST_SCENES:
        objs = synth.scene_objects(scene, p0)
        res[scene] = {}
        for noise in synth.ROBUST_NOISES:
            s, r = synth.robustness_pair(scene, noise, n)
            S, R = torch.from_numpy(s).cuda(), torch.from_numpy(r).cuda()
            lin = np.empty((n_tau, n_dop), np.complex128)
            s64, r64 = s.astype(np.complex128), r.astype(np.complex128)
            for j in range(n_tau):
                l = tau0 + j
                rs = np.concatenate([np.zeros(l), r64[:n - l]])
                lin[j] = np.fft.fft(s64 * np.conj(rs))[bins]
            surfaces = {
                "eq12a_bf16x2": nd.caf(S, R, tau0, n_tau, p0, n_dop, nd.BF16X2).cpu().numpy(),
                "eq12b_fp32": nd.caf12b(S, R, tau0, n_tau, p0, n_dop).cpu().numpy(),
                "eq11_linear": lin,
            }
            res[scene][noise] = {}
            for k, v in surfaces.items():
                m = synth.object_margin(v, objs)
                res[scene][noise][k] = {"detected": m["detected"], "objects": m["objects"],
                                        "margin_db": round(m["margin_db"], 3)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=100)  # clocks settle after ~100 calls
    ap.add_argument("--form", default="fp32", choices=["fp32", "bf16x2", "fp8"],
                    help="the reported form (default: FP32, the fastest and most accurate)")
    ap.add_argument("--forms", default="fp32,bf16x2,fp8", help="forms to time (comma list)")
    ap.add_argument("--autotune", action="store_true",
                    help="time every plan and split of the single-surface forms first and use the fastest "
                         "(default: the library's built-in choice, the plan a caller gets without tuning)")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="batched section: the built-in plan instead of the autotuned one")
    ap.add_argument("--plan", action="append", default=[], metavar="FORM=NAME:KSPLIT",
                    help="force a tile plan and split count for a form (no autotuning for it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every extra section (same as --extras '')")
    ap.add_argument("--extras", default="config2,forward,batched,adjoint,surfaces,robustness,nfft",
                    help="extra sections to run (comma list of config2, forward, batched, adjoint, "
                         "surfaces, robustness, nfft)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size per step (a known-size "
                         "kernel for calibrating HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported "
              "(the surface would shard by delay rows, see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1402_0532_amd as nd
    import synth
    from paper_1402_0532_amd import tune

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c = synth.config3()
    n, tau0, n_tau, p0, n_dop = c["n"], c["tau0"], c["n_tau"], c["p0"], c["n_dop"]
    cells = n_tau * n_dop
    flops_per_call = 16.0 * n * cells
    s = torch.from_numpy(c["s"]).to(dev)
    r = torch.from_numpy(c["r"]).to(dev)

    # the reported form is timed last: the others warm the clocks up before it
    forms = [f for f in args.forms.split(",") if f and f != args.form] + [args.form]
    results = {}
    outs = {}
    tuned = {}
    forced = {}
    for spec in args.plan:
        form, rest = spec.split("=", 1)
        name, ks = rest.split(":")
        forced[form] = (name, int(ks))
    for form in forms:
        prec = nd.PRECISIONS[form]
        if form in forced:
            name, ks = forced[form]
            idx = [k for k in range(nd.plan_count(prec)) if nd.plan_name(prec, k) == name]
            if not idx:
                sys.exit("bench.py: no plan %r for form %s" % (name, form))
            nd.set_plan(prec, idx[0], ks)
        elif args.autotune:
            tuned[form] = tune.autotune_caf(s, r, tau0, n_tau, p0, n_dop, prec, use_cache=False)
        ws = torch.empty(nd.caf_workspace_bytes(n, tau0, n_tau, p0, n_dop, prec),
                         dtype=torch.uint8, device=dev)
        out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=dev)
        for _ in range(args.warmup):
            nd.caf(s, r, tau0, n_tau, p0, n_dop, prec, out=out, ws=ws)
        torch.cuda.synchronize()
        # the timed steps: nothing but the calls
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(args.steps):
            nd.caf(s, r, tau0, n_tau, p0, n_dop, prec, out=out, ws=ws)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1) / args.steps
        # the same steps again with the library's kernel events on (each call then records
        # two event pairs on its stream, which costs the call a few microseconds): the
        # duration of each half's kernel
        nd.prof_read()  # drop anything recorded before
        nd.prof_read(1)
        nd.prof_enable(True)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev3 = torch.cuda.Event(enable_timing=True)
        ev2.record()
        for _ in range(args.steps):
            nd.caf(s, r, tau0, n_tau, p0, n_dop, prec, out=out, ws=ws)
        ev3.record()
        if args.calib_copy_mib:
            src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
            dst = torch.empty_like(src)
            for _ in range(args.steps):
                dst.copy_(src)
            del src, dst
        torch.cuda.synchronize()
        nd.prof_enable(False)
        k_ms, k_cnt = nd.prof_read()
        t_ms, t_cnt = nd.prof_read(1)
        ms_instr = ev2.elapsed_time(ev3) / args.steps
        kern_ms = k_ms / max(k_cnt, 1)
        tsum_ms = t_ms / t_cnt if t_cnt else None
        plan, ks = nd.get_plan(prec, n, n_tau, p0, n_dop)
        pname = nd.plan_name(prec, plan)
        # sign-split plans: the D half (twiddle x lag signs) is dsum_kernel on the matrix
        # cores (8 N flops per cell), or for the FP32 plan a decimated FFT of the exact lag
        # signs (dft512_kernel: the FFT's flops on the vector units); the T half (twiddle
        # signs x lag values) is lsum_kernel on the vector units. The roofline is the half
        # whose kernel takes longer.
        split = pname.startswith(SPLIT_PLAN_PREFIXES)
        fft = pname.startswith("fp32s_")
        if fft:
            kernel_flops = fft_flops_per_row(n, n_dop) * n_tau
            bound, peak, unit, kname = "alu", VALU_FP32_TFLOPS, "TFLOP/s", (
                "dft512_kernel (twiddle half as a decimated FFT of the exact lag signs; 5 L log2 L flops per "
                "length-L FFT plus 8 flops per phase term and bin; unpacked FP32 FMA peak)")
        else:
            kernel_flops = flops_per_call / 2 if split else flops_per_call
            bound, peak, unit = "mfma", PEAK_TFLOPS[form], "TFLOP/s"
            kname = "dsum_kernel (8 N flops per cell)" if split else "contraction (16 N flops per cell)"
        achieved = kernel_flops / (kern_ms * 1e-3) / 1e12
        kernels = {"d_half": {"kernel": kname, "ms": kern_ms, "bound": bound, "achieved": achieved,
                              "peak": peak, "unit": unit, "frac": achieved / peak}}
        if split and tsum_ms:
            t_achieved = tsum_ops(n, n_tau, p0, n_dop) / (tsum_ms * 1e-3) / 1e12
            kernels["t_half"] = {
                "kernel": "lsum_kernel (twiddle-sign half: 18 ops per Eq. (6) lag product, 2 prefix adds per "
                          "sample, 2 ops per sign change of csgn(W^{bk}); vector-lane operation peak)",
                "ms": tsum_ms, "bound": "alu", "achieved": t_achieved, "peak": VALU_LANE_TOPS,
                "unit": "Top/s", "frac": t_achieved / VALU_LANE_TOPS}
        dom = max(kernels, key=lambda k: kernels[k]["ms"])  # the kernel that takes longest
        results[form] = {
            "cells_per_s": cells / (ms * 1e-3),
            "ms_per_step": ms,
            "wall_ms_per_step": wall * 1e3 / args.steps,
            "ms_per_step_with_kernel_events": ms_instr,
            "timed_kernel_ms": kernels[dom]["ms"],
            "timed_kernel_tflops": kernels[dom]["achieved"],
            "bound": kernels[dom]["bound"],
            "peak_tflops": kernels[dom]["peak"],
            "unit": kernels[dom]["unit"],
            "frac_of_peak": kernels[dom]["frac"],
            "plan": pname,
            "ksplit": ks,
            "timed_kernel": kernels[dom]["kernel"],
            "dominant": dom,
            "kernels": kernels,
            "algorithmic_tflops_whole_call": flops_per_call / (ms * 1e-3) / 1e12,
        }
        if form in tuned:
            results[form]["autotune"] = {k: tuned[form][k] for k in ("name", "ksplit", "ms", "tried")}
        outs[form] = out.cpu().numpy()
        del ws

    # the plain FP32 path: the same sign-split contraction on FP32 operands and the FP32
    # matrix cores, its fastest tile plan (every contraction plan timed)
    plain = None
    if "fp32" in forms:
        cands = []
        for k in range(nd.plan_count(nd.FP32)):
            name = nd.plan_name(nd.FP32, k)
            if not name.startswith("fp32_"):
                continue
            nd.set_plan(nd.FP32, k, 0)
            ms_k, kern_k, _ = time_caf(nd, torch, s, r, (n, tau0, n_tau, p0, n_dop), nd.FP32,
                                       max(3, args.steps // 4), 2)
            cands.append((ms_k, kern_k, name))
        nd.set_plan(nd.FP32, -1, 0)
        ms_p, kern_p, name_p = min(cands)
        tf = flops_per_call / (kern_p * 1e-3) / 1e12
        plain = {"plan": name_p, "ms_per_step": ms_p, "cells_per_s": cells / (ms_p * 1e-3),
                 "contraction_kernel_ms": kern_p, "contraction_tflops_algorithmic": tf,
                 "frac_of_fp32_mfma_peak": tf / PEAK_TFLOPS["fp32"],
                 "plans_timed": {c[2]: c[0] for c in cands}}
    fft_form = results.get("fp32")
    for form, rres in results.items():
        rres["speedup_vs_plain_fp32"] = plain["ms_per_step"] / rres["ms_per_step"] if plain else None
        rres["speedup_vs_fp32_fft_form"] = fft_form["ms_per_step"] / rres["ms_per_step"] if fft_form else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        nthr = oracle.num_threads()
        rows = list(range(nthr))  # one row per thread: the oracle runs rows in parallel
        t0 = time.perf_counter()
        Ao, sc = oracle.caf(c["s"], c["r"], tau0, n_tau, p0, n_dop, rows=np.array(rows))
        t1 = time.perf_counter() - t0
        per_batch = max(t1, 1e-3)
        batches = max(1, int(args.cpu_seconds / per_batch))
        rows2 = list(range(nthr, min(n_tau, nthr * (1 + batches))))
        t0 = time.perf_counter()
        Ao2, sc2 = oracle.caf(c["s"], c["r"], tau0, n_tau, p0, n_dop, rows=np.array(rows2))
        t2 = time.perf_counter() - t0
        cpu = {
            "value": len(rows2) * n_dop / t2,
            "unit": "cells/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP64 literal oracle, delay rows %d..%d x all %d Doppler bins of the same "
                      "N=65536 surface (%.1f s)" % (rows2[0], rows2[-1], n_dop, t2),
        }
        # max l1-relative error of each form on the sampled rows
        allrows = np.array(rows + rows2)
        Aor = np.concatenate([Ao, Ao2])
        scr = np.concatenate([sc, sc2])
        for form, o in outs.items():
            g = o[allrows].astype(np.complex128)
            err = (np.abs(g.real - Aor.real) + np.abs(g.imag - Aor.imag)) / np.where(scr > 0, scr, 1)
            results[form]["max_l1_rel_err_vs_oracle"] = float(err.max())
            results[form]["err_rows_checked"] = int(len(allrows))

    extras = {}
    want = set() if args.no_extras else set(x for x in args.extras.split(",") if x)
    if "config2" in want:
        extras["config2"] = bench_config2(nd, synth, torch, args)
    if "forward" in want:
        extras["forward"] = bench_forward(nd, torch, args)
    if "batched" in want:
        extras["batched"] = bench_batched(nd, tune, synth, torch, args)
    if "adjoint" in want:
        extras["adjoint"] = bench_adjoint(nd, synth, torch, args)
    if "surfaces" in want:
        extras.update(bench_other_surfaces(nd, synth, torch, args))
    if "robustness" in want:
        extras["robustness"] = bench_robustness(nd, synth, torch, args)
    if "nfft" in want:
        extras["nfft"] = bench_nfft(nd, torch, args)

    main_res = results[args.form]
    line = {
        "metric": "ambiguity cells/s (tau x Doppler) at N=65536",
        "value": main_res["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.form,
        "data": "synthetic",
        "config": {"workload": "caf_n65536_tau1024_dop512", "n": n, "tau0": tau0,
                   "n_tau": n_tau, "p0": p0, "n_dop": n_dop, "form": args.form},
        "roofline": {
            "bound": main_res["bound"],
            "achieved": main_res["timed_kernel_tflops"],
            "peak": main_res["peak_tflops"],
            "unit": main_res["unit"],
            "frac": main_res["frac_of_peak"],
            "traffic": load_traffic(args.form, main_res["dominant"]),
            "kernel": main_res["timed_kernel"],
        },
        "speedup_vs_plain_fp32": main_res["speedup_vs_plain_fp32"],
        "cpu_baseline": cpu,
        "forms": results,
        "plain_fp32": plain,
        **extras,
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
