"""Python binding of libndft.so: the multiplication-free NDFT (Eq. (7)) and the NDFT
cross-ambiguity surface (Eq. (12a)) of Bozkurt et al. (arXiv 1402.0532) on MI355X.

This module only marshals arguments: torch tensors provide device memory and the
current stream; every step of the computation runs in the HIP kernels of libndft.so.
There is no CPU or PyTorch fallback.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

FP32 = 0
BF16X2 = 1
FP8 = 2
PRECISIONS = {"fp32": FP32, "bf16x2": BF16X2, "fp8": FP8}

__all__ = [
    "FP32", "BF16X2", "FP8", "forward", "nfft", "caf", "caf12b", "caf12c", "caf_backward", "caf_batched", "caf_batched_dev", "BatchPlan",
    "pack_batch",
    "NDFTCaf", "dbg_signs", "dbg_split", "plan_count", "plan_name", "set_plan", "get_plan",
    "prof_enable", "prof_read", "version",
]


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p.lower()]
    return int(p)


def _stream_handle() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_c64(t: torch.Tensor, name: str, ndim: int) -> None:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex64:
        raise TypeError("%s must be a complex64 tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on a GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dim() != ndim:
        raise ValueError("%s must have %d dimension(s)" % (name, ndim))


def _check_out(out: torch.Tensor, shape, device) -> None:
    """A caller-supplied output must be a contiguous complex64 tensor of exactly the
    result's shape on the inputs' device (the kernels write every element of it)."""
    _check_c64(out, "out", len(shape))
    if tuple(out.shape) != tuple(shape):
        raise ValueError("out must have shape %s, got %s" % (tuple(shape), tuple(out.shape)))
    if out.device != device:
        raise ValueError("out must be on %s" % (device,))


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _ws_for(ws: torch.Tensor | None, nbytes: int, device) -> torch.Tensor | None:
    """The caller's workspace if it is a contiguous byte tensor of at least nbytes on
    device, else a new one."""
    if (ws is None or not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or not ws.is_contiguous()
            or ws.device != device or ws.numel() < nbytes):
        return _workspace(nbytes, device)
    return ws


def version() -> str:
    return _lib.load().ndft_version().decode()


def forward(x: torch.Tensor, k0: int = 0, k_count: int | None = None, prec=FP32) -> torch.Tensor:
    """NDFT (Eq. (7)) of each row of x [batch, n] at bins k0 .. k0+k_count-1 (mod n)."""
    lib = _lib.load()
    if x.dim() == 1:
        return forward(x[None], k0, k_count, prec)[0]
    _check_c64(x, "x", 2)
    batch, n = x.shape
    k_count = n if k_count is None else int(k_count)
    p = _prec(prec)
    out = torch.empty((batch, k_count), dtype=torch.complex64, device=x.device)
    nbytes = lib.ndft_forward_workspace(batch, n, k0, k_count, p)
    ws = _workspace(nbytes, x.device)
    st = lib.ndft_forward(_ptr(x), _ptr(out), batch, n, int(k0), k_count, p, _ptr(ws),
                          nbytes, _stream_handle())
    _lib.check(st, "ndft_forward")
    return out


def caf(s: torch.Tensor, r: torch.Tensor, tau0: int, n_tau: int, p0: int, n_dop: int,
        prec=FP32, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. (12a) surface A[n_tau, n_dop]: delays tau0 + l, Doppler bins p0 + q (mod n)."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    n = s.shape[0]
    if r.shape[0] != n:
        raise ValueError("surv and ref must have the same length")
    p = _prec(prec)
    if r.device != s.device:
        raise ValueError("surv and ref must be on the same device")
    if out is None:
        out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device)
    else:
        _check_out(out, (n_tau, n_dop), s.device)
    nbytes = lib.ndft_caf_workspace(n, tau0, n_tau, p0, n_dop, p)
    ws = _ws_for(ws, nbytes, s.device)
    st = lib.ndft_caf(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop), _ptr(out),
                      p, _ptr(ws), nbytes, _stream_handle())
    _lib.check(st, "ndft_caf")
    return out


NFFT_EVERY_BUTTERFLY = 0
NFFT_PRINTED = 1


def nfft(x: torch.Tensor, reading: int = NFFT_EVERY_BUTTERFLY, ws: torch.Tensor | None = None) -> torch.Tensor:
    """NFFT of Section 3 (radix-2 DIT with the operator of Eq. (6) in the butterflies) of
    each row of x [batch, n] complex64, n a power of two up to 2^24; FP32. reading:
    NFFT_EVERY_BUTTERFLY (every twiddle product by Eq. (6)) or NFFT_PRINTED (ordinary
    twiddle products, the operator in the length-1 sums)."""
    lib = _lib.load()
    if x.dim() == 1:
        return nfft(x[None], reading, ws)[0]
    _check_c64(x, "x", 2)
    batch, n = x.shape
    out = torch.empty_like(x)
    nbytes = int(lib.ndft_nfft_workspace(batch, n))
    ws = _ws_for(ws, nbytes, x.device)
    _lib.check(lib.ndft_nfft(_ptr(x), _ptr(out), batch, n, int(reading), _ptr(ws) if nbytes else None, nbytes,
                             _stream_handle()), "ndft_nfft")
    return out


def caf12b(s: torch.Tensor, r: torch.Tensor, tau0: int, n_tau: int, p0: int, n_dop: int,
           prec=FP32, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. (12b) surface A[n_tau, n_dop] (lag product of Eq. (6), then the ordinary DFT);
    FP32 only."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    n = s.shape[0]
    if r.shape[0] != n:
        raise ValueError("surv and ref must have the same length")
    p = _prec(prec)
    if r.device != s.device:
        raise ValueError("surv and ref must be on the same device")
    if out is None:
        out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device)
    else:
        _check_out(out, (n_tau, n_dop), s.device)
    nbytes = lib.ndft_caf12b_workspace(n, tau0, n_tau, p0, n_dop, p)
    ws = _ws_for(ws, nbytes, s.device)
    st = lib.ndft_caf12b(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop), _ptr(out),
                         p, _ptr(ws) if nbytes else None, nbytes, _stream_handle())
    _lib.check(st, "ndft_caf12b")
    return out


def caf12b_workspace_bytes(n: int, tau0: int, n_tau: int, p0: int, n_dop: int, prec=FP32) -> int:
    return int(_lib.load().ndft_caf12b_workspace(n, tau0, n_tau, p0, n_dop, _prec(prec)))


def caf12c(s: torch.Tensor, r: torch.Tensor, tau0: int, n_tau: int, p0: int, n_dop: int,
           prec=BF16X2, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. (12c) surface A[n_tau, n_dop] (ordinary lag product, then the Eq. (6) operator
    with the twiddle). BF16X2 and FP8 run a sign-split plan with the twiddle half on the
    matrix cores; FP32 takes the twiddle half as an FFT of the exact lag signs, or the fast
    exact transform for n a power of two up to 4096 and wide windows."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    n = s.shape[0]
    if r.shape[0] != n:
        raise ValueError("surv and ref must have the same length")
    p = _prec(prec)
    if r.device != s.device:
        raise ValueError("surv and ref must be on the same device")
    if out is None:
        out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device)
    else:
        _check_out(out, (n_tau, n_dop), s.device)
    nbytes = lib.ndft_caf12c_workspace(n, tau0, n_tau, p0, n_dop, p)
    ws = _ws_for(ws, nbytes, s.device)
    st = lib.ndft_caf12c(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop), _ptr(out),
                         p, _ptr(ws), nbytes, _stream_handle())
    _lib.check(st, "ndft_caf12c")
    return out


def caf12c_workspace_bytes(n: int, tau0: int, n_tau: int, p0: int, n_dop: int, prec=BF16X2) -> int:
    return int(_lib.load().ndft_caf12c_workspace(n, tau0, n_tau, p0, n_dop, _prec(prec)))


def caf_workspace_bytes(n: int, tau0: int, n_tau: int, p0: int, n_dop: int, prec=FP32) -> int:
    return int(_lib.load().ndft_caf_workspace(n, tau0, n_tau, p0, n_dop, _prec(prec)))


def caf_backward(s: torch.Tensor, r: torch.Tensor, tau0: int, n_tau: int, p0: int, n_dop: int,
                 grad_A: torch.Tensor, prec=FP32, need_grad_s: bool = True):
    """Adjoint of caf: (grad_ref, grad_surv or None) for upstream grad_A [n_tau, n_dop]."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    _check_c64(grad_A, "grad_A", 2)
    n = s.shape[0]
    if tuple(grad_A.shape) != (n_tau, n_dop):
        raise ValueError("grad_A must be [n_tau, n_dop]")
    p = _prec(prec)
    gr = torch.empty(n, dtype=torch.complex64, device=s.device)
    gs = torch.empty(n, dtype=torch.complex64, device=s.device) if need_grad_s else None
    nbytes = lib.ndft_caf_backward_workspace(n, tau0, n_tau, p0, n_dop, p)
    ws = _workspace(nbytes, s.device)
    st = lib.ndft_caf_backward(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop),
                               _ptr(grad_A), _ptr(gr), _ptr(gs), p, _ptr(ws), nbytes,
                               _stream_handle())
    _lib.check(st, "ndft_caf_backward")
    return gr, gs


class NDFTCaf(torch.autograd.Function):
    """Differentiable Eq. (12a) surface; gradients through libndft's hand adjoint."""

    @staticmethod
    def forward(ctx, s, r, tau0, n_tau, p0, n_dop, prec=FP32):
        ctx.save_for_backward(s, r)
        ctx.args = (int(tau0), int(n_tau), int(p0), int(n_dop), _prec(prec))
        return caf(s.detach(), r.detach(), tau0, n_tau, p0, n_dop, prec)

    @staticmethod
    def backward(ctx, grad_A):
        s, r = ctx.saved_tensors
        tau0, n_tau, p0, n_dop, prec = ctx.args
        gr, gs = caf_backward(s.detach(), r.detach(), tau0, n_tau, p0, n_dop,
                              grad_A.contiguous(), prec, need_grad_s=ctx.needs_input_grad[0])
        return (gs if ctx.needs_input_grad[0] else None,
                gr if ctx.needs_input_grad[1] else None, None, None, None, None, None)


class BatchPlan:
    """A prepared batch of CPIs for the persistent batched surface kernel.

    cpis: list of dicts with n, surv_off, ref_off, out_off, tau0, n_tau, p0, n_dop
    (offsets in complex elements into the pools). chunk: samples per work item (0 =
    library default). The workspace holds the tables and stays owned by this object.
    """

    def __init__(self, cpis, prec=FP32, device="cuda", chunk: int = 0):
        lib = _lib.load()
        self.prec = _prec(prec)
        self.n_cpi = len(cpis)
        arr = (_lib.NdftCpi * self.n_cpi)()
        for k, c in enumerate(cpis):
            for f in ("n", "surv_off", "ref_off", "out_off", "tau0", "n_tau", "p0", "n_dop"):
                setattr(arr[k], f, int(c[f]))
        self._arr = arr
        self.ws_bytes = int(lib.ndft_caf_batched_workspace(arr, self.n_cpi, self.prec, int(chunk)))
        if self.ws_bytes == 0:
            raise RuntimeError("ndft_caf_batched_workspace: invalid batch")
        self.ws = _workspace(self.ws_bytes, device)
        self.batch = _lib.NdftBatch()
        st = lib.ndft_caf_batched_prepare(arr, self.n_cpi, self.prec, int(chunk), _ptr(self.ws),
                                          self.ws_bytes, ctypes.byref(self.batch))
        _lib.check(st, "ndft_caf_batched_prepare")

    @property
    def plan_name(self) -> str:
        return plan_name(self.prec, self.batch.plan)

    def run(self, surv_pool, ref_pool, out_pool) -> torch.Tensor:
        lib = _lib.load()
        _check_c64(surv_pool, "surv_pool", 1)
        _check_c64(ref_pool, "ref_pool", 1)
        _check_c64(out_pool, "out_pool", 1)
        if not (surv_pool.device == ref_pool.device == out_pool.device == self.ws.device):
            raise ValueError("pools and workspace must be on one device")
        # the kernels read and write every element the descriptors name
        need_s = max(c.surv_off + c.n for c in self._arr)
        need_r = max(c.ref_off + c.n for c in self._arr)
        need_o = max(c.out_off + c.n_tau * c.n_dop for c in self._arr)
        if surv_pool.numel() < need_s or ref_pool.numel() < need_r or out_pool.numel() < need_o:
            raise ValueError("pools too small for the batch: need surv %d, ref %d, out %d elements"
                             % (need_s, need_r, need_o))
        st = lib.ndft_caf_batched(ctypes.byref(self.batch), _ptr(surv_pool), _ptr(ref_pool),
                                  _ptr(out_pool), _ptr(self.ws), self.ws_bytes, _stream_handle())
        _lib.check(st, "ndft_caf_batched")
        return out_pool


def caf_batched(plan: BatchPlan, surv_pool, ref_pool, out_pool):
    return plan.run(surv_pool, ref_pool, out_pool)


CPI_FIELDS = ("n", "surv_off", "ref_off", "out_off", "tau0", "n_tau", "p0", "n_dop")


def cpi_table(descs, device="cuda") -> torch.Tensor:
    """CPI descriptors as the device table ndft_caf_batched_dev reads: int64 [n_cpi, 8]."""
    return torch.tensor([[int(d[f]) for f in CPI_FIELDS] for d in descs], dtype=torch.int64, device=device)


def caf_batched_dev_workspace_bytes(n_cpi: int, max_n: int, max_tau: int, max_dop: int, prec=FP32) -> int:
    return int(_lib.load().ndft_caf_batched_dev_workspace(int(n_cpi), int(max_n), int(max_tau), int(max_dop),
                                                          _prec(prec)))


def caf_batched_dev(surv_pool, ref_pool, out_pool, cpis_dev: torch.Tensor, prec=FP32, ws: torch.Tensor = None,
                    status: torch.Tensor = None) -> torch.Tensor:
    """Batched surfaces from device-resident descriptors (cpis_dev int64 [n_cpi, 8], see
    cpi_table) with no host-side preparation; ws: a uint8 device buffer (its size bounds
    the work-item chunking). status (optional int32 [1] device tensor) receives the
    batch's status after the call (0 = ran); nothing is synchronized here."""
    lib = _lib.load()
    for t, name in ((surv_pool, "surv_pool"), (ref_pool, "ref_pool"), (out_pool, "out_pool")):
        _check_c64(t, name, 1)
    if cpis_dev.dtype != torch.int64 or cpis_dev.dim() != 2 or cpis_dev.shape[1] != 8 or not cpis_dev.is_contiguous():
        raise ValueError("cpis_dev must be a contiguous int64 [n_cpi, 8] tensor")
    if ws is None or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 device tensor")
    devs = {surv_pool.device, ref_pool.device, out_pool.device, cpis_dev.device, ws.device}
    if len(devs) != 1:
        raise ValueError("pools, descriptors and workspace must be on one device")
    st = lib.ndft_caf_batched_dev(_ptr(surv_pool), _ptr(ref_pool), _ptr(out_pool), _ptr(cpis_dev),
                                  int(cpis_dev.shape[0]), _prec(prec), _ptr(ws), ws.numel(), _stream_handle())
    _lib.check(st, "ndft_caf_batched_dev")
    if status is not None:
        if status.dtype != torch.int32 or status.numel() < 1 or status.device != ws.device:
            raise ValueError("status must be an int32 device tensor")
        _lib.check(lib.ndft_caf_batched_dev_status(_ptr(ws), _ptr(status), _stream_handle()),
                   "ndft_caf_batched_dev_status")
    return out_pool


def pack_batch(cpis):
    """Concatenate per-CPI numpy arrays into pools; returns (surv_pool, ref_pool, descs,
    out_len) with descs ready for BatchPlan."""
    import numpy as np

    descs = []
    so = ro = oo = 0
    for c in cpis:
        n = int(c["n"])
        descs.append(dict(n=n, surv_off=so, ref_off=ro, out_off=oo, tau0=int(c["tau0"]),
                          n_tau=int(c["n_tau"]), p0=int(c["p0"]), n_dop=int(c["n_dop"])))
        so += n
        ro += n
        oo += int(c["n_tau"]) * int(c["n_dop"])
    surv = np.concatenate([np.asarray(c["s"], np.complex64) for c in cpis])
    ref = np.concatenate([np.asarray(c["r"], np.complex64) for c in cpis])
    return surv, ref, descs, oo


def dbg_signs(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, twiddle: bool = True,
              lag: bool = True):
    """Exact sign operands used by the kernels: (tw [n_dop, n, 2], lag [n_tau, n, 2]) int8."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    n = s.shape[0]
    tw = torch.empty((n_dop, n, 2), dtype=torch.int8, device=s.device) if twiddle else None
    lg = torch.empty((n_tau, n, 2), dtype=torch.int8, device=s.device) if lag else None
    st = lib.ndft_dbg_signs(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop),
                            _ptr(tw), _ptr(lg), _stream_handle())
    _lib.check(st, "ndft_dbg_signs")
    return tw, lg


def dbg_split(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, prec=BF16X2, lin: bool = False,
              lag: bool = True, T: bool = True):
    """Sign operands of the sign-split plans, from the plan's own lag kernel: (lag [n_tau, n, 2]
    int8 lag signs as the matrix-core half consumes them, T [n_tau, n_dop] complex64 twiddle-
    sign half; bins p = 0 mod n hold the whole cell). lin selects the Eq. (12c) lag product."""
    lib = _lib.load()
    _check_c64(s, "surv", 1)
    _check_c64(r, "ref", 1)
    n = s.shape[0]
    if r.shape[0] != n:
        raise ValueError("surv and ref must have the same length")
    p = _prec(prec)
    lg = torch.empty((n_tau, n, 2), dtype=torch.int8, device=s.device) if lag else None
    tt = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device) if T else None
    nbytes = (lib.ndft_caf12c_workspace if lin else lib.ndft_caf_workspace)(n, tau0, n_tau, p0, n_dop, p)
    ws = _workspace(nbytes, s.device)
    st = lib.ndft_dbg_split(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop), p,
                            1 if lin else 0, _ptr(lg), _ptr(tt), _ptr(ws), nbytes, _stream_handle())
    _lib.check(st, "ndft_dbg_split")
    return lg, tt


def fast_tables_cached(reset: bool = False) -> int:
    """Bit mask of the lengths (bit lg: N = 2^lg) whose fast-transform tables the current
    device holds; reset clears it after reading."""
    m = int(_lib.load().ndft_dbg_fast_tables(1 if reset else 0))
    if m < 0:
        raise RuntimeError("ndft_dbg_fast_tables: no current device")
    return m


def plan_count(prec=FP32) -> int:
    return int(_lib.load().ndft_plan_count(_prec(prec)))


def plan_name(prec, plan: int) -> str:
    v = _lib.load().ndft_plan_name(_prec(prec), int(plan))
    return None if v is None else v.decode()


def set_plan(prec, plan: int = -1, ksplit: int = 0) -> None:
    _lib.check(_lib.load().ndft_set_plan(_prec(prec), int(plan), int(ksplit)), "ndft_set_plan")


def get_plan(prec, n: int, n_cols: int, p0: int, n_bins: int):
    """(plan index, ksplit) the library would use for this shape."""
    a = ctypes.c_int32()
    b = ctypes.c_int32()
    _lib.check(_lib.load().ndft_get_plan(_prec(prec), n, n_cols, p0, n_bins, ctypes.byref(a),
                                         ctypes.byref(b)), "ndft_get_plan")
    return a.value, b.value


def prof_enable(on: bool = True) -> None:
    _lib.check(_lib.load().ndft_prof_enable(1 if on else 0), "ndft_prof_enable")


def prof_read(slot: int = 0):
    """Summed milliseconds and launch count of the timed kernel since the last read:
    slot 0 the contraction (or the FP32 sign-split plan's FFT), slot 1 the twiddle-sign
    kernel of the sign-split plans."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _lib.check(_lib.load().ndft_prof_read_slot(int(slot), ctypes.byref(ms), ctypes.byref(cnt)),
               "ndft_prof_read_slot")
    return ms.value, cnt.value
