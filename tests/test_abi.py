"""The C ABI library: loads without a GPU, exports every declared symbol, and rejects
invalid arguments on the host before anything is enqueued (no device memory touched:
the pointers passed here are NULL or host addresses)."""
import ctypes
import os
import re

import pytest

from paper_1402_0532_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ndft.h")

INVAL, UNSUPPORTED, WORKSPACE = 1, 2, 3


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ndft_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name
    assert set(_lib.SIGNATURES) == set(names)


def test_status_strings_and_version():
    lib = _lib.load()
    for st in range(5):
        assert lib.ndft_status_string(st).startswith(b"NDFT_")
    assert b"gfx950" in lib.ndft_version()


def _host_buf(nbytes=4096):
    buf = ctypes.create_string_buffer(nbytes + 256)
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    return buf, ctypes.c_void_p(addr)


@pytest.mark.parametrize(
    "n,tau0,n_tau,p0,n_dop",
    [(0, 0, 1, 0, 1), (8, -1, 1, 0, 1), (8, 0, 0, 0, 1), (8, 4, 5, 0, 1), (8, 0, 1, 0, 0),
     (8, 0, 1, 0, 9), ((1 << 24) + 1, 0, 1, 0, 1)],
)
def test_caf_rejects_bad_shapes(n, tau0, n_tau, p0, n_dop):
    lib = _lib.load()
    keep, p = _host_buf()
    st = lib.ndft_caf(p, p, n, tau0, n_tau, p0, n_dop, p, 0, p, 4096, None)
    assert st == INVAL
    assert lib.ndft_caf_workspace(n, tau0, n_tau, p0, n_dop, 0) == 0
    st = lib.ndft_dbg_signs(p, p, n, tau0, n_tau, p0, n_dop, p, p, None)
    assert st == INVAL


def test_caf_rejects_null_misaligned_and_precision():
    lib = _lib.load()
    keep, p = _host_buf()
    odd = ctypes.c_void_p(p.value + 4)
    assert lib.ndft_caf(None, p, 16, 0, 4, 0, 4, p, 0, p, 4096, None) == INVAL
    assert lib.ndft_caf(p, p, 16, 0, 4, 0, 4, None, 0, p, 4096, None) == INVAL
    assert lib.ndft_caf(odd, p, 16, 0, 4, 0, 4, p, 0, p, 4096, None) == INVAL
    assert lib.ndft_caf(p, p, 16, 0, 4, 0, 4, p, 7, p, 4096, None) == INVAL
    # FP8 is a supported form for the surface (here the workspace is too small) ...
    assert lib.ndft_caf(p, p, 16, 0, 4, 0, 4, p, 2, None, 0, None) == WORKSPACE
    # ... but the adjoint has no FP8 form
    assert lib.ndft_caf_backward(p, p, 16, 0, 4, 0, 4, p, p, None, 2, p, 4096, None) == UNSUPPORTED


def test_caf_rejects_small_or_misaligned_workspace():
    lib = _lib.load()
    keep, p = _host_buf()
    need = lib.ndft_caf_workspace(4096, 0, 256, 0, 4096, 0)
    assert need > 0
    assert lib.ndft_caf(p, p, 4096, 0, 256, 0, 4096, p, 0, None, 0, None) == WORKSPACE
    assert lib.ndft_caf(p, p, 4096, 0, 256, 0, 4096, p, 0, p, need - 1, None) == WORKSPACE
    odd = ctypes.c_void_p(p.value + 8)
    assert lib.ndft_caf(p, p, 4096, 0, 256, 0, 4096, p, 0, odd, need, None) == WORKSPACE


def test_forward_rejects_bad_args():
    lib = _lib.load()
    keep, p = _host_buf()
    assert lib.ndft_forward(p, p, 1, 0, 0, 1, 0, p, 4096, None) == INVAL
    assert lib.ndft_forward(p, p, 1, 8, 0, 9, 0, p, 4096, None) == INVAL
    assert lib.ndft_forward(p, p, -1, 8, 0, 8, 0, p, 4096, None) == INVAL
    assert lib.ndft_forward(None, p, 2, 8, 0, 8, 0, p, 4096, None) == INVAL
    assert lib.ndft_forward(p, p, 0, 8, 0, 8, 0, None, 0, None) == 0  # empty batch: no-op
    assert lib.ndft_forward(p, p, 2, 8, 0, 8, 9, p, 4096, None) == INVAL


def test_workspace_query_is_consistent():
    lib = _lib.load()
    # symmetric Doppler window: 257 base bins (0..256) serve bins -256..255
    a = lib.ndft_caf_workspace(65536, 0, 1024, -256, 512, 0)
    b = lib.ndft_caf_workspace(65536, 0, 1024, -256, 512, 0)
    assert a == b and a % 256 == 0 and a > 0
    plan = ctypes.c_int32()
    ks = ctypes.c_int32()
    assert lib.ndft_get_plan(0, 65536, 1024, -256, 512, ctypes.byref(plan), ctypes.byref(ks)) == 0
    # ksplit counts matrix-core sample chunks: 0 for a plan without a matrix part
    assert 0 <= plan.value < lib.ndft_plan_count(0) and ks.value >= 0


def test_plan_table():
    lib = _lib.load()
    for prec in (0, 1):
        cnt = lib.ndft_plan_count(prec)
        assert cnt >= 1
        names = [lib.ndft_plan_name(prec, k) for k in range(cnt)]
        assert all(names) and len(set(names)) == cnt
        assert lib.ndft_plan_name(prec, cnt) is None
        assert lib.ndft_set_plan(prec, cnt, 0) == INVAL
        assert lib.ndft_set_plan(prec, 0, 3) == 0
        assert lib.ndft_set_plan(prec, -1, 0) == 0
    assert lib.ndft_plan_count(5) == 0


@pytest.mark.parametrize(
    "n,tau0,n_tau,p0,n_dop",
    [(0, 0, 1, 0, 1), (8, -1, 1, 0, 1), (8, 0, 0, 0, 1), (8, 4, 5, 0, 1), (8, 0, 1, 0, 0),
     (8, 0, 1, 0, 9), ((1 << 24) + 1, 0, 1, 0, 1)],
)
def test_caf12c_rejects_bad_shapes(n, tau0, n_tau, p0, n_dop):
    lib = _lib.load()
    keep, p = _host_buf()
    assert lib.ndft_caf12c(p, p, n, tau0, n_tau, p0, n_dop, p, 1, p, 4096, None) == INVAL
    assert lib.ndft_caf12c_workspace(n, tau0, n_tau, p0, n_dop, 1) == 0


def test_caf12c_precisions_and_workspace():
    lib = _lib.load()
    keep, p = _host_buf()
    odd = ctypes.c_void_p(p.value + 4)
    assert lib.ndft_caf12c(None, p, 16, 0, 4, 0, 4, p, 1, p, 4096, None) == INVAL
    assert lib.ndft_caf12c(odd, p, 16, 0, 4, 0, 4, p, 1, p, 4096, None) == INVAL
    assert lib.ndft_caf12c(p, p, 16, 0, 4, 0, 4, p, 7, p, 4096, None) == INVAL
    # only the sign-split forms compute Eq. (12c); every precision has one
    for prec in (0, 1, 2):
        need = lib.ndft_caf12c_workspace(65536, 0, 1024, -256, 512, prec)
        assert need > 0
        assert lib.ndft_caf12c(p, p, 65536, 0, 1024, -256, 512, p, prec, None, 0, None) == WORKSPACE
        # every Doppler window, also one whose bases reach N / 2
        assert lib.ndft_caf12c_workspace(1002, 0, 8, 0, 1002, prec) > 0


def test_caf12b_arguments_and_workspace():
    lib = _lib.load()
    keep, p = _host_buf()
    assert lib.ndft_caf12b(None, p, 16, 0, 4, 0, 4, p, 0, p, 4096, None) == INVAL
    assert lib.ndft_caf12b(p, p, 8, 4, 5, 0, 1, p, 0, p, 4096, None) == INVAL
    assert lib.ndft_caf12b(p, p, 16, 0, 4, 0, 4, p, 7, p, 4096, None) == INVAL
    # the outer transform is an FP32 decimated DFT: no split-BF16 / FP8 form
    assert lib.ndft_caf12b(p, p, 16, 0, 4, 0, 4, p, 1, p, 4096, None) == UNSUPPORTED
    assert lib.ndft_caf12b(p, p, 16, 0, 4, 0, 4, p, 2, p, 4096, None) == UNSUPPORTED
    assert lib.ndft_caf12b_workspace(16, 0, 4, 0, 4, 1) == 0
    # transform length 512 and a work-group per delay row: no partial surfaces, only the
    # inputs with their signs (16 B per sample, the reference after n zeros)
    assert lib.ndft_caf12b_workspace(4096, 0, 300, -200, 400, 0) == 48 * 4096
    # N = 65536 with 1024 delays: the same; with few delays the phases of a row split over
    # work-groups: 128 phases in groups of 16, eight partial surfaces of 4 x 512
    assert lib.ndft_caf12b_workspace(65536, 0, 1024, -256, 512, 0) == 48 * 65536
    assert lib.ndft_caf12b_workspace(65536, 0, 4, -256, 512, 0) == 8 * 4 * 512 * 8
    assert lib.ndft_caf12b(p, p, 65536, 0, 4, -256, 512, p, 0, None, 0, None) == WORKSPACE
    # more than 1024 bins: the phase-group kernel again
    assert lib.ndft_caf12b_workspace(65536, 0, 1024, -600, 1200, 0) == 8 * 1024 * 1200 * 8


def test_nfft_arguments():
    lib = _lib.load()
    keep, p = _host_buf()
    for n in (0, 3, 12, 1 << 25, -4):
        assert lib.ndft_nfft(p, p, 1, n, 0, None, 0, None) == INVAL
        assert lib.ndft_nfft_workspace(1, n) == 0
    assert lib.ndft_nfft(p, p, -1, 8, 0, None, 0, None) == INVAL
    assert lib.ndft_nfft(None, p, 1, 8, 0, None, 0, None) == INVAL
    assert lib.ndft_nfft(p, p, 1, 8, 2, None, 0, None) == INVAL  # no such reading
    assert lib.ndft_nfft(p, p, 0, 8, 1, None, 0, None) == 0  # nothing to do
    # rows up to 8192 samples need no workspace; longer ones ping-pong rows and a table
    assert lib.ndft_nfft_workspace(100, 8192) == 0
    assert lib.ndft_nfft_workspace(3, 1 << 16) == 3 * (1 << 16) * 8 + ((1 << 16) - 8192) * 8
    assert lib.ndft_nfft(p, p, 3, 1 << 16, 0, None, 0, None) == WORKSPACE


def test_fp32_plan_choice_rules():
    # the FP32 sign-split plan (twiddle half by FFT) is the built-in choice for narrow
    # Doppler windows when N has a power-of-two factor of at least 64, else a contraction
    lib = _lib.load()
    plan = ctypes.c_int32()
    ks = ctypes.c_int32()

    def name(n, n_cols, p0, n_bins):
        assert lib.ndft_get_plan(0, n, n_cols, p0, n_bins, ctypes.byref(plan), ctypes.byref(ks)) == 0
        return lib.ndft_plan_name(0, plan.value).decode()

    assert name(65536, 1024, -256, 512).startswith("fp32s_") and ks.value == 0
    assert name(16384, 100, -64, 128).startswith("fp32s_")
    assert name(4096, 256, 0, 4096) == "fp32x_fast_exact"      # bases up to N / 2, N = 2^12
    assert name(1024, 64, -500, 1000) == "fp32x_fast_exact"
    assert not name(8192, 256, 0, 8192).startswith("fp32s_")   # beyond the fast transform's rows
    assert not name(65540, 3, -2, 5).startswith("fp32s_")      # N = 4 x odd
    assert not name(1000, 64, -3, 7).startswith("fp32s_")      # N = 8 x 125


@pytest.mark.parametrize(
    "n,tau0,n_tau,p0,n_dop",
    [(0, 0, 1, 0, 1), (8, -1, 1, 0, 1), (8, 0, 0, 0, 1), (8, 4, 5, 0, 1), (8, 0, 1, 0, 0),
     (8, 0, 1, 0, 9), ((1 << 24) + 1, 0, 1, 0, 1)],
)
def test_dbg_split_rejects_bad_shapes(n, tau0, n_tau, p0, n_dop):
    lib = _lib.load()
    keep, p = _host_buf()
    assert lib.ndft_dbg_split(p, p, n, tau0, n_tau, p0, n_dop, 1, 0, p, p, p, 4096, None) == INVAL


def test_dbg_split_arguments():
    lib = _lib.load()
    keep, p = _host_buf()
    odd = ctypes.c_void_p(p.value + 4)
    args = (65536, 0, 1024, -256, 512)
    assert lib.ndft_dbg_split(None, p, *args, 1, 0, p, p, p, 4096, None) == INVAL
    assert lib.ndft_dbg_split(odd, p, *args, 1, 0, p, p, p, 4096, None) == INVAL
    assert lib.ndft_dbg_split(p, p, *args, 1, 0, p, odd, p, 4096, None) == INVAL  # misaligned T
    assert lib.ndft_dbg_split(p, p, *args, 7, 0, p, p, p, 4096, None) == INVAL    # precision
    assert lib.ndft_dbg_split(p, p, *args, 1, 2, p, p, p, 4096, None) == INVAL    # lin is 0 or 1
    # the narrow window takes a sign-split plan in every precision: the hook needs the
    # surface call's workspace
    for prec in (0, 1, 2):
        need = lib.ndft_caf_workspace(*args, prec)
        assert need > 0
        assert lib.ndft_dbg_split(p, p, *args, prec, 0, p, p, None, 0, None) == WORKSPACE
        assert lib.ndft_dbg_split(p, p, *args, prec, 1, p, p, None, 0, None) == WORKSPACE
    # the full-window N = 4096 surface takes a combined (non-split) plan in split-BF16
    assert lib.ndft_dbg_split(p, p, 4096, 0, 256, 0, 4096, 1, 0, p, p, p, 1 << 40, None) == UNSUPPORTED


def test_unsupported_shape_rejected_before_any_launch():
    # a twiddle table that exceeds the LDS a plan leaves free is refused on the host,
    # before anything is enqueued (host pointers here: any launch would fault), and the
    # workspace query reports 0 for it
    # (no workspace is passed, so an accepted shape stops at the workspace check and
    # nothing can be launched in either case)
    lib = _lib.load()
    keep, p = _host_buf()
    seen = set()
    for n in (1 << 22, 1 << 24):
        for prec in (0, 1, 2):
            for (n_tau, p0, n_dop) in ((4, -2048, 4096), (4, -4, 8)):
                need = lib.ndft_caf_workspace(n, 0, n_tau, p0, n_dop, prec)
                st = lib.ndft_caf(p, p, n, 0, n_tau, p0, n_dop, p, prec, None, 0, None)
                assert st == (WORKSPACE if need > 0 else UNSUPPORTED), (n, prec, n_dop, need, st)
                seen.add(st)
    assert UNSUPPORTED in seen  # some plan's table does not fit at these lengths


def test_fast_tables_hook_without_a_device():
    # with no device current the hook reports -1 instead of a mask (and touches nothing)
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    assert _lib.load().ndft_dbg_fast_tables(0) == -1
    assert _lib.load().ndft_dbg_fast_tables(1) == -1
