"""FP64 CPU oracle for the NDFT and the NDFT cross-ambiguity surface.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code with the
GPU path (``paper_1402_0532_amd``) and does not import it.

The numerical work lives in ``ndft_oracle.c`` (plain C, FP64, literal Eqs. (1)-(7),
(12a), (12b) and (12c)); this module only loads it with ctypes and marshals numpy arrays. Inputs are
complex arrays (normally complex64 upcast exactly to complex128).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle64.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle64.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
             "-std=gnu11", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_rop.argtypes = [D, D]
        lib.oracle_rop.restype = D
        lib.oracle_cop.argtypes = [P, P, P]
        lib.oracle_twiddle.argtypes = [I, I, P]
        lib.oracle_exact_sign_of_sum.argtypes = [P, P, ctypes.c_int]
        lib.oracle_exact_sign_of_sum.restype = ctypes.c_int
        lib.oracle_lag_row.argtypes = [P, P, I, I, P, P]
        lib.oracle_lag_row_lin.argtypes = [P, P, I, I, P, P]
        lib.oracle_twiddle_signs.argtypes = [I, I, I, P]
        lib.oracle_ndft.argtypes = [P, I, I, I, I, P, P]
        lib.oracle_ndft.restype = ctypes.c_int
        lib.oracle_caf.argtypes = [P, P, I, I, I, I, I, P, I, P, P]
        lib.oracle_caf.restype = ctypes.c_int
        lib.oracle_caf_lin.argtypes = [P, P, I, I, I, I, I, P, I, P, P]
        lib.oracle_caf_lin.restype = ctypes.c_int
        lib.oracle_caf_dft.argtypes = [P, P, I, I, I, I, I, P, I, P, P]
        lib.oracle_caf_dft.restype = ctypes.c_int
        lib.oracle_nfft.argtypes = [P, I, I, P]
        lib.oracle_nfft.restype = ctypes.c_int
        lib.oracle_nfft32.argtypes = [P, I, I, P]
        lib.oracle_nfft32.restype = ctypes.c_int
        lib.oracle_nfft_outer.argtypes = [P, I, I, P]
        lib.oracle_nfft_outer.restype = ctypes.c_int
        lib.oracle_nfft32_outer.argtypes = [P, I, I, P]
        lib.oracle_nfft32_outer.restype = ctypes.c_int
        lib.oracle_caf_grad.argtypes = [P, P, I, I, I, I, I, P, P, P]
        lib.oracle_caf_grad.restype = ctypes.c_int
        lib.oracle_caf_loss.argtypes = [P, P, I, I, I, I, I, P]
        lib.oracle_caf_loss.restype = D
        lib.oracle_caf_loss_fd.argtypes = [P, P, I, I, I, I, I, P, P, I, D, P]
        lib.oracle_caf_loss_fd.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def rop(a: float, b: float) -> float:
    """Eq. (1)-(2)."""
    return float(_load().oracle_rop(a, b))


def cop(a: complex, b: complex) -> complex:
    """Eq. (6)."""
    A = _c128([a])
    B = _c128([b])
    out = np.zeros(1, np.complex128)
    _load().oracle_cop(_ptr(A), _ptr(B), _ptr(out))
    return complex(out[0])


def twiddle(m: int, n: int) -> complex:
    out = np.zeros(1, np.complex128)
    _load().oracle_twiddle(int(m), int(n), _ptr(out))
    return complex(out[0])


def exact_sign_of_sum(values, coeffs) -> int:
    v = np.ascontiguousarray(values, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.int32)
    return int(_load().oracle_exact_sign_of_sum(_ptr(v), _ptr(c), len(v)))


def lag_row(s, r, d: int):
    """z[i] = s[i] (x) conj(r[i-d]) and its exact component signs (int8 [n][2])."""
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    z = np.zeros(n, np.complex128)
    sg = np.zeros((n, 2), np.int8)
    _load().oracle_lag_row(_ptr(s), _ptr(r), n, int(d), _ptr(z), _ptr(sg))
    return z, sg


def lag_row_lin(s, r, d: int):
    """Eq. (12c) lag row: z[i] = s[i] conj(r[i-d]) (ordinary product) and its exact
    component signs (int8 [n][2])."""
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    z = np.zeros(n, np.complex128)
    sg = np.zeros((n, 2), np.int8)
    _load().oracle_lag_row_lin(_ptr(s), _ptr(r), n, int(d), _ptr(z), _ptr(sg))
    return z, sg


def twiddle_signs(n: int, p0: int, n_dop: int) -> np.ndarray:
    """csgn(W^{(p0+q) i mod N}) as int8 [n_dop][n][2]."""
    out = np.zeros((n_dop, n, 2), np.int8)
    _load().oracle_twiddle_signs(int(n), int(p0), int(n_dop), _ptr(out))
    return out


def ndft(x, k0: int = 0, k_count: int | None = None):
    """Eq. (7) on each row of x [batch][n]. Returns (X [batch][k_count], scale)."""
    x = _c128(x)
    if x.ndim == 1:
        x = x[None, :]
    batch, n = x.shape
    k_count = n if k_count is None else int(k_count)
    X = np.zeros((batch, k_count), np.complex128)
    sc = np.zeros((batch, k_count), np.float64)
    rc = _load().oracle_ndft(_ptr(x), batch, n, int(k0), k_count, _ptr(X), _ptr(sc))
    if rc:
        raise ValueError("oracle_ndft: invalid arguments")
    return X, sc


def caf(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, rows=None):
    """Eq. (12a) surface. Returns (A [rows][n_dop], scale [rows][n_dop])."""
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    if rows is None:
        rows_arr = None
        nr = n_tau
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rows_arr.shape[0]
    A = np.zeros((nr, n_dop), np.complex128)
    sc = np.zeros((nr, n_dop), np.float64)
    rc = _load().oracle_caf(
        _ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop),
        None if rows_arr is None else _ptr(rows_arr), nr, _ptr(A), _ptr(sc),
    )
    if rc:
        raise ValueError("oracle_caf: invalid arguments")
    return A, sc


def nfft(x):
    """NFFT of Section 3 (radix-2 DIT, twiddle products by Eq. (6)) of each row of x
    [batch][n] (n a power of two), FP64."""
    x = np.atleast_2d(_c128(x))
    X = np.zeros_like(x)
    if _load().oracle_nfft(_ptr(x), x.shape[0], x.shape[1], _ptr(X)):
        raise ValueError("oracle_nfft: n must be a power of two")
    return X


def nfft32(x):
    """The same recursion in FP32 arithmetic (complex64 in and out)."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex64)
    X = np.zeros_like(x)
    if _load().oracle_nfft32(_ptr(x), x.shape[0], x.shape[1], _ptr(X)):
        raise ValueError("oracle_nfft32: n must be a power of two")
    return X


def nfft_outer(x):
    """The printed reading of Eq. (10): ordinary products with W_n^k at every level of the
    radix-2 recursion, the operator of Eq. (6) in the length-1 sums at its bottom
    (x (x) 1). FP64, rows of x [batch][n] (n a power of two)."""
    x = np.atleast_2d(_c128(x))
    X = np.zeros_like(x)
    if _load().oracle_nfft_outer(_ptr(x), x.shape[0], x.shape[1], _ptr(X)):
        raise ValueError("oracle_nfft_outer: n must be a power of two")
    return X


def nfft32_outer(x):
    """The same recursion in FP32, each product and sum rounded on its own."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex64)
    X = np.zeros_like(x)
    if _load().oracle_nfft32_outer(_ptr(x), x.shape[0], x.shape[1], _ptr(X)):
        raise ValueError("oracle_nfft32_outer: n must be a power of two")
    return X


def _surface(fn, s, r, tau0, n_tau, p0, n_dop, rows):
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    if rows is None:
        rows_arr = None
        nr = n_tau
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rows_arr.shape[0]
    A = np.zeros((nr, n_dop), np.complex128)
    sc = np.zeros((nr, n_dop), np.float64)
    rc = fn(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop),
            None if rows_arr is None else _ptr(rows_arr), nr, _ptr(A), _ptr(sc))
    if rc:
        raise ValueError("oracle surface: invalid arguments")
    return A, sc


def caf12b(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, rows=None):
    """Eq. (12b) surface (lag product of Eq. (6), then the ordinary DFT). Returns
    (A [rows][n_dop], scale [rows][n_dop]), scale the l1 mass of the real products."""
    return _surface(_load().oracle_caf_dft, s, r, tau0, n_tau, p0, n_dop, rows)


def caf12c(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, rows=None):
    """Eq. (12c) surface (linear lag product, then the Eq. (6) operator with the
    twiddle). Returns (A [rows][n_dop], scale [rows][n_dop])."""
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    if rows is None:
        rows_arr = None
        nr = n_tau
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rows_arr.shape[0]
    A = np.zeros((nr, n_dop), np.complex128)
    sc = np.zeros((nr, n_dop), np.float64)
    rc = _load().oracle_caf_lin(
        _ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0), int(n_dop),
        None if rows_arr is None else _ptr(rows_arr), nr, _ptr(A), _ptr(sc),
    )
    if rc:
        raise ValueError("oracle_caf_lin: invalid arguments")
    return A, sc


def caf11(s, r, tau0: int, n_tau: int, p0: int, n_dop: int):
    """The ordinary cross-ambiguity function of Eq. (11): for each delay l the DFT of the
    lag products s[i] conj(r[i - l]) (r zero before the record) at bins p = p0 + q mod N,
    in FP64 (numpy's FFT as the DFT step). Comparison surface of the detection runs of
    Section 5; returns A [n_tau][n_dop] complex128."""
    s = _c128(s)
    r = _c128(r)
    n = s.shape[0]
    bins = (int(p0) + np.arange(int(n_dop))) % n
    A = np.zeros((int(n_tau), int(n_dop)), np.complex128)
    for j in range(int(n_tau)):
        d = int(tau0) + j
        rd = np.zeros(n, np.complex128)
        rd[d:] = r[: n - d]
        A[j] = np.fft.fft(s * np.conj(rd))[bins]
    return A


def caf_grad(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, G):
    """(grad_r, grad_s) of a real loss with upstream G = dL/dReA + j dL/dImA."""
    s = _c128(s)
    r = _c128(r)
    G = _c128(G)
    n = s.shape[0]
    gr = np.zeros(n, np.complex128)
    gs = np.zeros(n, np.complex128)
    rc = _load().oracle_caf_grad(_ptr(s), _ptr(r), n, int(tau0), int(n_tau), int(p0),
                                 int(n_dop), _ptr(G), _ptr(gr), _ptr(gs))
    if rc:
        raise ValueError("oracle_caf_grad: invalid arguments")
    return gr, gs


def caf_loss(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, w) -> float:
    s = _c128(s)
    r = _c128(r)
    w = np.ascontiguousarray(w, dtype=np.float64)
    return float(_load().oracle_caf_loss(_ptr(s), _ptr(r), s.shape[0], int(tau0), int(n_tau),
                                         int(p0), int(n_dop), _ptr(w)))


def caf_loss_fd(s, r, tau0: int, n_tau: int, p0: int, n_dop: int, w, coords, h: float = 1e-4):
    """Central differences of sum w|A|^2 at coords (2m -> Re r[m], 2m+1 -> Im r[m])."""
    s = _c128(s)
    r = _c128(r)
    w = np.ascontiguousarray(w, dtype=np.float64)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    out = np.zeros(c.shape[0], np.float64)
    rc = _load().oracle_caf_loss_fd(_ptr(s), _ptr(r), s.shape[0], int(tau0), int(n_tau),
                                    int(p0), int(n_dop), _ptr(w), _ptr(c), c.shape[0],
                                    float(h), _ptr(out))
    if rc:
        raise ValueError("oracle_caf_loss_fd: invalid arguments")
    return out
