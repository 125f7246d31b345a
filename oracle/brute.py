"""Pure-Python brute-force NDFT / cross-ambiguity evaluation for tiny sizes (N <= 16).

TEST INFRASTRUCTURE ONLY: used by the test suite to pin the FP64 C oracle; nothing in
the product path imports it.

Every step is the paper's definition written out with Python scalars:

* ``rop``  -- Eq. (1) with the sign table of Eq. (2): sign(a*b)(|a|+|b|), 0 otherwise.
* ``cop``  -- Eq. (6): a_r(x)b_r - a_i(x)b_i + j(a_i(x)b_r + b_i(x)a_r).
* ``ndft`` -- Eq. (7): X[k] = sum_n W^{kn mod N} (x) x[n], W = e^{-j2pi/N}, no 1/N.
* ``caf``  -- Eq. (12a) read as ((s[i] (x) conj(r[i-d])) (x) W^{ip}), r[m<0] = 0.
* ``caf12b`` -- Eq. (12b): (s[i] (x) conj(r[i-d])) W^{ip}, the DFT ordinary.
* ``caf12c`` -- Eq. (12c): (s[i] conj(r[i-d])) (x) W^{ip}, the lag product ordinary.

Lag products are evaluated in exact rational arithmetic (``fractions.Fraction``) so
their signs are exact; twiddles are FP64 except at quadrant multiples, where they are
exactly 1, -j, -1, +j.
"""
from __future__ import annotations

import math
from fractions import Fraction


def _sign_of_product(a, b) -> int:
    # Eq. (2)
    if (a > 0 and b > 0) or (a < 0 and b < 0):
        return 1
    if (a < 0 and b > 0) or (a > 0 and b < 0):
        return -1
    return 0


def rop(a, b):
    """Eq. (1): a (x) b = sign(a*b)(|a| + |b|)."""
    s = _sign_of_product(a, b)
    if s == 0:
        return 0
    return s * (abs(a) + abs(b))


def cop(a: tuple, b: tuple) -> tuple:
    """Eq. (6) on (re, im) pairs."""
    ar, ai = a
    br, bi = b
    return (rop(ar, br) - rop(ai, bi), rop(ai, br) + rop(bi, ar))


def twiddle(m: int, n: int) -> tuple:
    """W^m, W = e^{-j2pi/N}, exponent reduced mod N; exact at quadrant multiples."""
    m %= n
    if (4 * m) % n == 0:
        return [(1.0, 0.0), (0.0, -1.0), (-1.0, 0.0), (0.0, 1.0)][(4 * m) // n]
    th = 2.0 * math.pi * m / n
    return (math.cos(th), -math.sin(th))


def ndft(x: list, k0: int = 0, k_count: int | None = None) -> list:
    """Eq. (7) for one vector x of complex numbers; returns complex results."""
    n = len(x)
    k_count = n if k_count is None else k_count
    out = []
    for q in range(k_count):
        k = (k0 + q) % n
        re = im = 0.0
        for t in range(n):
            xr = Fraction(float(x[t].real))
            xi = Fraction(float(x[t].imag))
            a, b = cop(twiddle(k * t, n), (xr, xi))
            re += float(a)
            im += float(b)
        out.append(complex(re, im))
    return out


def lag_product(s: complex, r: complex) -> tuple:
    """s (x) conj(r) in exact rational arithmetic (Eq. (6) on the Eq. (11) product)."""
    a = (Fraction(float(s.real)), Fraction(float(s.imag)))
    b = (Fraction(float(r.real)), -Fraction(float(r.imag)))
    return cop(a, b)


def caf(s: list, r: list, tau0: int, n_tau: int, p0: int, n_dop: int) -> list:
    """Eq. (12a): rows l (delay tau0+l), columns q (Doppler bin p0+q mod N)."""
    n = len(s)
    rows = []
    for l in range(n_tau):
        d = tau0 + l
        z = [lag_product(s[i], r[i - d] if i - d >= 0 else 0j) for i in range(n)]
        row = []
        for q in range(n_dop):
            p = (p0 + q) % n
            re = im = 0.0
            for i in range(n):
                a, b = cop(z[i], twiddle(i * p, n))
                re += float(a)
                im += float(b)
            row.append(complex(re, im))
        rows.append(row)
    return rows


def linear_lag_product(s: complex, r: complex) -> tuple:
    """s conj(r), the ordinary product of Eq. (11), in exact rational arithmetic."""
    ar, ai = Fraction(float(s.real)), Fraction(float(s.imag))
    br, bi = Fraction(float(r.real)), -Fraction(float(r.imag))
    return (ar * br - ai * bi, ai * br + ar * bi)


def caf12c(s: list, r: list, tau0: int, n_tau: int, p0: int, n_dop: int) -> list:
    """Eq. (12c): the ordinary lag product, then Eq. (6) with W^{ip}; r[m < 0] = 0."""
    n = len(s)
    rows = []
    for l in range(n_tau):
        d = tau0 + l
        z = [linear_lag_product(s[i], r[i - d] if i - d >= 0 else 0j) for i in range(n)]
        row = []
        for q in range(n_dop):
            p = (p0 + q) % n
            re = im = 0.0
            for i in range(n):
                a, b = cop(z[i], twiddle(i * p, n))
                re += float(a)
                im += float(b)
            row.append(complex(re, im))
        rows.append(row)
    return rows


def caf12b(s: list, r: list, tau0: int, n_tau: int, p0: int, n_dop: int) -> list:
    """Eq. (12b): the Eq. (6) lag product (exact), then the ordinary DFT with W^{ip}."""
    n = len(s)
    rows = []
    for l in range(n_tau):
        d = tau0 + l
        z = [lag_product(s[i], r[i - d] if i - d >= 0 else 0j) for i in range(n)]
        row = []
        for q in range(n_dop):
            p = (p0 + q) % n
            acc = 0j
            for i in range(n):
                wr, wi = twiddle(i * p, n)
                acc += complex(float(z[i][0]), float(z[i][1])) * complex(wr, wi)
            row.append(acc)
        rows.append(row)
    return rows


def nfft(x: list) -> list:
    """Section 3 NFFT: radix-2 decimation in time down to single samples; each butterfly
    X[k] = E[k] + cop(O[k], W_n^k), X[k + n/2] = E[k] - cop(O[k], W_n^k)."""
    n = len(x)
    if n == 1:
        return [(Fraction(float(x[0].real)), Fraction(float(x[0].imag)))]
    E = nfft(x[0::2])
    O = nfft(x[1::2])
    out = [None] * n
    for k in range(n // 2):
        wr, wi = twiddle(k, n)
        t = cop(O[k], (Fraction(wr), Fraction(wi)))
        out[k] = (E[k][0] + t[0], E[k][1] + t[1])
        out[k + n // 2] = (E[k][0] - t[0], E[k][1] - t[1])
    return out
