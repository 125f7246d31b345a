"""The identity behind the sign-split form, checked on the oracle (no GPU).

Section 2, Eq. (1)-(2): x (x) y = x sgn(y) + y sgn(x) for reals, so with the complex
operator of Eq. (6) every term of the Eq. (12a) surface splits as
    z (x) W = csgn(W) z + W csgn(z)        (ordinary complex products),
and the surface is T + D with T = sum_k csgn(W^{pk}) z_k and D = sum_k W^{pk} csgn(z_k).
The split-BF16 sign-split kernels evaluate T by runs of constant csgn(W^{pk}) (it only
changes where pk mod N crosses a multiple of N/4, with a single exact zero there) and D
on the matrix cores. This test evaluates both halves from the oracle's lag rows and the
exact twiddle signs (FP64 sums, run by run for T as the kernel walks them) and compares
T + D with the oracle's surface; it also pins the run rule against the twiddle signs the
oracle computes sample by sample.
"""
import numpy as np
import pytest

import oracle
import synth


def quarter_signs(m, n):
    """csgn(W^m) from the quarter of m (the rule the kernels use), as (re, im) ints."""
    m4 = 4 * m
    q = int(m4 >= n) + int(m4 >= 2 * n) + int(m4 >= 3 * n)
    exact = m4 == q * n
    sc = 1 if q in (0, 3) else -1
    st = -1 if q < 2 else 1
    if exact:
        if q & 1:
            sc = 0
        else:
            st = 0
    return sc, st


@pytest.mark.parametrize("n", [16, 17, 30, 1000, 1002, 4096])
def test_quarter_rule_matches_twiddle_signs(n):
    ts = oracle.twiddle_signs(n, 0, n)  # [bin][sample][re, im] for bins 0..n-1
    for p in range(0, n, max(1, n // 23)):
        for k in range(n):
            assert tuple(ts[p, k]) == quarter_signs((p * k) % n, n), (n, p, k)


def runs(b, k0, k1, n):
    """Runs [ks, ke) of constant csgn(W^{b k}) covering k0 .. k1 - 1."""
    out = []
    k = k0
    while k < k1:
        m = (b * k) % n
        sc, st = quarter_signs(m, n)
        q = int(4 * m >= n) + int(4 * m >= 2 * n) + int(4 * m >= 3 * n)
        if b == 0:
            ln = k1 - k
        elif 4 * m == q * n:
            ln = 1
        else:
            num, den = (q + 1) * n - 4 * m, 4 * b
            ln = -(-num // den)
        ke = min(k1, k + ln)
        out.append((k, ke, sc, st))
        k = ke
    return out


@pytest.mark.parametrize("shape", [(1002, 3, 4, 0, 1002, True), (999, 0, 3, -50, 101, False),
                                   (4096, 5, 3, -256, 512, False), (1200, 0, 3, -96, 192, True)])
def test_sign_split_halves_sum_to_surface(shape):
    n, tau0, n_tau, p0, n_dop, integer = shape
    s, r = synth.random_pair(n, seed=n + 11, zeros=0.1, integer=integer)
    A, sc = oracle.caf(s, r, tau0, n_tau, p0, n_dop)
    chunk = 256
    for t in range(n_tau):
        z, zs = oracle.lag_row(s, r, tau0 + t)
        csz = zs[:, 0] + 1j * zs[:, 1]
        for q in range(0, n_dop, max(1, n_dop // 12)):  # a spread of bins, both signs
            p = (p0 + q) % n
            # T: runs of constant twiddle sign over chunks, prefix sums inside a chunk
            T = 0j
            for c0 in range(0, n, chunk):
                c1 = min(n, c0 + chunk)
                P = np.concatenate([[0], np.cumsum(z[c0:c1])])
                for ks, ke, a, b in runs(p, c0, c1, n):
                    T += complex(a, b) * (P[ke - c0] - P[ks - c0])
            k = np.arange(n)
            W = np.array([oracle.twiddle(int(m), n) for m in (p * k) % n])
            D = np.sum(W * csz)
            got = T + D
            err = abs(got.real - A[t, q].real) + abs(got.imag - A[t, q].imag)
            assert err <= 1e-9 * max(sc[t, q], 1.0), (shape, t, q, got, A[t, q])


def part_runs(b, k0, k1, n, part):
    """Runs of one part of csgn(W^{b k}) alone: the real part changes only where b k mod N
    crosses N/4 or 3N/4, the imaginary part only where it crosses 0 or N/2 (each exactly
    zero on such a point)."""
    out = []
    k = k0
    while k < k1:
        m = (b * k) % n
        q = int(4 * m >= n) + int(4 * m >= 2 * n) + int(4 * m >= 3 * n)
        exact = 4 * m == q * n
        if part == 0:
            s = 1 if q in (0, 3) else -1
            s = 0 if exact and q % 2 == 1 else s
            target = n if q == 0 else (3 * n if q < 3 else 5 * n)
        else:
            s = -1 if q < 2 else 1
            s = 0 if exact and q % 2 == 0 else s
            target = 2 * n if q < 2 else 4 * n
        if b == 0:
            ln = k1 - k
        elif s == 0:
            ln = 1
        else:
            ln = -(-(target - 4 * m) // (4 * b))
        ke = min(k1, k + ln)
        out.append((k, ke, s))
        k = ke
    return out


@pytest.mark.parametrize("n", [17, 30, 1000, 1002, 4096])
def test_part_runs_match_quarter_rule(n):
    for b in list(range(0, min(n, 40))) + list(range(n // 2 - 3, n // 2 + 1)):
        for part in (0, 1):
            got = np.zeros(n, int)
            for ks, ke, s in part_runs(b, 0, n, n, part):
                got[ks:ke] = s
            want = np.array([quarter_signs((b * k) % n, n)[part] for k in range(n)])
            assert np.array_equal(got, want), (n, b, part)
