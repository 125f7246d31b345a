"""The identity behind the sign-split form, checked on the oracle (no GPU).

Section 2, Eq. (1)-(2): x (x) y = x sgn(y) + y sgn(x) for reals, so with the complex
operator of Eq. (6) every term of the Eq. (12a) surface splits as
    z (x) W = csgn(W) z + W csgn(z)        (ordinary complex products),
and the surface is T + D with T = sum_k csgn(W^{pk}) z_k and D = sum_k W^{pk} csgn(z_k).
The split-BF16 sign-split kernels evaluate T by runs of constant csgn(W^{pk}) (it only
changes where pk mod N crosses a multiple of N/4, with a single exact zero there) and D
on the matrix cores. This test evaluates both halves from the oracle's lag rows and the
exact twiddle signs (FP64 sums, run by run for T as the kernel walks them) and compares
T + D with the oracle's surface; it also pins the crossing walk of the kernel (the next sign
change from a remainder, the exact zeros, the P / R prefix tables) against the twiddle signs
the oracle computes sample by sample.
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


@pytest.mark.parametrize("form", ["12a", "12c"])
@pytest.mark.parametrize("shape", [(1002, 3, 4, 0, 1002, True), (999, 0, 3, -50, 101, False),
                                   (4096, 5, 3, -256, 512, False), (1200, 0, 3, -96, 192, True)])
def test_sign_split_halves_sum_to_surface(shape, form):
    """Both surfaces: Eq. (12a) (lag product by Eq. (6)) and Eq. (12c) (ordinary lag
    product); the split only needs the lag values and their exact signs."""
    n, tau0, n_tau, p0, n_dop, integer = shape
    s, r = synth.random_pair(n, seed=n + 11, zeros=0.1, integer=integer)
    surface, row = (oracle.caf, oracle.lag_row) if form == "12a" else (oracle.caf12c, oracle.lag_row_lin)
    A, sc = surface(s, r, tau0, n_tau, p0, n_dop)
    chunk = 256
    for t in range(n_tau):
        z, zs = row(s, r, tau0 + t)
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


def first_crossing(b, kb, n, part):
    """The walker state at sample kb: offset of the next crossing at or after kb, its rem
    (4b k_i minus the crossing value; 0 when the crossing sample is the exact zero) and the
    sign just before it. Crossings of the real part lie at u = N + 2N i, those of the
    imaginary part at u = 2N i, with u = 4 b k."""
    if b == 0:
        return 1 << 30, 1, (1 if part == 0 else 0)
    fb = 4 * b
    w = (4 * ((b * kb) % n) - fb) % (4 * n)  # u of sample kb - 1, mod 4N
    if part == 0:
        cu = n if w < n else (3 * n if w < 3 * n else 5 * n)
        sg = -1 if cu == 3 * n else 1
    else:
        cu = 2 * n if w < 2 * n else 4 * n
        sg = -1 if cu == 2 * n else 1
    d = cu - w
    cq = -(-d // fb)
    return cq - 1, cq * fb - d, sg


def crossing_step(nk, rem, sg, b, n):
    """The next crossing: 2N / 4b samples on, in whole samples by the remainder."""
    fb = 4 * b
    q0, r0 = (2 * n) // fb, (2 * n) % fb
    t = rem - r0
    return nk + q0 + (1 if t < 0 else 0), (t + fb if t < 0 else t), -sg


def walk_signs(b, kb, k1, n, part):
    """Per-sample signs of one part over kb .. k1 - 1 rebuilt from the crossings alone."""
    out = np.zeros(k1 - kb, int)
    nk, rem, sg = first_crossing(b, kb, n, part)
    k = 0
    while k < k1 - kb:
        stop = min(nk, k1 - kb)
        out[k:stop] = sg
        k = stop
        if k >= k1 - kb:
            break
        if rem == 0:  # exact: the crossing sample itself is zero
            out[k] = 0
            k += 1
        nk, rem, sg = crossing_step(nk, rem, sg, b, n)
    return out


@pytest.mark.parametrize("n", [17, 30, 1000, 1002, 4096])
def test_crossing_walk_matches_quarter_rule(n):
    bases = sorted(set(list(range(0, min(n // 2 + 1, 40))) + list(range(n // 2 - 3, n // 2 + 1))))
    for b in bases:
        want = [np.array([quarter_signs((b * k) % n, n)[part] for k in range(2 * n)]) for part in (0, 1)]
        for kb in (0, 1, 5, n // 4, n // 2 + 1, n - 1, n + 3):
            for part in (0, 1):
                got = walk_signs(b, kb, 2 * n, n, part)
                assert np.array_equal(got, want[part][kb:]), (n, b, kb, part)


@pytest.mark.parametrize("shape", [(4096, 7, 256), (1000, 3, 256), (65536, 0, 256), (1200, 11, 64)])
def test_crossing_tables_give_twiddle_sign_sums(shape):
    """The sum the kernel forms over a block that starts at kb, chunk by chunk: for each
    crossing the sign before it times 2 P(k) (or R(k) = P(k) + P(k + 1) when exact), P the
    prefix sum within the chunk (each chunk's table starts from 0), plus, per chunk, the sign
    after its last crossing times the chunk total, equals sum_k csgn(W^{bk}) z_k (FP64,
    random z)."""
    n, kb, chunk = shape
    rng = np.random.default_rng(n + kb)
    nch = 3
    z = rng.standard_normal(nch * chunk) + 1j * rng.standard_normal(nch * chunk)
    k = kb + np.arange(nch * chunk)
    for b in sorted(set([0, 1, 2, 3, 5, 64, 127, 128, 129, n // 256, n // 8 - 1, n // 2])):
        sc = np.array([quarter_signs((b * int(kk)) % n, n) for kk in k])
        want = np.sum(sc[:, 0] * z) + 1j * np.sum(sc[:, 1] * z)
        got = [0j, 0j]
        for part in (0, 1):
            nk, rem, sg = first_crossing(b, kb, n, part)
            for c in range(nch):
                zc = z[c * chunk:(c + 1) * chunk]
                P = np.concatenate([[0], np.cumsum(zc)])
                R = P[:-1] + P[1:]
                while nk < chunk:
                    got[part] += sg * (R[nk] if rem == 0 else 2 * P[nk])
                    nk, rem, sg = crossing_step(nk, rem, sg, b, n)
                got[part] += sg * P[chunk]
                nk -= chunk
        total = got[0] + 1j * got[1]
        assert abs(total - want) <= 1e-9 * (1 + np.sum(np.abs(z))), (shape, b, total, want)


def test_chunk_local_sums_round_less_on_dc_rows():
    """Why the prefix sums restart at every chunk: on a row whose values keep one sign,
    block-wide prefix sums grow with the block while T stays small, and the FP32 rounding
    of every crossing term grows with them; chunk-local sums keep every term within one
    chunk's sum. Modelled in FP32 (numpy float32 cumulative sums) against FP64."""
    n, kb, chunk, nch = 65536, 0, 256, 32
    rng = np.random.default_rng(5)
    z = (1.0 + 0.01 * rng.standard_normal(nch * chunk)).astype(np.float32)
    b = n // 256  # the largest base the sign-split plans admit
    k = kb + np.arange(nch * chunk)
    sc = np.array([quarter_signs((b * int(kk)) % n, n)[0] for kk in k], np.float64)
    want = float(np.sum(sc * z.astype(np.float64)))

    def model(local):
        nk, rem, sg = first_crossing(b, kb, n, 0)
        acc = np.float32(0.0)
        g = np.float32(0.0)
        for c in range(nch):
            zc = z[c * chunk:(c + 1) * chunk]
            P = np.concatenate([[np.float32(0.0)], np.cumsum(zc, dtype=np.float32)]) + (np.float32(0.0) if local else g)
            P = P.astype(np.float32)
            R = (P[:-1] + P[1:]).astype(np.float32)
            while nk < chunk:
                acc = np.float32(acc + np.float32(sg) * (R[nk] if rem == 0 else np.float32(2.0) * P[nk]))
                nk, rem, sg = crossing_step(nk, rem, sg, b, n)
            if local:
                acc = np.float32(acc + np.float32(sg) * P[chunk])
            g = P[chunk]
            nk -= chunk
        if not local:
            acc = np.float32(acc + np.float32(sg) * g)
        return float(acc)

    scale = float(np.sum(np.abs(z)))
    e_local = abs(model(True) - want) / scale
    e_block = abs(model(False) - want) / scale
    assert e_local <= 2e-7
    assert e_local < e_block
