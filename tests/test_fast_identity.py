"""CPU model of the regrouping behind the fast exact transform (plan fp32x_fast_exact),
checked against the literal NDFT of Eq. (7) in the FP64 oracle.

With the identity of Eq. (6), X = S z + F csgn(z) (S = csgn(F)). For N = 2^n the first
term T[p] = sum_k phi(p k mod N) z_k, phi(m) = csgn(W^m), is regrouped as
  p = 2^v u (u odd):  T[p] = y_v[0] + sum_w C_{N / 2^(v+w)}(y_v[2^w .])[u],
with y_v the row folded to length N / 2^v and C_L(y)[u] = sum_{t odd < L} phi_L(u t) y[t]
a cyclic correlation over the odd residues mod L = {(-1)^e 5^a}. This model evaluates every
correlation directly (no FFT) in exact index arithmetic, so a wrong fold, group order or
residue map fails here, apart from the GPU kernels that evaluate the same sums with FFTs.
"""
import numpy as np
import pytest

import oracle


def phi(m, n):
    """csgn(W^m) from the quadrant of m (exact zeros on the axes)."""
    m = np.asarray(m) % n
    c = np.where((4 * m < n) | (4 * m > 3 * n), 1, np.where((4 * m == n) | (4 * m == 3 * n), 0, -1))
    t = np.where((m == 0) | (2 * m == n), 0, np.where(2 * m < n, -1, 1))
    return c + 1j * t


def odd_group(L):
    """The odd residues mod L in the order (e, a) -> (-1)^e 5^a, a < L / 4 ({1} for L = 2)."""
    if L == 2:
        return np.array([1])
    q = L // 4
    g = np.array([pow(5, a, L) for a in range(q)])
    return np.concatenate([g, (L - g) % L])


def model_T(z):
    n = len(z)
    lg = n.bit_length() - 1
    T = np.zeros(n, complex)
    T[0] = z.sum()
    for v in range(lg):
        M = n >> v
        y = z.reshape(-1, M).sum(axis=0)  # fold: y[k] = sum_j z[k + j M]
        u = np.arange(1, M, 2)
        acc = np.full(len(u), y[0], complex)  # k' = 0: phi = 1
        for w in range(lg - v):
            L = M >> w
            G = odd_group(L)
            assert sorted(G.tolist()) == list(range(1, L, 2))  # a permutation of the odd residues
            # C[u] = sum over t in the group of phi_L(u t) y[2^w t], u taken mod L
            C = {int(g1): np.sum(phi(g1 * G, L) * y[G << w]) for g1 in G}
            acc += np.array([C[int(x % L)] for x in u])
        T[u << v] = acc
    return T


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128])
def test_regrouped_twiddle_sign_half_equals_the_ndft(n):
    rng = np.random.default_rng(n)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    x.real[rng.uniform(size=n) < 0.2] = 0.0
    z = x.astype(np.complex128)
    sig = np.sign(z.real) + 1j * np.sign(z.imag)
    X = model_T(z) + np.fft.fft(sig)  # S z + F csgn(z)
    Xo, scale = oracle.ndft(z[None, :])
    err = (np.abs(X.real - Xo[0].real) + np.abs(X.imag - Xo[0].imag)) / np.where(scale[0] > 0, scale[0], 1)
    assert err.max() < 1e-12


def test_group_of_powers_of_five():
    # 5 has order L / 4 mod L = 2^l (l >= 3), and +-5^a covers the odd residues once
    for l in range(3, 13):
        L = 1 << l
        G = odd_group(L)
        assert len(set(G.tolist())) == L // 2 and all(g % 2 == 1 for g in G)
        assert pow(5, L // 4, L) == 1 and pow(5, L // 8, L) != 1
