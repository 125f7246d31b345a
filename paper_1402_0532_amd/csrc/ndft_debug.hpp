// Test hook kernel: the exact ternary sign operands the contraction uses.
#pragma once

#include "ndft_device.hpp"

namespace ndft {

// idx < ntw:      tw[idx] for (q, i) = (idx / n, idx % n): signs of W^{(p0n + q) i mod n}
// idx - ntw:      lag[.] for (l, i): signs of s[i] (x) conj(r[i - tau0 - l]), r[m < 0] = 0
__global__ __launch_bounds__(256) void dbg_signs_kernel(const float2 *s, const float2 *r, int n, int tau0, int p0n,
                                                        long long ntw, long long nlag, int8_t *tw, int8_t *lag)
{
    long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx < ntw) {
        long long q = idx / n;
        int i = (int)(idx % n);
        long long p = (p0n + q) % n;
        int m = (int)((p * i) % n);
        TwSign g = twiddle_sign(m, n);
        tw[2 * idx] = (int8_t)g.c;
        tw[2 * idx + 1] = (int8_t)g.t;
        return;
    }
    idx -= ntw;
    if (idx >= nlag) return;
    int l = (int)(idx / n);
    int i = (int)(idx % n);
    int d = tau0 + l;
    float2 rv = i - d >= 0 ? r[i - d] : make_float2(0.0f, 0.0f);
    Lag z = lag_product(s[i], rv);
    lag[2 * idx] = (int8_t)z.sr;
    lag[2 * idx + 1] = (int8_t)z.si;
}

} // namespace ndft
