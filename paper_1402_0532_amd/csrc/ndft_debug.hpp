// Test hook kernel: the exact ternary sign operands the contraction uses.
#pragma once

#include <cstdint>

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

// Test hook kernel: decodes the lag-sign code words that the sign-split plans' lag kernel
// (lsum_kernel) leaves in the workspace, so a test can compare the sign operands the
// matrix kernels actually consume with exact signs. One thread per (delay l, sample k):
// word ((k / 32 * n_cols_pad + l) * 2 + (k / 4) % 2) * 4 + (k / 8) % 4 holds samples
// 4 (k / 4) .. + 3; sample e = k % 4 has its real-part field (sign bit, non-zero bit) at
// bits 15:14, 31:30, 13:12, 29:28 for e = 0..3 and its imaginary-part field four bits
// lower. A field decodes to 0 (00), +1 (01) or -1 (11); the unused pattern 10 is passed
// on as 2 so that a test sees it.
// packed != 0: the packed layout (wpc words per delay row; the fields of samples 0..3 of a
// word 8 bits lower).
__global__ __launch_bounds__(256) void dbg_decode_codes_kernel(const uint32_t *codes, int n_cols_pad, int n,
                                                               long long total, int8_t *lag, int packed,
                                                               long long wpc)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const long long l = idx / n;
    const long long k = idx % n;
    const long long word = packed ? l * wpc + (k >> 3)
                                  : (((k >> 5) * n_cols_pad + l) * 2 + ((k >> 2) & 1)) * 4 + ((k >> 3) & 3);
    const uint32_t c = codes[word];
    const int e = (int)(k & 3);
    const int pos = ((e & 1) ? 30 - 2 * (e >> 1) : 14 - 2 * (e >> 1)) - (packed && !(k & 4) ? 8 : 0);
    const uint32_t fr = (c >> pos) & 3u, fi = (c >> (pos - 4)) & 3u;
    auto dec = [](uint32_t f) -> int8_t { return f == 0u ? 0 : (f == 1u ? 1 : (f == 3u ? -1 : 2)); };
    lag[2 * idx] = dec(fr);
    lag[2 * idx + 1] = dec(fi);
}

} // namespace ndft
