// NFFT of Section 3 (Eq. (10)): the radix-2 decimation-in-time FFT with the twiddle
// product of every butterfly replaced by the complex operator of Eq. (6),
//   X[k] = E[k] + O[k] (x) W_n^k,   X[k + n/2] = E[k] - O[k] (x) W_n^k,
// recursively down to single samples (W_n^0 = 1 included, so no multiplication is left;
// E / O are the NFFTs of the even / odd samples). A work-group takes 8192 / N rows at a
// time (one for N = 8192): the rows and a twiddle table W_N^m (m < N/2, FP64 cosine and
// sine rounded once to FP32, exact at the quadrant points) live in LDS, and log2 N
// radix-2 Stockham passes over all its rows, which evaluate the
// recursion's butterflies in the same operations (each lane holds its butterflies'
// outputs between the two barriers of a pass). The operator is not associative, so
// butterflies cannot be merged into higher radices. FP32 adds only: the result is the
// recursion evaluated in FP32, bit for bit.
#pragma once

#include <hip/hip_runtime.h>

namespace ndft {

constexpr int kNfftMaxN = 8192;
constexpr int kNfftThreads = 1024;

// Eq. (1) with the sign table of Eq. (2), FP32: one rounding
__device__ __forceinline__ float rop32(float a, float b)
{
    const float m = fabsf(a) + fabsf(b);
    const bool pos = (a > 0.0f && b > 0.0f) || (a < 0.0f && b < 0.0f);
    const bool neg = (a > 0.0f && b < 0.0f) || (a < 0.0f && b > 0.0f);
    return pos ? m : (neg ? -m : 0.0f);
}

// Eq. (6): o (x) w
__device__ __forceinline__ float2 cop32(float2 o, float2 w)
{
    return make_float2(rop32(o.x, w.x) - rop32(o.y, w.y), rop32(o.y, w.x) + rop32(w.y, o.x));
}

// Dynamic LDS: rpb rows of n entries, then n / 2 twiddles. Row groups g = blockIdx.x,
// + gridDim.x, ... of rpb = 8192 / n rows each (n a power of two).
__global__ __launch_bounds__(kNfftThreads) void nfft_kernel(const float2 *__restrict__ x, float2 *__restrict__ X,
                                                           long long batch, int n, int rpb)
{
    extern __shared__ float2 nfft_lds[];
    float2 *buf = nfft_lds, *tw = nfft_lds + (size_t)rpb * n;
    constexpr int CNT = kNfftMaxN / 2 / kNfftThreads;
    const int tid = threadIdx.x, h = n >> 1;
    const int lh = 31 - __builtin_clz(max(h, 1)); // log2 of h (h >= 1 when n >= 2)
    for (int m = tid; m < h; m += kNfftThreads) {
        float2 w;
        if ((4 * m) % n == 0) { // quadrant points: exactly 1, -j
            w = (4 * m) / n == 0 ? make_float2(1.0f, 0.0f) : make_float2(0.0f, -1.0f);
        } else {
            const double th = 2.0 * 3.14159265358979323846 * (double)m / (double)n;
            w = make_float2((float)cos(th), (float)(-sin(th)));
        }
        tw[m] = w;
    }
    for (long long b0 = (long long)blockIdx.x * rpb; b0 < batch; b0 += (long long)gridDim.x * rpb) {
        const int rows = (int)min((long long)rpb, batch - b0);
        const float2 *xr = x + b0 * n;
        for (int i = tid; i < rows * n; i += kNfftThreads) buf[i] = xr[i];
        __syncthreads(); // also orders the table before its first use
        for (int p = 1; p < n; p <<= 1) {
            float2 y0[CNT], y1[CNT];
            int dst[CNT];
            const int tstep = n / (2 * p); // W_{2p}^k = W_n^{k n / 2p}
#pragma unroll
            for (int c = 0; c < CNT; ++c) {
                const int w = tid + c * kNfftThreads; // butterfly i of row r
                const int r = w >> lh, i = w & (h - 1);
                dst[c] = -1;
                if (r < rows) {
                    const int k = i & (p - 1);
                    const float2 *row = buf + r * n;
                    const float2 u0 = row[i], t = cop32(row[i + h], tw[k * tstep]);
                    y0[c] = make_float2(u0.x + t.x, u0.y + t.y);
                    y1[c] = make_float2(u0.x - t.x, u0.y - t.y);
                    dst[c] = r * n + (i - k) * 2 + k;
                }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CNT; ++c)
                if (dst[c] >= 0) {
                    buf[dst[c]] = y0[c];
                    buf[dst[c] + p] = y1[c];
                }
            __syncthreads();
        }
        float2 *Xr = X + b0 * n;
        for (int i = tid; i < rows * n; i += kNfftThreads) Xr[i] = buf[i];
        __syncthreads(); // buf is refilled for the next row
    }
}

} // namespace ndft
