// Device arithmetic of the NDFT hot path on gfx950: exact ternary signs, the lag
// product of Eq. (6) in sign-split form, twiddle signs from integer quadrant tests and
// twiddle values from a two-level table.
//
// The kernels rely on an exact identity of the paper's operator (Eq. (1)-(2)):
//     a (x) b = sign(a b)(|a| + |b|) = a sign(b) + b sign(a)
// (check the nine sign cases; both sides are 0 when either operand is 0). Applied to
// the four real operators of Eq. (6) it gives, with csgn(a) = sign(a_r) + j sign(a_i),
//     a (x) b = csgn(a) b + a csgn(b)          (ordinary complex products),
// so an NDFT (Eq. (7)) is  X = S x + F csgn(x)  with F the DFT matrix and S = csgn(F)
// ternary. Products with a ternary operand are exact, which is what lets the dense
// part run on matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ndft {

// Ternary sign of a float from its bits: +0 and -0 give 0, denormals give +-1, so the
// result does not depend on flush-to-zero settings (Eq. (2): sign 0 "otherwise").
__device__ __forceinline__ float sgnf(float x)
{
    uint32_t u = __float_as_uint(x);
    float one = __uint_as_float((u & 0x80000000u) | 0x3f800000u);
    return (u << 1) ? one : 0.0f;
}

__device__ __forceinline__ int isgn(int v) { return min(max(v, -1), 1); }

// Exact sign of (a + b) - (c + d) for finite a, b, c, d >= 0 given as floats.
// In FP64 each pair sum is split exactly into value + error (Knuth's TwoSum). Rounding
// to nearest is monotone, so unequal rounded sums order the exact sums; equal rounded
// sums leave the difference of the two error terms, which FP64 compares exactly.
__device__ __forceinline__ int cmp_sum_exact(float a, float b, float c, float d)
{
    double A = a, B = b, C = c, D = d;
    double x = A + B;
    double bx = x - A;
    double ax = x - bx;
    double xe = (A - ax) + (B - bx);
    double y = C + D;
    double by = y - C;
    double ay = y - by;
    double ye = (C - ay) + (D - by);
    if (x != y) return x > y ? 1 : -1;
    return xe > ye ? 1 : (xe < ye ? -1 : 0);
}

// Lag product z = s (x) conj(r) of Eq. (6) (the conjugate is that of Eq. (11)) and the
// exact signs of its components.
//   z_r = s_r(x)r_r - s_i(x)(-r_i) = s_r(x)r_r + s_i(x)r_i
//   z_i = s_i(x)r_r + (-r_i)(x)s_r = s_i(x)r_r - r_i(x)s_r
// Each real operator x(x)y = x sign(y) + y sign(x) is one rounding of +-(|x|+|y|).
// FP32 rounding is monotone, so a non-zero FP32 result carries the exact sign; a zero
// result from two non-zero operators is resolved by the exact comparison above.
struct Lag {
    float zr, zi; // value (FP32)
    float sr, si; // exact sign of each component, in {-1, 0, +1}
};

// Sample packed with its exact component signs: (re, im, g sign re, g sign im). The
// kernels use g = 1, or g = 1/2 where they want every Eq. (1) operator halved (an exact
// scaling: each operator value x g sign(y) + y g sign(x) is then half the exact one).
__device__ __forceinline__ float4 with_signs(float2 x, float g = 1.0f)
{
    return make_float4(x.x, x.y, g * sgnf(x.x), g * sgnf(x.y));
}

// Lag product from signed samples s = (s_r, s_i, sgn s_r, sgn s_i), r likewise.
__device__ __forceinline__ Lag lag_product4(float4 s, float4 r)
{
    float t1 = fmaf(s.x, r.z, r.x * s.z); // s_r (x) r_r
    float t2 = fmaf(s.y, r.w, r.y * s.w); // s_i (x) r_i
    float t3 = fmaf(s.y, r.z, r.x * s.w); // s_i (x) r_r
    float t4 = fmaf(r.y, s.z, s.x * r.w); // r_i (x) s_r
    Lag z;
    z.zr = t1 + t2;
    z.zi = t3 - t4;
    z.sr = sgnf(z.zr);
    z.si = sgnf(z.zi);
    if (z.zr == 0.0f && t1 != 0.0f) {
        int c = cmp_sum_exact(fabsf(s.x), fabsf(r.x), fabsf(s.y), fabsf(r.y));
        z.sr = sgnf(t1) * (float)c;
    }
    if (z.zi == 0.0f && t3 != 0.0f) {
        int c = cmp_sum_exact(fabsf(s.y), fabsf(r.x), fabsf(r.y), fabsf(s.x));
        z.si = sgnf(t3) * (float)c;
    }
    return z;
}

__device__ __forceinline__ Lag lag_product(float2 s, float2 r)
{
    return lag_product4(with_signs(s), with_signs(r));
}

// Identity producer (plain NDFT of x): a signed sample as it is.
__device__ __forceinline__ Lag identity_entry(float4 x)
{
    Lag z;
    z.zr = x.x;
    z.zi = x.y;
    z.sr = x.z;
    z.si = x.w;
    return z;
}

// Signs of the twiddle W^m = e^{-j 2 pi m / N} = cos(2 pi m/N) - j sin(2 pi m/N),
// 0 <= m < N, from integer comparisons on u = 4m (exact, 0 where the math gives 0):
//   sign cos  = sign(u - N) * sign(u - 3N)       (+ for u < N or u > 3N)
//   sign(-sin) = sign(u - 2N) * sign(u)          (- for 0 < u < 2N)
struct TwSign {
    int c, t;
};

__device__ __forceinline__ TwSign twiddle_sign(int m, int n)
{
    int u = m << 2;
    TwSign s;
    s.c = __mul24(isgn(u - n), isgn(u - 3 * n));
    s.t = __mul24(isgn(u - 2 * n), min(u, 1));
    return s;
}

// Two-level twiddle table in LDS: W^m = coarse[m >> tb] * fine[m & (2^tb - 1)] with
// coarse[q] = W^{q 2^tb}, fine[k] = W^k, each entry {cos, -sin} rounded from FP64.
// The FP32 product is within a few ulp of W^m; components whose exact value is 0 are
// forced to 0 from the integer sign.
__device__ __forceinline__ float2 twiddle_value(const float2 *__restrict__ coarse,
                                                const float2 *__restrict__ fine, int m, int tb,
                                                TwSign sg)
{
    float2 a = coarse[m >> tb];
    float2 b = fine[m & ((1 << tb) - 1)];
    float c = fmaf(a.x, b.x, -a.y * b.y);
    float t = fmaf(a.x, b.y, a.y * b.x);
    c = sg.c ? c : 0.0f;
    t = sg.t ? t : 0.0f;
    return make_float2(c, t);
}

// Fill the two-level table (all threads of the block take part; caller syncs). The fine
// entries are multiplied by fine_scale (a power of two: the products are scaled exactly).
__device__ __forceinline__ void build_twiddle_tables(float2 *coarse, float2 *fine, int n, int tb,
                                                     int n_coarse, int tid, int nthreads, float fine_scale = 1.0f)
{
    int nf = 1 << tb;
    for (int idx = tid; idx < n_coarse + nf; idx += nthreads) {
        long long m = idx < n_coarse ? ((long long)idx << tb) : (long long)(idx - n_coarse);
        float2 w;
        if ((4 * m) % n == 0) { // quadrant points: exactly 1, -j, -1, +j
            const int q = (int)((4 * m) / n) & 3;
            w = q == 0 ? make_float2(1.f, 0.f)
                       : (q == 1 ? make_float2(0.f, -1.f) : (q == 2 ? make_float2(-1.f, 0.f) : make_float2(0.f, 1.f)));
        } else {
            double x = 2.0 * (double)m / (double)n; // angle / pi
            double sn, cs;
            sincospi(x, &sn, &cs);
            w = make_float2((float)cs, (float)(-sn));
        }
        if (idx < n_coarse)
            coarse[idx] = w;
        else
            fine[idx - n_coarse] = make_float2(w.x * fine_scale, w.y * fine_scale);
    }
}

} // namespace ndft
