// The Eq. (12b) surface: the lag product of Eq. (6), then the ordinary DFT,
//   A[l][q] = sum_i z_l[i] W^{i p},  z_l[i] = s[i] (x) conj(r[i - d]),  p = p0 + q mod N.
// The outer transform is linear, so it needs no matrix-core contraction: each range row is
// a DFT restricted to the requested bins, computed by decimation in time. With N = M L
// (L the largest power of two dividing N, at most 512) and i = m + M t,
//   A[l][p] = sum_{m < M} W^{m p} Y_m[p mod L],   Y_m[k] = sum_{t < L} z[m + M t] W_L^{t k},
// so one range row costs M length-L FFTs plus M terms per requested bin, instead of N
// terms per bin. A work-group takes one delay and MB consecutive phases m (MB L = 8192
// samples): it forms their lag products (consecutive lanes read consecutive samples),
// runs the MB FFTs in LDS with radix-8/4/2 Stockham passes (each lane holds its
// butterflies' inputs in registers between the two barriers of a pass), and adds its
// phases' share of every requested bin. Shares of the work-groups of a delay are partial
// surfaces, added in a fixed order by dft12b_reduce_kernel (deterministic).
//
// LDS layout: transform j, entry x at j S + x + x / 8 with the row stride S = L + L / 8 + 1
// (L >= 8). The pad after every 8 entries spreads the strided writes of the first passes
// over the banks; the odd row stride spreads the fill, whose lanes run across transforms.
//
// SRC selects what is transformed: DFT_LAG the lag products (the Eq. (12b) surface);
// DFT_SIGNS their exact signs, D(l, p) = sum_i W^{ip} csgn(z_l[i]), the twiddle half of the
// Eq. (12a) sign-split form (see ndft_signsplit.hpp), which its FP32 form takes from here
// instead of the matrix cores; DFT_LIN_SIGNS the exact signs of the ordinary lag product
// s conj(r), the same half of the Eq. (12c) surface. For the halves, bin p = 0 is left out
// (the twiddle-sign kernel sums base 0 whole) and the result is added to the surface the
// reduction of the other half wrote.
//
// FP32 throughout; twiddles come from the two-level table (exact 0 / +-1 at quadrant
// points, a few ulp elsewhere), the FFT's inner twiddles as powers of one table entry.
#pragma once

#include "ndft_device.hpp"

namespace ndft {

constexpr int kDftTile = 8192;    // complex samples per work-group
constexpr int kDftThreads = 512;
constexpr int kDftMaxLog = 9;     // L <= 512
constexpr int DFT_LAG = 0, DFT_SIGNS = 1, DFT_LIN_SIGNS = 2;
// DFT_CODES (whole-row kernel only): the exact signs as the 2-bit codes the twiddle-sign
// kernel wrote (of whichever lag product it formed), read instead of recomputed.
constexpr int DFT_CODES = 3;

struct Dft12bParams {
    const float2 *s, *r;  // complex64 inputs, n samples each
    // the whole-row kernel (L = 512): the inputs with their exact signs, (re, im, sign re,
    // sign im): s4[n] and r4[2 n] (n zeros, then the reference, so r[m < 0] reads 0)
    const float4 *s4, *r4;
    // DFT_CODES: the sign codes in the packed layout (see ndft_signsplit.hpp), code_wpc
    // words per delay row, row l for delay row l; code_bytes of them (< 2^31)
    const uint32_t *codes;
    int code_wpc;
    unsigned code_bytes;
    int n, tau0, n_tau;
    int p0n, n_dop;       // first bin (reduced mod n) and bin count
    int M, MB, n_mg;      // phases, phases per work-group, work-groups per delay
    int tb, n_coarse;     // two-level twiddle table of W^v, v in [0, n)
    float2 *out;          // n_mg == 1: the surface [n_tau][n_dop]; else partials [n_mg][n_tau][n_dop]
    int accumulate;       // n_mg == 1: add to the surface instead of writing it
};

__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 caddf(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csubf(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a times -j
__device__ __forceinline__ float2 cmulnj(float2 a) { return make_float2(a.y, -a.x); }

// padded LDS row stride and entry offset (see above)
template <int LB>
constexpr int dft_row_stride()
{
    return (1 << LB) + ((1 << LB) >> 3) + (LB >= 3 ? 1 : 0);
}
template <int LB>
constexpr int dft_lds_entries()
{
    return (kDftTile >> LB) * dft_row_stride<LB>();
}
__device__ __forceinline__ int dft_pad(int x) { return x + (x >> 3); }

__device__ __forceinline__ float2 table_twiddle(const float2 *coarse, const float2 *fine, int v, int tb)
{
    return cmulf(coarse[v >> tb], fine[v & ((1 << tb) - 1)]);
}

// In-register forward DFTs of size 2, 4, 8: U_s = sum_r u_r e^{-2 pi j r s / R}.
__device__ __forceinline__ void dft2(float2 &a, float2 &b)
{
    const float2 t = a;
    a = caddf(t, b);
    b = csubf(t, b);
}

__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    const float2 t0 = caddf(a0, a2), t1 = csubf(a0, a2);
    const float2 t2 = caddf(a1, a3), t3 = cmulnj(csubf(a1, a3));
    a0 = caddf(t0, t2);
    a2 = csubf(t0, t2);
    a1 = caddf(t1, t3);
    a3 = csubf(t1, t3);
}

template <int R>
__device__ __forceinline__ void small_dft(float2 (&u)[R])
{
    if constexpr (R == 2) {
        dft2(u[0], u[1]);
    } else if constexpr (R == 4) {
        dft4(u[0], u[1], u[2], u[3]);
    } else {
        static_assert(R == 8, "radix 2, 4 or 8");
        // even and odd samples, then U_s = E_s + W8^s O_s, U_{s+4} = E_s - W8^s O_s
        dft4(u[0], u[2], u[4], u[6]);
        dft4(u[1], u[3], u[5], u[7]);
        const float c = 0.70710678118654752f;
        const float2 o1 = make_float2(c * (u[3].x + u[3].y), c * (u[3].y - u[3].x)); // W8 O_1
        const float2 o2 = cmulnj(u[5]);                                              // W8^2 O_2
        const float2 o3 = make_float2(c * (u[7].y - u[7].x), -c * (u[7].x + u[7].y)); // W8^3 O_3
        const float2 e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
        u[0] = caddf(e0, o0);
        u[4] = csubf(e0, o0);
        u[1] = caddf(e1, o1);
        u[5] = csubf(e1, o1);
        u[2] = caddf(e2, o2);
        u[6] = csubf(e2, o2);
        u[3] = caddf(e3, o3);
        u[7] = csubf(e3, o3);
    }
}

// One radix-R Stockham pass over mb transforms of length L = 2^LB held in X[b][t]: the
// butterfly (b, i), i < L / R, with k = i mod p (p the length of the sub-transforms done
// so far) takes x[b][i + r L / R], turns input r by e^{-2 pi j r k / (R p)}, and writes
// its R-point DFT to x[b][(i - k) R + k + r p]. All reads happen before the first write.
template <int R, int LB>
__device__ __forceinline__ void stockham_pass(float2 *X, int mb, int p, int n, const float2 *coarse,
                                              const float2 *fine, int tb, int tid)
{
    constexpr int L = 1 << LB, Q = L / R, S = dft_row_stride<LB>();
    constexpr int CNT = (kDftTile / R + kDftThreads - 1) / kDftThreads;
    float2 u[CNT][R];
    int drow[CNT], dx[CNT]; // destination row start and entry (before the pad)
    const int nb = mb * Q;
    const int vstep = n / (R * p); // W_N^{k n / (R p)} = e^{-2 pi j k / (R p)}
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        const int w = tid + c * kDftThreads;
        drow[c] = -1;
        dx[c] = 0;
        if (w < nb) {
            const int b = w / Q, i = w % Q;
            const int k = i & (p - 1);
            const float2 *src = X + b * S;
#pragma unroll
            for (int r = 0; r < R; ++r) u[c][r] = src[dft_pad(i + r * Q)];
            if (p > 1) {
                const float2 w1 = table_twiddle(coarse, fine, k * vstep, tb);
                float2 wr = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    u[c][r] = cmulf(u[c][r], wr);
                    if (r + 1 < R) wr = cmulf(wr, w1);
                }
            }
            small_dft<R>(u[c]);
            drow[c] = b * S;
            dx[c] = (i - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CNT; ++c)
        if (drow[c] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) X[drow[c] + dft_pad(dx[c] + r * p)] = u[c][r];
        }
    __syncthreads();
}

// Radix 8 while three or more bits remain, then one radix-4 or radix-2 pass.
template <int LB, int REM>
__device__ __forceinline__ void fft_passes(float2 *X, int mb, int p, int n, const float2 *coarse,
                                           const float2 *fine, int tb, int tid)
{
    if constexpr (REM >= 3) {
        stockham_pass<8, LB>(X, mb, p, n, coarse, fine, tb, tid);
        fft_passes<LB, REM - 3>(X, mb, p * 8, n, coarse, fine, tb, tid);
    } else if constexpr (REM == 2) {
        stockham_pass<4, LB>(X, mb, p, n, coarse, fine, tb, tid);
    } else if constexpr (REM == 1) {
        stockham_pass<2, LB>(X, mb, p, n, coarse, fine, tb, tid);
    }
}

// The transformed value of one sample pair (s[i], r[i - d]): the lag product of Eq. (6)
// (DFT_LAG), its exact signs (DFT_SIGNS), or the exact signs of the ordinary lag product
// s conj(r) (DFT_LIN_SIGNS).
template <int SRC>
__device__ __forceinline__ float2 dft_source(float2 a, float2 b)
{
    if constexpr (SRC == DFT_LIN_SIGNS) {
        // s conj(r) from FP32 products: the rounded sum carries the exact sign when it
        // exceeds 2^-22 of the parts' magnitude (each product and the sum are off by at
        // most 2^-24 of their size, or 2^-150 below the normal range, which the 2^-100
        // floor covers); a zero sample gives exact zeros; otherwise FP64, where both
        // FP32 x FP32 products are exact and one rounding of their sum keeps the sign
        const float p1 = a.x * b.x, p2 = a.y * b.y, p3 = a.y * b.x, p4 = a.x * b.y;
        const float zr = p1 + p2, zi = p3 - p4;
        const float mr = fabsf(p1) + fabsf(p2), mi = fabsf(p3) + fabsf(p4);
        const bool zero = (a.x == 0.0f && a.y == 0.0f) || (b.x == 0.0f && b.y == 0.0f);
        const bool sure = fabsf(zr) > 0x1p-22f * mr && mr >= 0x1p-100f && fabsf(zi) > 0x1p-22f * mi &&
                          mi >= 0x1p-100f;
        float2 u = zero ? make_float2(0.0f, 0.0f) : make_float2(sgnf(zr), sgnf(zi));
        if (!zero && !sure) {
            const double sx = a.x, sy = a.y, rx = b.x, ry = b.y;
            const double zr64 = fma(sx, rx, sy * ry), zi64 = fma(sy, rx, -(sx * ry));
            u = make_float2((float)((zr64 > 0.0) - (zr64 < 0.0)), (float)((zi64 > 0.0) - (zi64 < 0.0)));
        }
        return u;
    } else {
        const Lag z = lag_product(a, b);
        return SRC == DFT_SIGNS ? make_float2(z.sr, z.si) : make_float2(z.zr, z.zi);
    }
}

// The same value on the common path only: the lag product's FP32 value (DFT_LAG), or the
// signs of the FP32 values with `unsure` set where the exact sign needs the slow path of
// dft_source (a zero component from non-zero operators, or an ordinary lag product too
// close to cancellation); the caller redoes those samples with dft_source.
template <int SRC>
__device__ __forceinline__ float2 dft_source_fast(float2 a, float2 b, bool &unsure)
{
    if constexpr (SRC == DFT_LIN_SIGNS) {
        const float p1 = a.x * b.x, p2 = a.y * b.y, p3 = a.y * b.x, p4 = a.x * b.y;
        const float zr = p1 + p2, zi = p3 - p4;
        const float mr = fabsf(p1) + fabsf(p2), mi = fabsf(p3) + fabsf(p4);
        const bool zero = (a.x == 0.0f && a.y == 0.0f) || (b.x == 0.0f && b.y == 0.0f);
        const bool sure = fabsf(zr) > 0x1p-22f * mr && mr >= 0x1p-100f && fabsf(zi) > 0x1p-22f * mi &&
                          mi >= 0x1p-100f;
        unsure = unsure || (!zero && !sure);
        return zero ? make_float2(0.0f, 0.0f) : make_float2(sgnf(zr), sgnf(zi));
    } else {
        const float4 s = with_signs(a), r = with_signs(b);
        const float t1 = fmaf(s.x, r.z, r.x * s.z); // s_r (x) r_r
        const float t2 = fmaf(s.y, r.w, r.y * s.w); // s_i (x) r_i
        const float t3 = fmaf(s.y, r.z, r.x * s.w); // s_i (x) r_r
        const float t4 = fmaf(r.y, s.z, s.x * r.w); // r_i (x) s_r
        const float zr = t1 + t2, zi = t3 - t4;
        if constexpr (SRC == DFT_LAG) {
            return make_float2(zr, zi);
        } else {
            unsure = unsure || (zr == 0.0f && t1 != 0.0f) || (zi == 0.0f && t3 != 0.0f);
            return make_float2(sgnf(zr), sgnf(zi));
        }
    }
}

// The Eq. (6) lag product from inputs that carry their signs (see with_signs), FP32 (the
// value dft_source gives for DFT_LAG).
__device__ __forceinline__ float2 lag_value_signed(float4 s, float4 r)
{
    const float t1 = fmaf(s.x, r.z, r.x * s.z); // s_r (x) r_r
    const float t2 = fmaf(s.y, r.w, r.y * s.w); // s_i (x) r_i
    const float t3 = fmaf(s.y, r.z, r.x * s.w); // s_i (x) r_r
    const float t4 = fmaf(r.y, s.z, s.x * r.w); // r_i (x) s_r
    return make_float2(t1 + t2, t3 - t4);
}

// The lag products and the first Stockham pass (p = 1: no inner twiddles) in one step:
// butterfly (b, i) loads its R samples t = i + r L / R of transform b straight from the
// inputs, forms their lag products and writes the R-point DFT to x[b][i R + r]. Lanes run
// over b first, so a wave's loads are runs of consecutive samples.
template <int LB, int SRC>
__device__ __forceinline__ void fill_first_pass(float2 *X, const Dft12bParams &P, int m0, int mb, int d, int tid)
{
    constexpr int L = 1 << LB, S = dft_row_stride<LB>();
    constexpr int R = LB >= 3 ? 8 : (LB == 2 ? 4 : (LB == 1 ? 2 : 1));
    constexpr int Q = L / R;
    constexpr int CNT = kDftTile / R / kDftThreads;
    static_assert(CNT * R * kDftThreads == kDftTile, "whole butterflies per thread");
    float2 sv[CNT][R], rv[CNT][R];
    int bi[CNT], ii[CNT];
    const int nb = mb * Q;
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        const int w = tid + c * kDftThreads;
        bi[c] = -1;
        ii[c] = 0;
        if (w < nb) {
            bi[c] = w % mb;
            ii[c] = w / mb;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sv[c][r] = make_float2(0.0f, 0.0f);
            rv[c][r] = make_float2(0.0f, 0.0f);
            if (bi[c] >= 0) {
                const int idx = m0 + bi[c] + P.M * (ii[c] + r * Q);
                sv[c][r] = P.s[idx];
                if (idx >= d) rv[c][r] = P.r[idx - d];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        if (bi[c] < 0) continue;
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u[r] = dft_source<SRC>(sv[c][r], rv[c][r]);
        }
        if constexpr (R > 1) small_dft<R>(u);
#pragma unroll
        for (int r = 0; r < R; ++r) X[bi[c] * S + dft_pad(ii[c] * R + r)] = u[r];
    }
}

// Grid: x = phase group (MB phases), y strides over the delays. Dynamic LDS: the table.
template <int LB, int SRC>
__global__ __launch_bounds__(kDftThreads) void dft12b_kernel(Dft12bParams P)
{
    constexpr int L = 1 << LB, S = dft_row_stride<LB>();
    __shared__ float2 X[dft_lds_entries<LB>()];
    extern __shared__ float2 tab[];
    float2 *coarse = tab, *fine = tab + P.n_coarse;
    const int tid = threadIdx.x;
    const int n = P.n, M = P.M, mg = blockIdx.x;
    const int m0 = mg * P.MB;
    const int mb = min(P.MB, M - m0);
    build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, kDftThreads);
    for (int l = blockIdx.y; l < P.n_tau; l += gridDim.y) {
        const int d = P.tau0 + l;
        // lag products of samples m0 + j + M t (j < mb, t < L), transformed into X[j]
        fill_first_pass<LB, SRC>(X, P, m0, mb, d, tid);
        __syncthreads(); // also orders the table build before its first use
        constexpr int LB0 = LB >= 3 ? 3 : LB; // bits of the first pass
        fft_passes<LB, LB - LB0>(X, mb, 1 << LB0, n, coarse, fine, P.tb, tid);
        // this group's phases' share of every requested bin: sum_j W^{(m0 + j) p} Y_j[p mod L],
        // the twiddle turned by W^p from one phase to the next and taken afresh from the
        // table every 16 phases (the rounding of the turns stays a few ulp)
        float2 *dst = P.out + ((size_t)mg * P.n_tau + l) * P.n_dop;
        for (int q = tid; q < P.n_dop; q += kDftThreads) {
            int p = P.p0n + q;
            p = p >= n ? p - n : p;
            const int kk = dft_pad(p & (L - 1));
            int v = (int)(((unsigned long long)(unsigned)m0 * (unsigned)p) % (unsigned)n);
            const float2 step = table_twiddle(coarse, fine, p, P.tb);
            float2 acc = make_float2(0.0f, 0.0f);
            float2 w = make_float2(1.0f, 0.0f);
            for (int j = 0; j < mb; ++j) {
                if ((j & 15) == 0) {
                    w = table_twiddle(coarse, fine, v, P.tb);
                    v = (int)(((long long)v + 16LL * p) % n);
                }
                const float2 y = X[j * S + kk];
                acc.x = fmaf(w.x, y.x, fmaf(-w.y, y.y, acc.x));
                acc.y = fmaf(w.x, y.y, fmaf(w.y, y.x, acc.y));
                w = cmulf(w, step);
            }
            if (SRC != DFT_LAG && p == 0) acc = make_float2(0.0f, 0.0f);
            if (P.accumulate) acc = caddf(acc, dst[q]);
            dst[q] = acc;
        }
        __syncthreads(); // X is refilled for the next delay
    }
}

// A[e] = sum over the phase groups g = 0 .. n_mg - 1 of part[g][e], in that order.
// accumulate: A[e] += that sum (A[e] first, then the groups in order).
__global__ __launch_bounds__(256) void dft12b_reduce_kernel(const float2 *part, int n_mg, long long cells,
                                                            float2 *A, int accumulate)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= cells) return;
    float2 acc = accumulate ? A[e] : make_float2(0.0f, 0.0f);
    for (int g = 0; g < n_mg; ++g) acc = caddf(acc, part[(long long)g * cells + e]);
    A[e] = acc;
}

} // namespace ndft
