// NFFT of Section 3 (Eq. (10)): the radix-2 decimation-in-time FFT whose butterflies carry
// the operator of Eq. (6). Two readings of the printed equation:
//   OUTER = false (the multiplication-free transform the text describes): every twiddle
//     product of a butterfly is the operator, X[k] = E[k] + O[k] (x) W_n^k, X[k + n/2] =
//     E[k] - O[k] (x) W_n^k, recursively down to single samples (W_n^0 = 1 included);
//   OUTER = true (the equation as printed): the twiddle in front of the odd half is an
//     ordinary complex product at every level, X[k] = E[k] + W_n^k O[k], and the operator
//     sits in the sums themselves, whose length-1 terms at the bottom are x (x) 1.
// E / O are the transforms of the even / odd samples. Both are evaluated butterfly by
// butterfly in FP32 in the recursion's own operations (products and sums rounded one by
// one, no fused multiply-add), so the result is the FP32 recursion bit for bit; twiddles
// are W_n^m = e^{-j 2 pi m / n} rounded once from FP64, exact at the quadrant points.
//
// Rows of up to 8192 samples are transformed in LDS by one work-group (8192 / L rows at a
// time): the log2 L radix-2 levels go up to three per Stockham pass (nfft_group_pass: the
// same butterflies, run in registers between the pass's two LDS barriers). LDS entry e of
// the rows sits at e + e / 8 (a pad after every 8: the first pass writes each lane's 8
// outputs side by side, which would put 16 lanes on 2 bank pairs), and the twiddles of
// level P (sub-length P, W_{2P}^k for k < P) are stored contiguously at P - 1 + k, so the
// lanes of a butterfly level read consecutive entries. Longer rows (n = 2^s L, L = 8192) take the recursion's lower
// levels in LDS, as the transforms of the 2^s decimated sequences x[j + 2^s t], and its top
// s levels as passes over global memory (nfft_combine_kernel): at stride S the transform of
// x[j::S] is the combination of those of x[j::2S] and x[j + S::2S].
#pragma once

#include <hip/hip_runtime.h>

namespace ndft {

constexpr int kNfftMaxN = 8192;            // rows transformed in LDS
constexpr int kNfftMaxLong = 1 << 24;      // longest row
constexpr int kNfftThreads = 1024;

// Eq. (1) with the sign table of Eq. (2), FP32: one rounding
// (|a| + |b| with the sign of a b, 0 when an operand is zero of either sign: the sign bit of
// the non-zero sum is the exclusive or of the operands' sign bits)
__device__ __forceinline__ float rop32(float a, float b)
{
    const float m = fabsf(a) + fabsf(b);
    const unsigned sg = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return (a == 0.0f || b == 0.0f) ? 0.0f : __uint_as_float(__float_as_uint(m) | sg);
}

// Eq. (6): o (x) w
__device__ __forceinline__ float2 cop32(float2 o, float2 w)
{
    return make_float2(rop32(o.x, w.x) - rop32(o.y, w.y), rop32(o.y, w.x) + rop32(w.y, o.x));
}

// ordinary complex product, each product and sum rounded on its own (no contraction into
// fused multiply-adds)
__device__ __forceinline__ float2 cmul_rn(float2 o, float2 w)
{
#pragma clang fp contract(off)
    const float p1 = o.x * w.x, p2 = o.y * w.y, p3 = o.x * w.y, p4 = o.y * w.x;
    return make_float2(p1 - p2, p3 + p4);
}

// W_n^m, m < n / 2
__device__ __forceinline__ float2 nfft_twiddle(int m, int n)
{
    if ((4LL * m) % n == 0) // quadrant points: exactly 1, -j
        return (4LL * m) / n == 0 ? make_float2(1.0f, 0.0f) : make_float2(0.0f, -1.0f);
    const double th = 2.0 * 3.14159265358979323846 * (double)m / (double)n;
    return make_float2((float)cos(th), (float)(-sin(th)));
}

// The twiddled odd term of a butterfly in the chosen reading.
template <bool OUTER>
__device__ __forceinline__ float2 nfft_odd(float2 o, float2 w)
{
    return OUTER ? cmul_rn(o, w) : cop32(o, w);
}

__device__ __forceinline__ int bitrev_bits(int q, int bits)
{
    return (int)(__brev((unsigned)q) >> (32 - bits)) & ((1 << bits) - 1);
}

// LDS slot of row entry e (one pad entry after every 8)
__device__ __forceinline__ int nfft_pad(int e) { return e + (e >> 3); }

// The per-level twiddle table of length-n rows in LDS: entry j < n - 1 holds, for level
// P = the largest power of two <= j + 1 and k = j + 1 - P, W_{2P}^k = W_n^{k n / (2P)}. The
// top level (P = n / 2: W_n^k) is evaluated, the lower levels are copied from it.
__device__ __forceinline__ void nfft_level_table(float2 *tw, int n, int tid)
{
    const int h = n >> 1;
    float2 *top = tw + h - 1;
    for (int k = tid; k < h; k += kNfftThreads) top[k] = nfft_twiddle(k, n);
    __syncthreads();
    for (int j = tid; j < h - 1; j += kNfftThreads) {
        const int P = 1 << (31 - __builtin_clz(j + 1));
        tw[j] = top[(j + 1 - P) * (h / P)];
    }
}

// LR consecutive radix-2 levels of the recursion, sub-length p -> 2^LR p, in one LDS round
// trip (Stockham order). Group (row, i), i < n / R: k = i mod p; the thread loads the R
// entries i + q n / R, which the LR levels combine among themselves only, and runs their
// butterflies in registers with the operations of the radix-2 passes: at level l (sub-length
// P = 2^l p) pair m < R / 2 takes (v[m], v[m + R/2]) with twiddle W_{2P}^{k + rev_l(m mod 2^l) p}
// and gives v'[2m] = v[m] + t, v'[2m + 1] = v[m] - t; value q then belongs at
// (i - k) R + k + rev_LR(q) p (rev_b: the b-bit reversal). The same butterflies on the same
// operands as log2 R radix-2 passes, so the result is unchanged bit for bit.
template <bool OUTER, int LR>
__device__ __forceinline__ void nfft_group_pass(float2 *buf, int rows, int n, int lg, int p, const float2 *tw,
                                                int tid)
{
    constexpr int R = 1 << LR, H = R / 2;
    constexpr int CNT = kNfftMaxN / R / kNfftThreads;
    const int lnr = lg - LR; // log2 of the groups per row
    const int nr = 1 << lnr;
    float2 v[CNT][R];
    int base[CNT];
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        const int w = tid + c * kNfftThreads;
        const int r = w >> lnr, i = w & (nr - 1);
        base[c] = -1;
        if (r < rows) {
            const int k = i & (p - 1);
            const int row = r * n;
#pragma unroll
            for (int q = 0; q < R; ++q) v[c][q] = buf[nfft_pad(row + i + q * nr)];
#pragma unroll
            for (int l = 0; l < LR; ++l) {
                const float2 *twl = tw + (p << l) - 1; // level P = 2^l p: W_{2P}^j at j
                float2 nv[R];
#pragma unroll
                for (int m = 0; m < H; ++m) {
                    const float2 t =
                        nfft_odd<OUTER>(v[c][m + H], twl[k + (l ? bitrev_bits(m & ((1 << l) - 1), l) : 0) * p]);
                    nv[2 * m] = make_float2(v[c][m].x + t.x, v[c][m].y + t.y);
                    nv[2 * m + 1] = make_float2(v[c][m].x - t.x, v[c][m].y - t.y);
                }
#pragma unroll
                for (int q = 0; q < R; ++q) v[c][q] = nv[q];
            }
            base[c] = r * n + (i - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CNT; ++c)
        if (base[c] >= 0) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[nfft_pad(base[c] + bitrev_bits(q, LR) * p)] = v[c][q];
        }
    __syncthreads();
}

// Dynamic LDS: rpb rows of n entries (padded: 9/8 of that), then the n - 1 entries of the
// per-level twiddle table. Row groups g = blockIdx.x, + gridDim.x, ... of rpb = 8192 / n rows
// each (n a power of two, rpb n = 8192: eight entries a thread). Row r (of `rows`) is read
// from x + (r / sub) * in_row + (r % sub) with element stride `sub` (sub = 1: plain rows;
// sub = 2^s: the decimated sequences of a long row of in_row = n sub samples) and written
// contiguously to X + r n. The next row group's entries are loaded into registers while the
// current one is transformed.
template <bool OUTER>
__global__ __launch_bounds__(kNfftThreads) void nfft_kernel(const float2 *__restrict__ x, float2 *__restrict__ X,
                                                           long long rows_total, int n, int rpb, int sub,
                                                           long long in_row)
{
    constexpr int EPT = kNfftMaxN / kNfftThreads; // entries a thread loads and stores
    extern __shared__ float2 nfft_lds[];
    float2 *buf = nfft_lds, *tw = nfft_lds + nfft_pad(rpb * n);
    const int tid = threadIdx.x;
    const int lg = 31 - __builtin_clz(n);   // log2 n
    const int ls = 31 - __builtin_clz(sub); // log2 sub
    const long long gstep = (long long)gridDim.x * rpb;
    // entry i = tid + c 1024 of a row group: row i >> lg, column i mod n; with sub = 1 the
    // group's rows are contiguous (entry i at i), with sub > 1 a group is one row (rpb = 1,
    // entry i at i sub): either way i << ls from the group's first entry
    auto load_group = [&](long long b0, float2(&v)[EPT]) {
        const long long rows = min((long long)rpb, rows_total - b0);
        // the group's first entry and each c's part of the offset are uniform; the thread's
        // part, tid sub 8 bytes, is below 2^24
        const char *src = reinterpret_cast<const char *>(x + (b0 >> ls) * in_row + (b0 & (sub - 1)));
        const unsigned voff = (unsigned)tid << (ls + 3);
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int i = tid + c * kNfftThreads;
            const char *srcc = src + ((size_t)(c * kNfftThreads) << (ls + 3));
            v[c] = (i >> lg) < rows ? *reinterpret_cast<const float2 *>(srcc + voff) : make_float2(0.0f, 0.0f);
        }
    };
    float2 pv[EPT];
    long long b0 = (long long)blockIdx.x * rpb;
    if (b0 < rows_total) load_group(b0, pv); // in flight while the table is built
    nfft_level_table(tw, n, tid);
    for (; b0 < rows_total; b0 += gstep) {
        const int rows = (int)min((long long)rpb, rows_total - b0);
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int i = tid + c * kNfftThreads;
            if ((i >> lg) < rows)
                buf[nfft_pad(i)] = OUTER ? cop32(pv[c], make_float2(1.0f, 0.0f)) : pv[c]; // the length-1 transforms
        }
        __syncthreads(); // also orders the table before its first use
        if (b0 + gstep < rows_total) load_group(b0 + gstep, pv);
        // log2 n radix-2 levels, up to three of them per LDS round trip
        for (int p = 1; p < n;) {
            const int left = lg - (31 - __builtin_clz(p)); // levels still to do
            if (left >= 3) {
                nfft_group_pass<OUTER, 3>(buf, rows, n, lg, p, tw, tid);
                p <<= 3;
            } else if (left == 2) {
                nfft_group_pass<OUTER, 2>(buf, rows, n, lg, p, tw, tid);
                p <<= 2;
            } else {
                nfft_group_pass<OUTER, 1>(buf, rows, n, lg, p, tw, tid);
                p <<= 1;
            }
        }
        float2 *Xr = X + b0 * n;
        float2 ov[EPT];
#pragma unroll
        for (int c = 0; c < EPT; ++c) ov[c] = buf[nfft_pad(tid + c * kNfftThreads)];
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int i = tid + c * kNfftThreads;
            if ((i >> lg) < rows) Xr[i] = ov[c];
        }
        __syncthreads(); // buf is refilled for the next row group
    }
}

// The top levels' twiddles of long rows (n > 8192), one contiguous table per level: the level
// whose halves have length h (8192 <= h <= n / 2) holds W_{2h}^k = W_n^{k n / (2h)}, k < h,
// at h - 8192 + k (n - 8192 entries in all), so the lanes of a pass read consecutive entries.
__device__ __forceinline__ int nfft_top_off(int h) { return h - kNfftMaxN; }

__global__ __launch_bounds__(256) void nfft_table_kernel(float2 *tw, int n)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n - kNfftMaxN) return;
    const int h = 1 << (31 - __builtin_clz(j + kNfftMaxN)); // the level: largest power of two <= j + 8192
    const int k = j + kNfftMaxN - h;
    tw[j] = nfft_twiddle((int)((long long)k * (n / (2 * h))), n);
}

// One top level of a long row (n samples per row): at stride S the transform of x[j::S]
// (length 2h, h = n / (2 S)) from those of x[j::2S] and x[j + S::2S] (length h each), laid
// out as [residue][k] per row: src holds 2S sequences of length h, dst S of length 2h.
// Butterfly (j, k): E = src[j h + k], O = src[(j + S) h + k], twiddle W_{2h}^k = W_n^{k S}.
template <bool OUTER>
__global__ __launch_bounds__(256) void nfft_combine_kernel(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                           const float2 *__restrict__ tw, long long batch, int n,
                                                           int S)
{
    const long long half = (long long)n / 2;
    const int h = n / (2 * S);
    const int lhalf = 30 - __builtin_clz(n), lh = 31 - __builtin_clz(h); // n, S powers of two
    const long long total = batch * half;
    for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < total; w += (long long)gridDim.x * 256) {
        const long long row = w >> lhalf;
        const int b = (int)(w & (half - 1)); // butterfly of the row: j = b / h, k = b % h
        const int j = b >> lh, k = b & (h - 1);
        const float2 *s = src + row * n;
        const float2 e = s[(long long)j * h + k];
        const float2 t = nfft_odd<OUTER>(s[(long long)(j + S) * h + k], tw[nfft_top_off(h) + k]); // W_{2h}^k
        float2 *d = dst + row * n + (long long)j * 2 * h;
        d[k] = make_float2(e.x + t.x, e.y + t.y);
        d[k + h] = make_float2(e.x - t.x, e.y - t.y);
    }
}

// Two top levels of a long row in one pass: strides 2S, then S. The transforms of length h4 =
// n / (4 S) of x[j::4S] (A), x[j + 2S::4S] (B), x[j + S::4S] (C) and x[j + 3S::4S] (D) give
// those of x[j::2S] (A, B) and x[j + S::2S] (C, D) at level 2S, and those the transform of
// x[j::S] at level S: thread (j, k), k < h4, takes both level-2S butterflies at k and the two
// level-S butterflies at k and k + h4 whose operands they produce. The butterflies and their
// operations are those of two single-level passes, so the result is the same bit for bit,
// with half the passes over global memory. src holds 4S sequences of length h4, dst S of
// length 4 h4.
template <bool OUTER>
__global__ __launch_bounds__(256) void nfft_combine2_kernel(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                            const float2 *__restrict__ tw, long long batch, int n,
                                                            int S)
{
    const long long quarter = (long long)n / 4;
    const int h4 = n / (4 * S);
    const int lq = 29 - __builtin_clz(n), lh4 = 31 - __builtin_clz(h4); // n, S powers of two
    const long long total = batch * quarter;
    for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < total; w += (long long)gridDim.x * 256) {
        const long long row = w >> lq;
        const int b = (int)(w & (quarter - 1));
        const int j = b >> lh4, k = b & (h4 - 1);
        const float2 *s = src + row * n;
        const float2 a = s[(long long)j * h4 + k], bv = s[(long long)(j + 2 * S) * h4 + k];
        const float2 c = s[(long long)(j + S) * h4 + k], d = s[(long long)(j + 3 * S) * h4 + k];
        const float2 w1 = tw[nfft_top_off(h4) + k];          // W_{2 h4}^k
        const float2 w2a = tw[nfft_top_off(2 * h4) + k];     // W_{4 h4}^k
        const float2 w2b = tw[nfft_top_off(2 * h4) + k + h4]; // W_{4 h4}^{k + h4}
        // level 2S: x[j::2S] at k and k + h4 (P), x[j + S::2S] likewise (Q)
        const float2 t1 = nfft_odd<OUTER>(bv, w1), t2 = nfft_odd<OUTER>(d, w1);
        const float2 pp = make_float2(a.x + t1.x, a.y + t1.y), pm = make_float2(a.x - t1.x, a.y - t1.y);
        const float2 qp = make_float2(c.x + t2.x, c.y + t2.y), qm = make_float2(c.x - t2.x, c.y - t2.y);
        // level S: butterflies k and k + h4 of x[j::S]
        const float2 u = nfft_odd<OUTER>(qp, w2a), v = nfft_odd<OUTER>(qm, w2b);
        float2 *o = dst + row * n + (long long)j * 4 * h4;
        o[k] = make_float2(pp.x + u.x, pp.y + u.y);
        o[k + 2 * h4] = make_float2(pp.x - u.x, pp.y - u.y);
        o[k + h4] = make_float2(pm.x + v.x, pm.y + v.y);
        o[k + 3 * h4] = make_float2(pm.x - v.x, pm.y - v.y);
    }
}

} // namespace ndft
