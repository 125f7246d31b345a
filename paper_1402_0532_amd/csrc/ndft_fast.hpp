// Fast exact transform of Eq. (7) for N = 2^n: every bin of X = S z + F csgn(z) (the
// identity of Eq. (6): a (x) b = csgn(a) b + a csgn(b), with S = csgn(F) the ternary twiddle
// signs) in O(N log N) operations per row instead of O(N) per bin.
//
// D = F csgn(z) is an ordinary DFT of the ternary signs: an FFT (radix-4 Stockham stages).
// T = S z: T[p] = sum_k phi(p k mod N) z_k with phi(m) = csgn(W^m) (W = e^{-2 pi j / N}) is
// not a Fourier sum, but it only depends on p k mod N, which the multiplicative structure of
// Z/N splits into cyclic correlations:
//  * p = 2^v u (u odd): phi_N(2^v u k) = phi_M(u k mod M) with M = N / 2^v, so T[p] is the
//    odd-bin transform of length M of the folded row y_v[k'] = sum_j z[k' + j M];
//  * k' = 2^w t (t odd), or k' = 0 (phi = 1): phi_M(u 2^w t) = phi_L(u t mod L), L = M / 2^w;
//  * the odd residues mod L = 2^l form the group {(-1)^e 5^a : e < 2, a < L / 4} (l >= 3;
//    {1, 3} for L = 4, {1} for L = 2), in which u t is (e1 xor e2, a1 + a2 mod L / 4):
//      C_L(y)[u] = sum_{t odd < L} phi_L(u t) y[t]
//    is a cyclic correlation of length L / 4 per sign pair, i.e. a DFT of y in that order,
//    a product with the DFT of phi_L in that order, and an inverse DFT.
//   T[2^v u] = y_v[0] + sum_{w < log2 M} C_{M / 2^w}(y_v[2^w .])[u mod M / 2^w].
// The correlations of one length L (the pairs v + w = n - l) run together as FFTs; those of
// lengths up to kFastDirectL are summed directly, all in one step, and added to T with the
// k' = 0 terms. Every step is a sum of the same products as the
// definition, regrouped, so the result is Eq. (7)'s up to FP32 rounding (a few ulp times
// log2 N of the l1 mass of the terms; the DFTs of phi_L are made in FP64 and rounded once).
//
// One 1024-thread work-group per row (rows looped over the grid), everything in LDS:
// the folds y_0 .. y_n (2N entries, up to four levels a step), two correlation buffers
// (N/2 each, at least 48), T (N), the signs (N char2), the group order and its inverse
// (N/2 ints each) and the two-level W_N table: 153 KB at N = 4096.
#pragma once

#include "ndft_device.hpp"
#include "ndft_dft12b.hpp"

namespace ndft {

constexpr int kFastThreads = 1024;
constexpr int kFastMinN = 8;
constexpr int kFastMaxN = 4096;
constexpr int kFastDirectL = 32; // correlation lengths summed directly
constexpr int kFastFftL = 6;      // log2 of the shortest correlation length done by FFT
constexpr int kFastLgMax = 12;    // log2 kFastMaxN
constexpr int kFastDirectEntries = 288; // sum_{l <= 5} (lg - l + 1) 2^(l-1) <= 274 (lg <= 12)

// sources of the rows
constexpr int FAST_X = 0;   // rows of x (Eq. (7))
constexpr int FAST_LAG = 1; // lag products of Eq. (6) at the delays tau0 + row (Eq. (12a))
constexpr int FAST_LIN = 2; // ordinary lag products s conj(r) at those delays (Eq. (12c))

struct FastParams {
    int n, lg;                 // N = 2^lg
    int rows;
    const float2 *x;           // FAST_X: rows of x, stride n
    const float2 *s, *r;       // FAST_LAG, FAST_LIN: surveillance and reference records
    int tau0;
    const int *gtab;           // the group order of the odd residues mod N: N / 2 entries
    const int *dlog;           // its inverse: index of odd u at (u - 1) / 2
    const float2 *spec;        // DFTs of phi_L in group order, L >= 2 kFastDirectL: [L][e][omega]
    int tb, n_coarse;          // two-level table of W_N
    int p0n, n_dop;            // requested bins: p0n + q mod N, q < n_dop
    float2 *out;               // [rows][n_dop]
};

// offset of the spectra of length L in FastParams::spec (L >= 2 kFastDirectL)
__host__ __device__ constexpr int fast_spec_off(int L) { return L / 2 - kFastDirectL; }

// entries of the spectra table, tables and workspace for length n
__host__ __device__ constexpr int fast_spec_entries(int n) { return n >= 2 * kFastDirectL ? fast_spec_off(2 * n) : 0; }

// LDS bytes of the row kernel for length n
__host__ __device__ constexpr int fast_lds_bytes(int n, int n_tab)
{
    return (4 * n + kFastDirectEntries + 16 * (kFastLgMax + 1) + (kFastLgMax + 1) + n_tab) * 8 + n * 2 + n * 4;
}

// (-1)^e 5^a mod L for L a power of two >= 4 (a < L / 4)
__device__ __forceinline__ int pow5_signed(int e, int a, int L)
{
    unsigned r = 1, b = 5, k = (unsigned)a;
    const unsigned mask = (unsigned)L - 1u;
    while (k) {
        if (k & 1u) r = (r * b) & mask;
        b = (b * b) & mask;
        k >>= 1;
    }
    return e ? (int)((L - r) & mask) : (int)r;
}

// Tables of one call. Blocks 0 .. nspec - 1: the DFT (length Q = L/4, FP64 radix-2) of
// phi_L in group order for the sign e, one block per (L, e), L = 2 kFastDirectL .. N; the
// last block: the group order of the odd residues mod N and its inverse.
constexpr int kFastTabThreads = 512;

__global__ __launch_bounds__(kFastTabThreads) void fast_tables_kernel(int n, int lg, int *gtab, int *dlog,
                                                                      float2 *spec)
{
    __shared__ double2 buf[2][kFastMaxN / 4];
    __shared__ double2 wq[kFastMaxN / 8]; // W_Q^m = (cos, sin) of -2 pi m / Q, m < Q / 2
    const int tid = threadIdx.x;
    const int nspec = lg >= 6 ? 2 * (lg - 5) : 0; // L = 64 .. n
    if ((int)blockIdx.x >= nspec) {
        const int qn = n / 4;
        for (int i = tid; i < n / 2; i += kFastTabThreads) {
            const int g = pow5_signed(i / qn, i % qn, n);
            gtab[i] = g;
            dlog[(g - 1) >> 1] = i;
        }
        return;
    }
    const int l = 6 + (int)blockIdx.x / 2, e = (int)blockIdx.x & 1;
    const int L = 1 << l, Q = L / 4;
    for (int a = tid; a < Q; a += kFastTabThreads) {
        const TwSign sg = twiddle_sign(pow5_signed(e, a, L), L);
        buf[0][a] = make_double2((double)sg.c, (double)sg.t);
    }
    for (int m = tid; m < Q / 2; m += kFastTabThreads) {
        double sn, cs;
        sincospi(-2.0 * (double)m / (double)Q, &sn, &cs);
        wq[m] = make_double2(cs, sn);
    }
    __syncthreads();
    int src = 0;
    for (int h = 1, ls = l - 3; h < Q; h <<= 1, --ls) {
        for (int j = tid; j < Q / 2; j += kFastTabThreads) {
            const int k = j & (h - 1);
            const double2 w = wq[k << ls]; // W_{2h}^k = W_Q^{k Q / (2h)}
            const double cs = w.x, sn = w.y;
            const double2 a = buf[src][j], b = buf[src][j + Q / 2];
            const double2 wb = make_double2(cs * b.x - sn * b.y, cs * b.y + sn * b.x);
            buf[src ^ 1][2 * j - k] = make_double2(a.x + wb.x, a.y + wb.y);
            buf[src ^ 1][2 * j - k + h] = make_double2(a.x - wb.x, a.y - wb.y);
        }
        __syncthreads();
        src ^= 1;
    }
    float2 *dst = spec + fast_spec_off(L) + e * Q;
    for (int w = tid; w < Q; w += kFastTabThreads) dst[w] = make_float2((float)buf[src][w].x, (float)buf[src][w].y);
}

// Stockham stages over nseq sequences of length Q = 2^lq in LDS, src -> dst: radix 4 while
// it fits, then one radix-2 stage; stage with sub-length h, j < Q / r, k = j mod h:
//   y[(j - k) r + k + t h] = sum_s x[j + s Q / r] W_{r h}^{s k} W_r^{s t}
// forward (INV = false) or inverse (conjugate twiddles, no scaling).
template <bool INV, int R>
__device__ __forceinline__ void fast_stockham_stage(const float2 *src, float2 *dst, int nseq, int lq, int lh,
                                                    int lgn, const float2 *coarse, const float2 *fine, int tb,
                                                    int tid)
{
    constexpr int LR = R == 4 ? 2 : 1;
    const int lqr = lq - LR, h = 1 << lh;        // Q / R = 2^lqr sub-transforms a sequence
    const int lstep = lgn - lh - LR;             // W_{R h}^m = W_N^{m N / (R h)}
    for (int t = tid; t < (nseq << lqr); t += kFastThreads) {
        const int sq = t >> lqr, j = t & ((1 << lqr) - 1), k = j & (h - 1);
        const float2 *sp = src + (sq << lq) + j;
        float2 *dp = dst + (sq << lq) + ((j - k) << LR) + k;
        float2 a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = sp[q << lqr];
#pragma unroll
        for (int q = 1; q < R; ++q) {
            float2 w = table_twiddle(coarse, fine, (q * k) << lstep, tb);
            if (INV) w.y = -w.y;
            a[q] = cmulf(w, a[q]);
        }
        if constexpr (R == 2) {
            dp[0] = caddf(a[0], a[1]);
            dp[h] = csubf(a[0], a[1]);
        } else {
            const float2 t0 = caddf(a[0], a[2]), t1 = csubf(a[0], a[2]);
            const float2 t2 = caddf(a[1], a[3]);
            float2 t3 = csubf(a[1], a[3]);
            t3 = INV ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x); // times -+j
            dp[0] = caddf(t0, t2);
            dp[h] = caddf(t1, t3);
            dp[2 * h] = csubf(t0, t2);
            dp[3 * h] = csubf(t1, t3);
        }
    }
}

// A whole length-2^lq transform of nseq sequences: stages alternate between the buffers;
// returns the one holding the result. Barriers after every stage.
template <bool INV>
__device__ __forceinline__ float2 *fast_fft(float2 *a, float2 *b, int nseq, int lq, int lgn, const float2 *coarse,
                                            const float2 *fine, int tb, int tid)
{
    int lh = 0;
    while (lh + 2 <= lq) {
        fast_stockham_stage<INV, 4>(a, b, nseq, lq, lh, lgn, coarse, fine, tb, tid);
        __syncthreads();
        float2 *t = a;
        a = b;
        b = t;
        lh += 2;
    }
    if (lh < lq) {
        fast_stockham_stage<INV, 2>(a, b, nseq, lq, lh, lgn, coarse, fine, tb, tid);
        __syncthreads();
        float2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// One pass of folds: levels v0 + 1 .. v0 + G from level v0 (m = the deepest level's length):
// thread k takes the 2^G entries k + i m of level v0 and writes the partial sums of each level.
template <int G>
__device__ __forceinline__ void fast_fold_pass(const float2 *src, float2 *const (&dst)[4], int m, int tid)
{
    for (int k = tid; k < m; k += kFastThreads) {
        float2 a[1 << G];
#pragma unroll
        for (int i = 0; i < (1 << G); ++i) a[i] = src[k + i * m];
#pragma unroll
        for (int g = 1; g <= G; ++g) {
            const int cnt = 1 << (G - g);
#pragma unroll
            for (int i = 0; i < (1 << (G - 1)); ++i)
                if (i < cnt) {
                    a[i] = caddf(a[i], a[i + cnt]);
                    dst[g - 1][k + i * m] = a[i];
                }
        }
    }
}

// The correlations of every length L = 2^l, 64 <= L <= N, side by side: l's 2 B_l sequences
// (B_l = lg - l + 1 pairs, two signs each) of length Q_l = 2^(l-2) sit at off_l = sum over
// shorter l of B 2^(l-1) in each of the two buffers. Every length takes the same number S of
// stages (those of the longest, ceil((lg - 2) / 2)): radix 4 first, then radix 2, then plain
// copies where a short length runs out of factors.
struct FastStage {
    int r, lh; // radix (1: copy) and sub-length log2 of the stage
};

__device__ __forceinline__ FastStage fast_stage_of(int lq, int S, int st)
{
    const int a = lq >= S ? lq - S : 0;      // radix-4 stages
    const int b = lq >= S ? 2 * S - lq : lq; // radix-2 stages
    if (st < a) return {4, 2 * st};
    if (st < a + b) return {2, 2 * a + (st - a)};
    return {1, lq};
}

// Global item g of a step over all lengths goes to thread g mod 1024: a length's items
// o .. o + items - 1 are taken by the loop below without decoding the length per item.
#define FAST_FOR_ITEMS(x, o, items)                                                                         \
    for (int x = (tid - (o)) & (kFastThreads - 1); x < (items); x += kFastThreads)

// A stage's work on one length comes in items of four entries (one radix-4 butterfly, two
// radix-2 butterflies of neighbouring j, or four copied entries), 64 items to a chunk, the
// lengths' chunks one after another; chunk c goes to wave c mod 16, so a wave's parameters
// are uniform and its lanes busy (at N = 4096: 32 chunks, two a wave).
struct FastChunk {
    int kind;  // 1: copy, 2: two radix-2 butterflies, 4: one radix-4 butterfly
    int off;   // the length's first entry in the buffers
    int lq;    // log2 Q (sequence length)
    int lqr;   // log2 (Q / radix)
    int lh;    // log2 of the sub-length h
    int lstep; // twiddle W_{radix h}^m = W_N^{m 2^lstep}
};

// One lane's item: its four inputs and the raw table entries of its twiddles.
struct FastItem {
    float2 a[4];
    float2 wc[2], wf[2];
};

__device__ __forceinline__ void fast_item_load(const FastChunk &f, const float2 *src, const float2 *coarse,
                                               const float2 *fine, int tb, int x, FastItem &it)
{
    const int fm = (1 << tb) - 1;
    if (f.kind == 4) {
        const int j = x & ((1 << f.lqr) - 1), k = j & ((1 << f.lh) - 1);
        const float2 *sp = src + f.off + ((x >> f.lqr) << f.lq) + j;
#pragma unroll
        for (int q = 0; q < 4; ++q) it.a[q] = sp[q << f.lqr];
        const int v = k << f.lstep;
        it.wc[0] = coarse[v >> tb];
        it.wf[0] = fine[v & fm];
    } else if (f.kind == 2) {
        // sub-items 2x and 2x + 1: the same sequence, j and j + 1 (j even)
        const int x2 = 2 * x, j = x2 & ((1 << f.lqr) - 1), k = j & ((1 << f.lh) - 1);
        const float2 *sp = src + f.off + ((x2 >> f.lqr) << f.lq) + j;
        const float4 u0 = *reinterpret_cast<const float4 *>(sp);
        const float4 u1 = *reinterpret_cast<const float4 *>(sp + (1 << f.lqr));
        it.a[0] = make_float2(u0.x, u0.y);
        it.a[2] = make_float2(u0.z, u0.w);
        it.a[1] = make_float2(u1.x, u1.y);
        it.a[3] = make_float2(u1.z, u1.w);
        const int v0 = k << f.lstep, v1 = f.lh ? (k + 1) << f.lstep : 0;
        it.wc[0] = coarse[v0 >> tb];
        it.wf[0] = fine[v0 & fm];
        it.wc[1] = coarse[v1 >> tb];
        it.wf[1] = fine[v1 & fm];
    } else {
        const float4 *sp = reinterpret_cast<const float4 *>(src + f.off + 4 * x);
        const float4 u0 = sp[0], u1 = sp[1];
        it.a[0] = make_float2(u0.x, u0.y);
        it.a[1] = make_float2(u0.z, u0.w);
        it.a[2] = make_float2(u1.x, u1.y);
        it.a[3] = make_float2(u1.z, u1.w);
    }
}

template <bool INV>
__device__ __forceinline__ void fast_item_store(const FastChunk &f, float2 *dst, int x, FastItem &it)
{
    const int h = 1 << f.lh;
    if (f.kind == 4) {
        const int j = x & ((1 << f.lqr) - 1), k = j & (h - 1);
        float2 *dp = dst + f.off + ((x >> f.lqr) << f.lq) + ((j - k) << 2) + k;
        float2 *a = it.a;
        // W, W^2, W^3 from one table read and two products
        float2 w = cmulf(it.wc[0], it.wf[0]);
        if (INV) w.y = -w.y;
        const float2 w2 = cmulf(w, w);
        a[1] = cmulf(w, a[1]);
        a[2] = cmulf(w2, a[2]);
        a[3] = cmulf(cmulf(w, w2), a[3]);
        const float2 t0 = caddf(a[0], a[2]), t1 = csubf(a[0], a[2]);
        const float2 t2 = caddf(a[1], a[3]);
        float2 t3 = csubf(a[1], a[3]);
        t3 = INV ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x); // times -+j
        const float2 y0 = caddf(t0, t2), y1 = caddf(t1, t3), y2 = csubf(t0, t2), y3 = csubf(t1, t3);
        if (h == 1) { // dp = 4 j: four neighbouring entries
            float4 *d4 = reinterpret_cast<float4 *>(dp);
            d4[0] = make_float4(y0.x, y0.y, y1.x, y1.y);
            d4[1] = make_float4(y2.x, y2.y, y3.x, y3.y);
        } else {
            dp[0] = y0;
            dp[h] = y1;
            dp[2 * h] = y2;
            dp[3 * h] = y3;
        }
    } else if (f.kind == 2) {
        const int x2 = 2 * x, j = x2 & ((1 << f.lqr) - 1), k = j & (h - 1);
        float2 *dp = dst + f.off + ((x2 >> f.lqr) << f.lq) + ((j - k) << 1) + k;
        float2 w0 = cmulf(it.wc[0], it.wf[0]), w1 = cmulf(it.wc[1], it.wf[1]);
        if (INV) {
            w0.y = -w0.y;
            w1.y = -w1.y;
        }
        const float2 b0 = cmulf(w0, it.a[1]), b1 = cmulf(w1, it.a[3]);
        const float2 s0 = caddf(it.a[0], b0), d0 = csubf(it.a[0], b0);
        const float2 s1 = caddf(it.a[2], b1), d1 = csubf(it.a[2], b1);
        float4 *d4 = reinterpret_cast<float4 *>(dp);
        if (h == 1) { // j -> 2 j, 2 j + 1; j + 1 -> 2 j + 2, 2 j + 3
            d4[0] = make_float4(s0.x, s0.y, d0.x, d0.y);
            d4[1] = make_float4(s1.x, s1.y, d1.x, d1.y);
        } else { // k + 1 < h: j + 1 lands next to j in both halves
            d4[0] = make_float4(s0.x, s0.y, s1.x, s1.y);
            *reinterpret_cast<float4 *>(dp + h) = make_float4(d0.x, d0.y, d1.x, d1.y);
        }
    } else {
        float4 *dp = reinterpret_cast<float4 *>(dst + f.off + 4 * x);
        dp[0] = make_float4(it.a[0].x, it.a[0].y, it.a[1].x, it.a[1].y);
        dp[1] = make_float4(it.a[2].x, it.a[2].y, it.a[3].x, it.a[3].y);
    }
}

template <bool INV>
__device__ __forceinline__ void fast_multi_stage(const float2 *src, float2 *dst, int lg, int S, int st,
                                                 const float2 *coarse, const float2 *fine, int tb, int tid)
{
    constexpr int NW = kFastThreads / 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    int cb = 0, off = 0;
#pragma unroll
    for (int l = kFastFftL; l <= kFastLgMax; ++l) { // unrolled: l is a constant in each copy
        if (l > lg) break;
        const int lq = l - 2, items = (lg - l + 1) << (l - 3), nc = (items + 63) >> 6;
        const FastStage s = fast_stage_of(lq, S, st);
        const int lr = s.r == 4 ? 2 : 1;
        const FastChunk f{s.r, off, lq, lq - lr, s.lh, lg - s.lh - lr};
        // this wave's chunks of the length: c = wave mod NW, cb <= c < cb + nc
        for (int c = cb + ((wave - cb) & (NW - 1)); c < cb + nc; c += NW) {
            const int x = ((c - cb) << 6) + lane;
            if (x < items) {
                FastItem it;
                fast_item_load(f, src, coarse, fine, tb, x, it);
                fast_item_store<INV>(f, dst, x, it);
            }
        }
        cb += nc;
        off += (lg - l + 1) << (l - 1);
    }
}

template <int MODE>
__global__ __launch_bounds__(kFastThreads) void fast_ndft_kernel(FastParams P)
{
    extern __shared__ float4 fsm4[]; // 16-byte aligned: the stages move entry pairs
    float2 *fsm = reinterpret_cast<float2 *>(fsm4);
    const int n = P.n, lg = P.lg, tid = threadIdx.x;
    // two regions of 2n entries: R1 holds the folds, then serves as an FFT buffer, then T;
    // R2 holds the gathered correlation inputs, then the other FFT buffer, then the FFT of
    // the signs
    float2 *R1 = fsm;
    float2 *R2 = R1 + 2 * n;
    float2 *SD = R2 + 2 * n;                    // direct correlations (<= 288 entries)
    float2 *SV = SD + kFastDirectEntries;       // their sums per fold level: [v][odd r < 32]
    float2 *YS = SV + 16 * (kFastLgMax + 1);    // y_v[0], v = 0 .. lg
    float2 *coarse = YS + (kFastLgMax + 1);
    float2 *fine = coarse + P.n_coarse;
    int *G = reinterpret_cast<int *>(fine + (1 << P.tb)); // group order mod n
    int *DL = G + n / 2;                                   // its inverse
    char2 *sig = reinterpret_cast<char2 *>(DL + n / 2);    // csgn(z)
    const int lqn = lg - 2; // n / 4 = 2^lqn
    auto yoff = [&](int v) { return 2 * n - ((2 * n) >> v); };
    // element i of the group order mod L = 2^l: i = e 2^(l-2) + a -> (-1)^e 5^a mod L
    auto gl = [&](int i, int l) {
        if (l == 1) return 1;
        const int e = i >> (l - 2), a = i & ((1 << (l - 2)) - 1);
        return G[(e << lqn) + a] & ((1 << l) - 1);
    };
    // index of the odd residue u mod 2^l in that order, from u's index iN = DL[u >> 1] in the
    // order mod N (u = (-1)^e 5^a mod N is the same mod 2^l, where 5 has order 2^(l-2))
    auto dlr = [&](int iN, int l) {
        if (l == 1) return 0;
        const int e = iN >> lqn, a = iN & ((1 << lqn) - 1);
        return (e << (l - 2)) + (a & ((1 << (l - 2)) - 1));
    };
    const int lsmall = min(lg, kFastFftL - 1); // lengths 2 .. 32: summed directly
    const int R = min(32, n);                  // the direct lengths divide R
    // offset of the direct correlations of length 2^l in SD: pairs c < lg - l + 1, 2^(l-1) each
    auto soff = [&](int l) {
        int o = 0;
        for (int k = 1; k < l; ++k) o += (lg - k + 1) << (k - 1);
        return o;
    };
    const int S = lg >= kFastFftL ? (lg - 1) / 2 : 0; // stages of the longest: ceil((lg - 2) / 2)

    build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, kFastThreads);
    for (int i = tid; i < n / 2; i += kFastThreads) {
        G[i] = P.gtab[i];
        DL[i] = P.dlog[i];
    }
    // a thread's samples k = tid + 1024 e, e < EPT (n <= 4096): the row's inputs are loaded a
    // row ahead into registers (FAST_LAG: the surveillance samples are the same every row)
    constexpr int EPT = kFastMaxN / kFastThreads;
    float2 pa[EPT], pb[EPT];
    auto load_row = [&](int row) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int k = tid + e * kFastThreads;
            if constexpr (MODE == FAST_X) {
                pa[e] = k < n ? P.x[(size_t)row * n + k] : make_float2(0.0f, 0.0f);
            } else {
                const int kr = k - (P.tau0 + row);
                pb[e] = k < n && kr >= 0 ? P.r[kr] : make_float2(0.0f, 0.0f);
            }
        }
    };
    if constexpr (MODE != FAST_X) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int k = tid + e * kFastThreads;
            pa[e] = k < n ? P.s[k] : make_float2(0.0f, 0.0f);
        }
    }
    if ((int)blockIdx.x < P.rows) load_row(blockIdx.x);
    for (int row = blockIdx.x; row < P.rows; row += gridDim.x) {
        __syncthreads(); // tables ready; the previous row's reads of LDS done
        // ---- the row and its exact signs ----
        float2 *Y = R1;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int k = tid + e * kFastThreads;
            if (k >= n) break;
            float zr, zi, sr, si;
            if constexpr (MODE == FAST_X) {
                zr = pa[e].x;
                zi = pa[e].y;
                sr = sgnf(pa[e].x);
                si = sgnf(pa[e].y);
            } else if constexpr (MODE == FAST_LAG) {
                const Lag z = lag_product(pa[e], pb[e]);
                zr = z.zr;
                zi = z.zi;
                sr = z.sr;
                si = z.si;
            } else {
                // s conj(r) in FP64: the products of FP32 values are exact, one rounding of
                // each sum keeps its sign (the FP32 value can underflow, the sign cannot)
                const double sx = pa[e].x, sy = pa[e].y, rx = pb[e].x, ry = pb[e].y;
                const double zr64 = fma(sx, rx, sy * ry), zi64 = fma(sy, rx, -(sx * ry));
                zr = (float)zr64;
                zi = (float)zi64;
                sr = zr64 > 0.0 ? 1.0f : (zr64 < 0.0 ? -1.0f : 0.0f);
                si = zi64 > 0.0 ? 1.0f : (zi64 < 0.0 ? -1.0f : 0.0f);
            }
            Y[k] = make_float2(zr, zi);
            sig[k] = make_char2((signed char)sr, (signed char)si);
        }
        if (row + (int)gridDim.x < P.rows) load_row(row + gridDim.x); // in flight through the row
        __syncthreads();
        // ---- folds y_v[k] = y_{v-1}[k] + y_{v-1}[k + n >> v], up to four levels a pass: a
        // thread takes the 2^g entries of level v0 that fold into one entry of level v0 + g ----
        for (int v0 = 0; v0 < lg; v0 += 4) {
            const int g4 = min(4, lg - v0);
            const int m = n >> (v0 + g4);
            float2 *const dst[4] = {Y + yoff(v0 + 1), Y + yoff(min(v0 + 2, lg)), Y + yoff(min(v0 + 3, lg)),
                                    Y + yoff(min(v0 + 4, lg))};
            const float2 *src = Y + yoff(v0);
            if (g4 == 4)
                fast_fold_pass<4>(src, dst, m, tid);
            else if (g4 == 3)
                fast_fold_pass<3>(src, dst, m, tid);
            else if (g4 == 2)
                fast_fold_pass<2>(src, dst, m, tid);
            else
                fast_fold_pass<1>(src, dst, m, tid);
            __syncthreads();
        }
        // ---- from the folds, in one step: y_v[0]; the direct correlations (lengths 2 .. 32)
        // C[c][i1] = sum_i2 phi_L(g1 g2) y_c[2^w g2]; the FFT correlations' inputs in
        // group order, [l][c][e][a] into R2 ----
        for (int v = tid; v <= lg; v += kFastThreads) YS[v] = Y[yoff(v)];
        {
            // the widest first: a length-32 sum is split over 4 neighbouring lanes and a
            // length-16 sum over 2 (4 terms a lane, their reads issued together), the partial
            // sums added across the lanes; 730 lanes at N = 4096
            int ou = 0;
#pragma unroll
            for (int l = kFastFftL - 1; l >= 1; --l) {
                if (l > lsmall) continue;
                const int L = 1 << l, half = L >> 1;
                const int lp = l >= 4 ? l - 3 : 0; // log2 of the lanes per sum
                const int T = half >> lp;         // terms a lane
                const int items = (lg - l + 1) << (l - 1), so = soff(l), o = ou;
                ou += items << lp;
                FAST_FOR_ITEMS(u, o, items << lp)
                {
                    const int it = u >> lp, part = u & ((1 << lp) - 1);
                    const int c = it >> (l - 1), i1 = it & (half - 1), w = lg - l - c;
                    const int g1 = gl(i1, l);
                    const float2 *y = Y + yoff(c);
                    float2 acc = make_float2(0.0f, 0.0f);
                    // this lane's terms: group-order indices part T .. part T + T - 1 (5^a, then
                    // L - 5^a, a < L / 4; {1} for L = 2)
#pragma unroll
                    for (int k = 0; k < (l >= 3 ? 4 : (l == 2 ? 2 : 1)); ++k) {
                        const int g2 = gl(part * T + k, l);
                        const TwSign ph = twiddle_sign((g1 * g2) & (L - 1), L);
                        const float2 yv = y[g2 << w];
                        // (ph.c + j ph.t) yv
                        acc.x += (float)ph.c * yv.x - (float)ph.t * yv.y;
                        acc.y += (float)ph.c * yv.y + (float)ph.t * yv.x;
                    }
                    if (lp >= 1) {
                        acc.x += __shfl_xor(acc.x, 1);
                        acc.y += __shfl_xor(acc.y, 1);
                    }
                    if (lp >= 2) {
                        acc.x += __shfl_xor(acc.x, 2);
                        acc.y += __shfl_xor(acc.y, 2);
                    }
                    if (part == 0) SD[so + it] = acc;
                }
            }
        }
        for (int l = kFastFftL, o = 0; l <= lg; o += (lg - l + 1) << (l - 1), ++l) {
            const int lh = l - 1;
            FAST_FOR_ITEMS(x, o, (lg - l + 1) << lh)
            {
                const int c = x >> lh, i = x & ((1 << lh) - 1), w = lg - l - c;
                R2[o + x] = Y[yoff(c) + (gl(i, l) << w)];
            }
        }
        __syncthreads();
        // ---- per fold level v, the direct correlations summed for each odd residue r < 32:
        // SV[v][r >> 1] = sum_{l <= 5, l <= lg - v} C_l[v][r mod 2^l] (the first FFT stage in
        // the same step: the folds are no longer read) ----
        for (int t = tid; t < (lg + 1) * (R >> 1); t += kFastThreads) {
            const int v = t / (R >> 1), rr = t - v * (R >> 1), iN = DL[rr];
            float2 acc = make_float2(0.0f, 0.0f);
            for (int l = 1; l <= lsmall && l <= lg - v; ++l) acc = caddf(acc, SD[soff(l) + (v << (l - 1)) + dlr(iN, l)]);
            SV[v * 16 + rr] = acc;
        }
        // ---- the FFT correlations: S forward stages, the products with the spectra, S
        // inverse stages, all lengths side by side ----
        float2 *src = R2, *dst = R1;
        for (int st = 0; st < S; ++st) {
            fast_multi_stage<false>(src, dst, lg, S, st, coarse, fine, P.tb, tid);
            __syncthreads();
            float2 *tmp = src;
            src = dst;
            dst = tmp;
        }
        if (S == 0) __syncthreads(); // SV complete
        // Chat[c][e1][om] = sum_e2 Fhat[e1 xor e2][om] Yhat[c][e2][-om], both e1 of an
        // (c, om) from one read of its inputs
        for (int l = kFastFftL, o = 0, oi = 0; l <= lg; o += (lg - l + 1) << (l - 1), oi += (lg - l + 1) << (l - 2), ++l) {
            const int lq = l - 2, Q = 1 << lq;
            const float2 *F = P.spec + fast_spec_off(1 << l);
            FAST_FOR_ITEMS(x, oi, (lg - l + 1) << lq)
            {
                const int c = x >> lq, om = x & (Q - 1), nom = (Q - om) & (Q - 1);
                const int b0 = o + ((2 * c) << lq), b1 = b0 + Q;
                const float2 y0 = src[b0 + nom], y1 = src[b1 + nom];
                const float2 f0 = F[om], f1 = F[Q + om];
                dst[b0 + om] = caddf(cmulf(f0, y0), cmulf(f1, y1));
                dst[b1 + om] = caddf(cmulf(f1, y0), cmulf(f0, y1));
            }
        }
        __syncthreads();
        {
            float2 *tmp = src;
            src = dst;
            dst = tmp;
        }
        for (int st = 0; st < S; ++st) {
            fast_multi_stage<true>(src, dst, lg, S, st, coarse, fine, P.tb, tid);
            __syncthreads();
            float2 *tmp = src;
            src = dst;
            dst = tmp;
        }
        const float2 *C = src; // the correlations (times Q_l); dst is free for T
        float2 *T = dst;
        // ---- T[2^v u] = y_v[0] + SV[v][u mod 32] + sum_{64 <= 2^l <= n >> v} C_l[v][u mod 2^l] / Q_l;
        // T[0] = the row's sum ----
        for (int p0 = tid; p0 < n; p0 += 4 * kFastThreads) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = p0 + e * kFastThreads;
                if (p >= n) break;
                if (p == 0) {
                    T[0] = YS[lg];
                    continue;
                }
                const int v = __builtin_ctz(p), u = p >> v, iN = DL[u >> 1];
                float2 acc = caddf(YS[v], SV[v * 16 + ((u & (R - 1)) >> 1)]);
                int o = 0;
#pragma unroll
                for (int li = 0; li <= kFastLgMax - kFastFftL; ++li) { // reads issued together
                    const int l = kFastFftL + li;
                    const bool ok = l <= lg - v;
                    const float2 cv = C[ok ? o + (v << (l - 1)) + dlr(iN, l) : 0];
                    const float sc = 1.0f / (float)(1 << (l - 2));
                    if (ok) acc = make_float2(fmaf(cv.x, sc, acc.x), fmaf(cv.y, sc, acc.y));
                    o += (lg - l + 1) << (l - 1);
                }
                T[p] = acc;
            }
        }
        // ---- D = F csgn(z): FFT of the signs in the other region ----
        float2 *DA = T == R1 ? R2 : R1;
        __syncthreads(); // C read
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int k = tid + e * kFastThreads;
            if (k < n) DA[k] = make_float2((float)sig[k].x, (float)sig[k].y);
        }
        __syncthreads();
        const float2 *D = fast_fft<false>(DA, DA + n, 1, lg, lg, coarse, fine, P.tb, tid);
        // ---- X[p] = T[p] + D[p] for the requested bins ----
        float2 *o = P.out + (size_t)row * P.n_dop;
        for (int q0 = tid; q0 < P.n_dop; q0 += 4 * kFastThreads) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = q0 + e * kFastThreads;
                if (q >= P.n_dop) break;
                int p = P.p0n + q;
                p = p >= n ? p - n : p;
                o[q] = caddf(T[p], D[p]);
            }
        }
    }
}

} // namespace ndft
