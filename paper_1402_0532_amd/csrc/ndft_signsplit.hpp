// Sign-split form of the split-BF16 cross-ambiguity surface (Eq. (12a)).
//
// With the complex operator of Eq. (6) written as a (x) b = csgn(a) b + a csgn(b) (plain
// complex products), every term of A(d, p) = sum_k z_k (x) W^{pk} (z_k the lag product of
// delay d, W = e^{-2 pi j / N}) splits into two sums:
//   T(d, p) = sum_k csgn(W^{pk}) z_k   -- the twiddle signs, ternary and piecewise constant
//                                         in k (they change where pk mod N crosses a
//                                         multiple of N/4), against the FP32 lag values;
//   D(d, p) = sum_k W^{pk} csgn(z_k)   -- the twiddles against the exact lag signs.
// T is evaluated run by run from prefix sums of z over chunks of samples (lsum_kernel, on
// the vector units: a handful of runs per base and chunk instead of one term per sample);
// D is a contraction on the matrix cores (dsum_kernel) of BF16 hi + lo twiddles against
// the lag signs, which lsum_kernel writes as 2-bit codes. Half the matrix work of the
// combined form, and no lag arithmetic in the matrix loop. Base 0 (twiddle 1) is done
// entirely in lsum_kernel: its D part is the plain sum of the signs.
//
// The split needs only the lag values and their exact signs, so the Eq. (12c) surface
// (the ordinary lag product s conj(r), then the Eq. (6) operator with the twiddle) runs on
// the same kernels: lsum_kernel<true> forms that product instead (FP64 from the FP32
// inputs, where both products are exact and one rounding of their sum keeps the sign).
//
// Both kernels write float4 (U, V, X, Y) partial planes of the same layout, so one
// reduction adds them: A[+b] = (U - V, X + Y), A[-b] = (U + V, X - Y) with
//   U = sum Re(c) Re(v), V = sum Im(c) Im(v), X = sum Re(c) Im(v), Y = sum Im(c) Re(v)
// for the coefficient c (csgn W or W) and the value v (z or csgn z) of each part.
#pragma once

#include "ndft_contract.hpp"
#include "ndft_device.hpp"
#include "ndft_surface_bf16.hpp"

namespace ndft {

// ------------------------------------------------------------------------------------
// lag signs as codes
// ------------------------------------------------------------------------------------
// One 32-bit word per (delay, 4 consecutive samples k0..k3): two bits (sign, non-zero) per
// sign, placed so that masking the word (after a shift by 0, 2, 4, 6) gives the BF16 pair
// of +-2 / 0 sign operands directly: sign re of k0 at bits 15:14, k1 at 31:30, k2 at
// 13:12, k3 at 29:28; sign im of k0 at 11:10, k1 at 27:26, k2 at 9:8, k3 at 25:24.
// Layout: [32-sample stage][delay column (padded)][half h][step q] words, where the word
// (h, q) covers samples stage*32 + 8q + 4h + 0..3 (the samples lane half h of a matrix
// step q consumes).
// Packed layout (the FP32 plan, whose FFT kernel reads the codes of one delay row at a
// time): [delay column (padded)][k / 8] words, one per delay and 8 consecutive samples: the
// used bytes of the two 4-sample words side by side (byte 1 of the word of samples 0..3,
// byte 1 of that of 4..7, byte 3 of the first, byte 3 of the second), so sample e's real
// field sits at bit 14, 30, 12, 28 (e mod 4 = 0 .. 3) less 8 for e < 4, its imaginary one
// 4 bits lower: half the bytes, and a delay row is contiguous.
constexpr unsigned kPackSel = 0x07030501u; // v_perm selector (w1, w0): w0.b1, w1.b1, w0.b3, w1.b3
__device__ __forceinline__ uint32_t sign_field(float s)
{
    return s == 0.0f ? 0u : (s < 0.0f ? 3u : 1u);
}

__device__ __forceinline__ uint32_t sign_field(double s)
{
    return s == 0.0 ? 0u : (s < 0.0 ? 3u : 1u);
}

// The ordinary lag product s conj(r) of Eq. (11) from complex64 samples, in FP64: each
// product of two FP32 values is exact there, so the single rounding of the fused sum gives
// each component with its exact sign (and 0 only for an exact 0).
__device__ __forceinline__ void linear_lag64(float4 s, float4 r, double &zr, double &zi)
{
    const double sx = s.x, sy = s.y, rx = r.x, ry = r.y;
    zr = fma(sx, rx, sy * ry);
    zi = fma(sy, rx, -(sx * ry));
}

// ------------------------------------------------------------------------------------
// twiddle-sign crossings
// ------------------------------------------------------------------------------------
// With u = 4 b k (the phase of W^{bk} in quarter turns times N), the real part of
// csgn(W^{bk}) is the sign of cos(2 pi u / 4N) and the imaginary part that of
// -sin(2 pi u / 4N). Each part is a square wave in u that changes only at its crossings
// u = phi + 2 N i (phi = N for the real part, 0 for the imaginary part) and is exactly 0
// where u hits one; the sign just before crossing i is (-1)^i for both parts. Crossing i
// falls at sample k_i = ceil((phi + 2 N i) / 4b); it is exact (sample k_i has the zero)
// when 4b k_i = phi + 2 N i. rem = 4b k_i - (phi + 2 N i) in [0, 4b) steps from one
// crossing to the next with q0 = floor(2N / 4b), r0 = 2N mod 4b: the next crossing is
// q0 + 1 samples on when rem < r0 (then rem += 4b - r0), q0 samples on otherwise
// (rem -= r0). A walker that stands at sample kb keeps the next crossing at or after kb:
// its offset nk >= 0 from the current chunk start, its rem, and the sign sg before it.
struct Crossing {
    int nk, rem;
    float sg;
};

template <int PART> // 0: real part (phi = N), 1: imaginary part (phi = 0)
__device__ __forceinline__ Crossing first_crossing(unsigned b, long long kb, int n)
{
    Crossing c;
    if (b == 0) { // u stays 0: real part +1, imaginary part 0, no crossing ahead
        c.nk = 0x3fffffff;
        c.rem = 1;
        c.sg = PART == 0 ? 1.0f : 0.0f;
        return c;
    }
    const int fb = 4 * (int)b;                               // <= 2N
    int w = 4 * (int)(((long long)b * kb) % n) - fb;        // u of sample kb - 1, mod 4N
    if (w < 0) w += 4 * n;
    int cu; // next crossing value above w (mod 4N, possibly past 4N)
    if (PART == 0) {
        cu = w < n ? n : (w < 3 * n ? 3 * n : 5 * n);
        c.sg = cu == 3 * n ? -1.0f : 1.0f;
    } else {
        cu = w < 2 * n ? 2 * n : 4 * n;
        c.sg = cu == 2 * n ? -1.0f : 1.0f;
    }
    const int d = cu - w;                 // > 0: the crossing lies d past sample kb - 1
    const int cq = (d + fb - 1) / fb;     // >= 1
    c.nk = cq - 1;
    c.rem = cq * fb - d;
    return c;
}

// ------------------------------------------------------------------------------------
// lsum_kernel: lag products, sign codes and the T part (plus base 0 entirely)
// ------------------------------------------------------------------------------------
struct LsumParams {
    const float2 *s, *r;      // complex64 inputs, n samples each
    int n, n_cols, tau0;
    BaseMap bm;               // every base, in partial-row order
    int n_bases;
    int n_bases_pad, n_cols_pad; // partial plane layout
    long long kchunk;         // samples per block (multiple of the chunk), k range of blockIdx.y
    long long k_end;          // samples covered by the codes (n rounded up to the chunk)
    uint32_t *codes;          // sign codes, see above
    long long code_wpc;       // packed layout: words per delay column (k_end / 8)
    float4 *part;             // this kernel's partial planes: [blockIdx.y][n_cols_pad][n_bases_pad]
};

constexpr int kLsumDelays = 16;   // delays per block
constexpr int kLsumChunk = 256;   // samples per chunk (prefix sums in LDS)
constexpr int kLsumBases = 256;   // base rows per block

// Window index with one pad entry per 8: the lanes of a wave read entries 8 apart, which
// the pad puts on different banks.
__device__ __forceinline__ int wpad(int i) { return i + (i >> 3); }

// Prefix tables: row o holds the 16 delays of the block (float2 each) at a stride of 17
// float2 plus 1 more after every 16 rows. The 32 writers of a delay pair store rows 8
// apart, which the odd stride and the per-16 shift spread over the banks; the walkers read
// rows at random. A walker reads the 8 delays it owns as four 8-byte pairs.
constexpr int kLsumRowF2 = kLsumDelays + 1;
__device__ __forceinline__ int prow(int o) { return (int)__umul24((unsigned)o, kLsumRowF2) + (o >> 4); }
constexpr int kLsumTabF2 = kLsumChunk * kLsumRowF2 + (kLsumChunk >> 4) + kLsumDelays;

// inclusive scan over the 32 lanes of each half wave (the 32 threads of one delay pair):
// within the DPP rows of 16 lanes, then row 1 (3) adds the last lane of row 0 (2)
__device__ __forceinline__ float half_scan32(float x)
{
#define NDFT_DPP_ADD(ctrl, rows)                                                               \
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, rows, 0xf, true))
    NDFT_DPP_ADD(0x111, 0xf); // row_shr:1
    NDFT_DPP_ADD(0x112, 0xf); // row_shr:2
    NDFT_DPP_ADD(0x114, 0xf); // row_shr:4
    NDFT_DPP_ADD(0x118, 0xf); // row_shr:8
    NDFT_DPP_ADD(0x142, 0xa); // row_bcast:15 into rows 1 and 3
#undef NDFT_DPP_ADD
    return x;
}

// sign bits of two floats at bits 15 (lo) and 31 (hi)
__device__ __forceinline__ uint32_t sign_pair(float hi, float lo)
{
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x070c030cu);
}

// Blocks: blockIdx.x = 16 delays, blockIdx.y = range of whole chunks, blockIdx.z = 256
// base rows (after row 0 when base 0 is present: base 0 is summed apart, from the block
// total of z and the sign counts). Lag phase: thread (dp, g) makes z for the delay pair
// 2 dp, 2 dp + 1 and samples 8 g .. 8 g + 7 of the chunk (the pair shares the s values and
// all but one r value). Crossing phase: a thread takes 8 of the delays and two base rows
// i and M - 1 - i of the group's M rows: the rows ascend in b and the crossings per chunk
// grow with b, so every thread walks about as many as any other.
//
// Per part and chunk, with P(k) the prefix sum of z over the chunk's first k samples,
//   sum_k S(k) z_k = S_end P(C) + sum_{crossings k_i < C} S_i (P(k_i) + P(k_i + e_i))
// (S_i the sign before crossing i, e_i = 1 when it is exact: the zero sample is then a
// run of its own; S_end the sign after the chunk's last crossing). The tables hold P at
// the chunk's C + 1 sample edges: P(k) + P(k) = 2 P(k) and R(k) = P(k) + P(k + 1), so a
// crossing costs one row read either way, and the end term comes once per chunk. The
// prefix sums restart at every chunk, so no term is larger than the sum of 256 |z|: the
// rounding of T is a few ulp of the chunk sums per crossing, however far the block's
// prefix sum grows (DC-heavy rows), instead of a few ulp of the block's prefix sum.
//
// LIN: the lag product of the Eq. (12c) surface (linear_lag64) instead of Eq. (6).
// PACK: the codes in the packed layout.
template <bool LIN, bool PACK>
__global__ __launch_bounds__(256, 2) void lsum_kernel(LsumParams L)
{
    constexpr int DT = kLsumDelays, C = kLsumChunk;
    constexpr int SPT = DT * C / 512; // samples per thread and delay (two delays each)
    static_assert(SPT == 8, "two code words per thread and delay");
    constexpr int RW = C + DT - 1;
    constexpr int WIN = C + RW;                   // window entries (s, then r)
    constexpr int WIT = (WIN + 255) / 256;        // window loads per thread
    __shared__ float4 sw[C + C / 8];              // s with signs (padded index)
    __shared__ float4 rw[RW + RW / 8 + 1];        // r with signs, the block's delays
    __shared__ float2 ptab[kLsumTabF2]; // P(o), o = 0 .. C
    __shared__ float2 rtab[kLsumTabF2]; // R(o) = P(o) + P(o + 1), o < C

    const int tid = threadIdx.x;
    const int n = L.n;
    const int c0 = blockIdx.x * DT;
    const int dmin = L.tau0 + c0;
    const long long kb = (long long)blockIdx.y * L.kchunk;
    const long long ke = min(kb + L.kchunk, L.k_end);

    // z work: delays dl0 = 2 dp and dl0 + 1, samples o0 .. o0 + 7 of the chunk
    const int dp = tid >> 5, g = tid & 31, o0 = g * SPT, dl0 = 2 * dp;
    const int col0 = c0 + dl0;

    // crossing work: delays dh * 8 .. + 7, base rows i and M - 1 - i of the group
    constexpr int DH = DT / 2;
    const int has0 = L.bm.nseg > 0 && L.bm.start[0] == 0;
    const int row_base = has0 + blockIdx.z * kLsumBases;
    const int M = min(kLsumBases, L.n_bases - row_base);
    const int pi = tid & 127, dh = tid >> 7;
    int bi[2];
    bool own[2];
    int fb[2], q0[2], r0[2];
    Crossing cr[2][2]; // [row][part]
    bi[0] = row_base + pi;
    bi[1] = row_base + M - 1 - pi;
    own[0] = pi < M && pi <= M - 1 - pi;
    own[1] = pi < M - 1 - pi;
    float acc[2][DH][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const unsigned b = (unsigned)base_of(L.bm, min(max(bi[j], 0), L.n_bases - 1));
        fb[j] = 4 * (int)b;
        q0[j] = b > 0 ? (2 * n) / fb[j] : 0; // >= 1: b <= N / 2
        r0[j] = b > 0 ? 2 * n - q0[j] * fb[j] : 0;
        cr[j][0] = first_crossing<0>(b, kb, n);
        cr[j][1] = first_crossing<1>(b, kb, n);
#pragma unroll
        for (int d = 0; d < DH; ++d)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[j][d][t] = 0.0f;
    }
    // sum of z over the block's chunks so far, delays dl0 + h, and counts of negative and
    // zero signs (this thread's samples; the 32 threads of the pair are added at the end):
    // base 0 of those delays
    float2 gq[2] = {make_float2(0.0f, 0.0f), make_float2(0.0f, 0.0f)};
    int ngr[2] = {0, 0}, ngi[2] = {0, 0}, zcr[2] = {0, 0}, zci[2] = {0, 0}, nfield = 0;

    // windows of a chunk (zero outside [0, n)): s[k0 + i], then r[k0 - dmax + i]
    auto win_load = [&](long long k0, float2 (&v)[WIT]) {
#pragma unroll
        for (int it = 0; it < WIT; ++it) {
            const int i = tid + it * 256;
            const long long idx = i < C ? k0 + i : k0 - (dmin + DT - 1) + (i - C);
            v[it] = make_float2(0.0f, 0.0f);
            if (i < WIN && idx >= 0 && idx < n) v[it] = (i < C ? L.s : L.r)[idx];
        }
    };
    auto win_store = [&](const float2 (&v)[WIT]) {
#pragma unroll
        for (int it = 0; it < WIT; ++it) {
            const int i = tid + it * 256;
            if (i < C)
                sw[wpad(i)] = with_signs(v[it]);
            else if (i < WIN)
                rw[wpad(i - C)] = with_signs(v[it]);
        }
    };

    {
        float2 v[WIT];
        win_load(kb, v);
        win_store(v);
    }
    __syncthreads();
    for (long long k0 = kb; k0 < ke; k0 += C) {
        float2 nv[WIT]; // next chunk's window, in flight during this chunk
        if (k0 + C < ke) win_load(k0 + C, nv);

        // ---- lag products of (dl0 + h, o0 .. o0 + 7): FP32 values (the operations of
        // lag_product4), their signs as codes ----
        // In groups of four samples (a scheduling barrier between groups keeps the loads
        // of one group in registers at a time): the values, the code word of each delay,
        // and the running prefix within the thread (zr, zi end up holding it). Delay dl0 + h
        // pairs sample o0 + j with r entry o0 + j + 15 - dl0 - h = rb + j + 1 - h.
        const int rb = o0 + DT - 2 - dl0;
        float zr[2][SPT], zi[2][SPT];
        uint32_t code[2][2]; // [delay][half]
        float mz = 3.0e38f; // smallest |component|
        float pr[2] = {0.0f, 0.0f}, pim[2] = {0.0f, 0.0f};
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            // sample 4 w + e meets r entries cn (delay dl0) and cp (delay dl0 + 1)
            float vr[2][4], vi[2][4];
            float4 cp = rw[wpad(rb + 4 * w)];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float4 a = sw[wpad(o0 + 4 * w + e)], cn = rw[wpad(rb + 4 * w + e + 1)];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float4 cc = h == 0 ? cn : cp;
                    if constexpr (LIN) {
                        double zr64, zi64;
                        linear_lag64(a, cc, zr64, zi64);
                        vr[h][e] = (float)zr64;
                        vi[h][e] = (float)zi64;
                    } else {
                        vr[h][e] = fmaf(a.x, cc.z, cc.x * a.z) + fmaf(a.y, cc.w, cc.y * a.w);
                        vi[h][e] = fmaf(a.y, cc.z, cc.x * a.w) - fmaf(cc.y, a.z, a.x * cc.w);
                    }
                    mz = fminf(mz, fminf(fabsf(vr[h][e]), fabsf(vi[h][e])));
                }
                cp = cn;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // a normal FP32 value carries the exact sign (see lag_product4, and
                // linear_lag64 rounded once more, which keeps a sign): the sign
                // bits go to the sign positions of the code word, every non-zero bit is set
                code[h][w] = (sign_pair(vr[h][1], vr[h][0]) & 0x80008000u) |
                             ((sign_pair(vr[h][3], vr[h][2]) >> 2) & 0x20002000u) |
                             ((sign_pair(vi[h][1], vi[h][0]) >> 4) & 0x08000800u) |
                             ((sign_pair(vi[h][3], vi[h][2]) >> 6) & 0x02000200u) | 0x55005500u;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    pr[h] += vr[h][e];
                    pim[h] += vi[h][e];
                    zr[h][4 * w + e] = pr[h];
                    zi[h][4 * w + e] = pim[h];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // zero or subnormal components (zero padding, integer or cancelling inputs): the
        // exact signs of lag_product4 (linear_lag64) for this thread's samples
        if (__builtin_amdgcn_ballot_w64(!(mz >= 1.17549435e-38f))) {
            if (!(mz >= 1.17549435e-38f)) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll 1
                    for (int j = 0; j < SPT; ++j) { // rolled: the FP64 test is long and rare
                        uint32_t fr, fi;
                        if constexpr (LIN) {
                            double zr64, zi64;
                            linear_lag64(sw[wpad(o0 + j)], rw[wpad(rb + j + 1 - h)], zr64, zi64);
                            fr = sign_field(zr64);
                            fi = sign_field(zi64);
                        } else {
                            const Lag e = lag_product4(sw[wpad(o0 + j)], rw[wpad(rb + j + 1 - h)]);
                            fr = sign_field(e.sr);
                            fi = sign_field(e.si);
                        }
                        const int q = j & 3;
                        const int pos_r = (q & 1) ? 30 - 2 * (q >> 1) : 14 - 2 * (q >> 1); // k0:14 k1:30 k2:12 k3:28
                        const uint32_t keep = ~((3u << pos_r) | (3u << (pos_r - 4)));
                        const uint32_t f = (fr << pos_r) | (fi << (pos_r - 4));
                        const bool w1 = j >= 4;
                        const uint32_t cw = ((w1 ? code[h][1] : code[h][0]) & keep) | f;
                        code[h][0] = w1 ? code[h][0] : cw;
                        code[h][1] = w1 ? cw : code[h][1];
                    }
#pragma unroll
                    for (int w = 0; w < 2; ++w) {
                        zcr[h] += 4 - __builtin_popcount(code[h][w] & 0x50005000u);
                        zci[h] += 4 - __builtin_popcount(code[h][w] & 0x05000500u);
                    }
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                ngr[h] += __builtin_popcount(code[h][w] & 0xa000a000u);
                ngi[h] += __builtin_popcount(code[h][w] & 0x0a000a00u);
            }
        }
        nfield += SPT;
        if constexpr (PACK) {
            // the thread's 8 samples are one packed word per delay
            const long long wi = (k0 + o0) >> 3;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (col0 + h < L.n_cols_pad)
                    L.codes[(long long)(col0 + h) * L.code_wpc + wi] =
                        __builtin_amdgcn_perm(code[h][1], code[h][0], kPackSel);
        } else {
            // the thread's 8 samples are one step q of a 32-sample stage: word (w, q) holds
            // samples 8 q + 4 w .. + 3
            const long long k = k0 + o0;
            const long long st = k >> 5;
            const int q = (int)((k >> 3) & 3);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (col0 + h < L.n_cols_pad) {
                    uint32_t *cw = L.codes + ((st * L.n_cols_pad + col0 + h) * 2) * 4 + q;
                    cw[0] = code[h][0];
                    cw[4] = code[h][1];
                }
            }
        }
        // prefix tables: P(o0 + 1 + j) = (earlier chunks) + (exclusive scan of the thread
        // totals) + zr[j]
        {
            float er[2], ei[2], lr[2], li[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                er[h] = half_scan32(pr[h]) - pr[h];
                ei[h] = half_scan32(pim[h]) - pim[h];
                lr[h] = er[h]; // P(o0 + j)
                li[h] = ei[h];
            }
            if (g == 0) {
                ptab[dl0] = make_float2(0.0f, 0.0f);
                ptab[dl0 + 1] = make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int j = 0; j < SPT; ++j) {
                float nr[2], ni[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    nr[h] = er[h] + zr[h][j];
                    ni[h] = ei[h] + zi[h][j];
                }
                float2 *pp = ptab + prow(o0 + j + 1) + dl0, *rp = rtab + prow(o0 + j) + dl0;
                pp[0] = make_float2(nr[0], ni[0]);
                pp[1] = make_float2(nr[1], ni[1]);
                rp[0] = make_float2(lr[0] + nr[0], li[0] + ni[0]);
                rp[1] = make_float2(lr[1] + nr[1], li[1] + ni[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    lr[h] = nr[h];
                    li[h] = ni[h];
                }
            }
        }
        __syncthreads(); // prefix tables complete; the windows are free again
        // the block total of z (base 0)
        {
            const float2 t0 = ptab[prow(C) + dl0], t1 = ptab[prow(C) + dl0 + 1];
            gq[0] = make_float2(gq[0].x + t0.x, gq[0].y + t0.y);
            gq[1] = make_float2(gq[1].x + t1.x, gq[1].y + t1.y);
        }

        if (k0 + C < ke) win_store(nv);

        // ---- T part: crossings within the chunk, per row and part (Re part into U, X;
        // Im part into Y, V) ----
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (__builtin_amdgcn_ballot_w64(own[j]) == 0) continue; // no row of the wave kept
            auto walk = [&](auto partc) {
                constexpr int PART = decltype(partc)::value;
                constexpr int IA = PART == 0 ? 0 : 3, IB = PART == 0 ? 2 : 1; // sums of P.x, P.y
                Crossing c = cr[j][PART];
                while (c.nk < C) {
                    const bool ex = c.rem == 0;
                    const float2 *t2 = (ex ? rtab : ptab) + prow(c.nk) + dh * DH;
                    const float wgt = ex ? c.sg : 2.0f * c.sg;
#pragma unroll
                    for (int d = 0; d < DH; ++d) {
                        const float2 v = t2[d];
                        acc[j][d][IA] = fmaf(wgt, v.x, acc[j][d][IA]);
                        acc[j][d][IB] = fmaf(wgt, v.y, acc[j][d][IB]);
                    }
                    c.sg = -c.sg;
                    const int t = c.rem - r0[j];
                    c.nk += q0[j] + (t < 0 ? 1 : 0);
                    c.rem = t < 0 ? t + fb[j] : t;
                }
                c.nk -= C;
                cr[j][PART] = c;
            };
            walk(std::integral_constant<int, 0>());
            walk(std::integral_constant<int, 1>());
            // the sign after the chunk's last crossing times the chunk total (row C)
#pragma unroll
            for (int d = 0; d < DH; ++d) {
                const float2 q = ptab[prow(C) + dh * DH + d];
                acc[j][d][0] = fmaf(cr[j][0].sg, q.x, acc[j][d][0]);
                acc[j][d][2] = fmaf(cr[j][0].sg, q.y, acc[j][d][2]);
                acc[j][d][3] = fmaf(cr[j][1].sg, q.x, acc[j][d][3]);
                acc[j][d][1] = fmaf(cr[j][1].sg, q.y, acc[j][d][1]);
            }
        }
        __syncthreads(); // next window stored, prefix tables read
    }
    // base 0: W = 1, so the T part is the sum of z and the D part that of the signs
    float4 *out = L.part + (long long)blockIdx.y * L.n_cols_pad * L.n_bases_pad;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
            ngr[h] += __shfl_xor(ngr[h], off, 32);
            ngi[h] += __shfl_xor(ngi[h], off, 32);
            zcr[h] += __shfl_xor(zcr[h], off, 32);
            zci[h] += __shfl_xor(zci[h], off, 32);
        }
        if (has0 && blockIdx.z == 0 && g == 0 && col0 + h < L.n_cols) {
            const int nf = 32 * nfield; // fields per part over the 32 threads
            out[(long long)(col0 + h) * L.n_bases_pad] = make_float4(gq[h].x + (float)(nf - zcr[h] - 2 * ngr[h]), 0.0f,
                                                                    gq[h].y + (float)(nf - zci[h] - 2 * ngi[h]), 0.0f);
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (!own[j]) continue;
#pragma unroll
        for (int d = 0; d < DH; ++d) {
            const int c = c0 + dh * DH + d;
            if (c < L.n_cols)
                out[(long long)c * L.n_bases_pad + bi[j]] =
                    make_float4(acc[j][d][0], acc[j][d][1], acc[j][d][2], acc[j][d][3]);
        }
    }
}

// ------------------------------------------------------------------------------------
// dsum_kernel: D part on the matrix cores
// ------------------------------------------------------------------------------------
// Per 8-sample step, lane (h, l32) of base block i holds the twiddle operand
// [hi(k0..k3), lo(k0..k3)] of Re W / 2 (A1) or Im W / 2 (A2) for base row 32 i + l32 and
// samples k0..k3 = step start + 4 h + 0..3, and the sign operand [s(k0..k3), s(k0..k3)]
// (+-2 / 0) of its delay column: U = A1.B1, X = A1.B2, Y = A2.B1, V = A2.B2 with B1 from
// the real signs, B2 from the imaginary ones.
// W^b from the two-level table whose fine entries hold W / 2
__device__ __forceinline__ float2 twiddle_step(const float2 *coarse, const float2 *fine, int tb, int b)
{
    const float2 a = coarse[b >> tb], c = fine[b & ((1 << tb) - 1)];
    return make_float2(2.0f * fmaf(a.x, c.x, -a.y * c.y), 2.0f * fmaf(a.x, c.y, a.y * c.x));
}

template <int NW, int WB, int KS>
struct DsumCfg {
    static constexpr int NT = 64 * NW;
    static constexpr int BT = 32 * WB;
    static constexpr int LT = 32 * NW;
    static constexpr int G = KS / 8;             // 8-sample steps per stage
    static constexpr int STAGE_A = G * 4 * BT;   // uint4 per stage (step, A1/A2, h, row)
    static constexpr int UNITS = G * 2 * BT;     // (step, h, row): four samples, both operands
    static constexpr int CW = KS / 32;           // code stages (32 samples) per stage
    static_assert(KS % 32 == 0, "whole code stages per stage");
};

// Twiddle operands of one unit (base b, four consecutive samples from index m): W^m / 2
// from the two-level table (fine entries W / 2), the next three by the step wb = W^b
// (three FP32 complex products: a few ulp, far below the BF16 hi + lo split);
// A1 = Re, A2 = Im, each [hi(4 samples), lo(4 samples)].
__device__ __forceinline__ void dsum_unit(const float2 *coarse, const float2 *fine, int tb, int m, float2 wb,
                                          uint4 &a1, uint4 &a2)
{
    const int mask = (1 << tb) - 1;
    float wr[4], wi[4];
    {
        const float2 a = coarse[m >> tb], c = fine[m & mask];
        wr[0] = fmaf(a.x, c.x, -a.y * c.y);
        wi[0] = fmaf(a.x, c.y, a.y * c.x);
    }
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        wr[j] = fmaf(wr[j - 1], wb.x, -wi[j - 1] * wb.y);
        wi[j] = fmaf(wr[j - 1], wb.y, wi[j - 1] * wb.x);
    }
    split_pair(wr[0], wr[1], a1.x, a1.z);
    split_pair(wr[2], wr[3], a1.y, a1.w);
    split_pair(wi[0], wi[1], a2.x, a2.z);
    split_pair(wi[2], wi[3], a2.y, a2.w);
}

struct DplaneParams {
    uint4 *planes;
    long long plane_stages;
    int n, tb, n_coarse;
    int stages_per_block;
    BaseMap bm;
};

// Twiddle planes of the D part: [base tile][stage][step][A1/A2][h][row] uint4, W / 2 in
// BF16 hi + lo.
template <int BT, int KS>
__global__ __launch_bounds__(256) void dplane_build_kernel(DplaneParams Q)
{
    extern __shared__ float2 tables[];
    constexpr int G = KS / 8;
    constexpr int STAGE_A = G * 4 * BT;
    constexpr int UNITS = G * 2 * BT; // (step, h, row): four samples, both operands
    float2 *coarse = tables;
    float2 *fine = tables + Q.n_coarse;
    const int n = Q.n;
    build_twiddle_tables(coarse, fine, n, Q.tb, Q.n_coarse, threadIdx.x, 256, 0.5f); // W / 2
    __syncthreads();
    const long long s0 = (long long)blockIdx.x * Q.stages_per_block;
    const long long s1 = min(s0 + Q.stages_per_block, Q.plane_stages);
    for (int u = threadIdx.x; u < UNITS; u += 256) {
        const int row = u % BT, qh = u / BT, h = qh & 1, q = qh >> 1;
        const int b = base_of(Q.bm, blockIdx.y * BT + row);
        const float2 wb = twiddle_step(coarse, fine, Q.tb, b);
        int m = (int)(((long long)b * (s0 * KS + 8 * q + 4 * h)) % n);
        const int dm = (int)(((long long)b * KS) % n);
        uint4 *dst = Q.planes + ((long long)blockIdx.y * Q.plane_stages + s0) * STAGE_A + ((q * 2) * 2 + h) * BT + row;
        for (long long st = s0; st < s1; ++st) {
            uint4 a1, a2;
            dsum_unit(coarse, fine, Q.tb, m, wb, a1, a2);
            dst[0] = a1;
            dst[2 * BT] = a2;
            dst += STAGE_A;
            m = add_mod(m, dm, n);
        }
    }
}

// Block order as surface_bf16_planes_kernel: blockIdx = tile_l * grp_stride + (tile_b *
// ksplit + kc), so the delay tiles reading one plane stream share an XCD. Sample chunks
// are whole stage pairs; the codes and planes cover n rounded up to the lsum chunk.
// GEN: the twiddle operands are made in the kernel (from a two-level table in LDS, the
// units of the next stage spread over the threads) instead of copied from planes; the
// matrix loop leaves the vector units nearly idle, and no plane pass is needed.
template <int NW, int WB, int KS, bool GEN>
__global__ __launch_bounds__(64 * NW, 1) void dsum_kernel(ContractParams P, const uint32_t *codes,
                                                         long long code_stages)
{
    using Cfg = DsumCfg<NW, WB, KS>;
    constexpr int NT = Cfg::NT, BT = Cfg::BT, LT = Cfg::LT, G = Cfg::G, STAGE_A = Cfg::STAGE_A, CW = Cfg::CW;
    constexpr int PLI = STAGE_A / NT;
    constexpr int UPT = (Cfg::UNITS + NT - 1) / NT; // generated units per thread
    static_assert(STAGE_A % NT == 0, "plane stages split evenly");
    __shared__ uint4 bufA0[STAGE_A];
    __shared__ uint4 bufA1[STAGE_A];
    extern __shared__ float2 tables[];

    const int grp = blockIdx.x % P.grp_stride;
    const int tile_l = blockIdx.x / P.grp_stride;
    if (grp >= P.tiles_b * P.ksplit) return;
    const int tile_b = grp / P.ksplit, kc = grp % P.ksplit;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int b0 = tile_b * BT, c0 = tile_l * LT;
    const int k_begin = kc * P.kchunk;
    const int k_end = min(P.n, k_begin + P.kchunk);
    const int npair = k_end > k_begin ? (k_end - k_begin + 2 * KS - 1) / (2 * KS) : 0;
    const int col = c0 + wave * 32 + l32;

    const uint4 *pl_src =
        GEN ? nullptr : P.planes + ((long long)tile_b * P.plane_stages + k_begin / KS) * STAGE_A + tid;
    // GEN: thread units (step q, half h, row) -> twiddle index m of the unit's first sample
    float2 *coarse = tables, *fine = tables + P.n_coarse;
    // When the block's threads cover whole (h, row) sets, a thread's units share the row
    // and h (only the step differs): one base, step and offset for all of them.
    constexpr bool SAME_ROW = NT % (2 * BT) == 0 && Cfg::UNITS % NT == 0;
    int un_off[UPT], un_m[UPT], un_dm[UPT];
    float2 un_wb[UPT];
    if (GEN) {
        build_twiddle_tables(coarse, fine, P.n, P.tb, P.n_coarse, tid, NT, 0.5f); // W / 2
#pragma unroll
        for (int it = 0; it < UPT; ++it) {
            const int u = min(tid + it * NT, Cfg::UNITS - 1);
            const int row = u % BT, qh = u / BT, uh = qh & 1, uq = qh >> 1;
            const int b = base_of(P.bm, b0 + row);
            un_off[it] = ((uq * 2) * 2 + uh) * BT + row; // A1; A2 at + 2 BT
            un_m[it] = (int)(((long long)b * (k_begin + 8 * uq + 4 * uh)) % P.n);
            un_dm[it] = (int)(((long long)b * KS) % P.n);
        }
        __syncthreads(); // tables
#pragma unroll
        for (int it = 0; it < UPT; ++it) {
            const int u = min(tid + it * NT, Cfg::UNITS - 1);
            un_wb[it] = twiddle_step(coarse, fine, P.tb, base_of(P.bm, b0 + u % BT));
        }
    }
    auto gen_unit = [&](uint4 *buf, int it) { // unit it of the stage after the last generated one
        if (Cfg::UNITS % NT == 0 || tid + it * NT < Cfg::UNITS) {
            uint4 a1, a2;
            const int off = SAME_ROW ? un_off[0] + it * 2 * NT : un_off[it]; // NT units = 2 NT uint4
            dsum_unit(coarse, fine, P.tb, un_m[it], un_wb[SAME_ROW ? 0 : it], a1, a2);
            buf[off] = a1;
            buf[off + 2 * BT] = a2;
            un_m[it] = add_mod(un_m[it], un_dm[SAME_ROW ? 0 : it], P.n);
        }
    };
    auto gen = [&](uint4 *buf) {
#pragma unroll
        for (int it = 0; it < UPT; ++it) gen_unit(buf, it);
    };
    // codes of (stage, col, h): one uint4 = the words of steps 0..3
    const uint4 *cd = reinterpret_cast<const uint4 *>(codes);
    long long cst = k_begin / 32;
    auto code_load = [&](long long st) {
        st = min(st, code_stages - 1); // prefetch past the last stage reads a valid, unused one
        return cd[(st * P.n_cols_pad + col) * 2 + h];
    };

    f32x16 acc[WB][4];
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][t][e] = 0.0f;

    struct AFrag {
        bf16x8 a[WB][2];
    };
    auto load_a = [&](const uint4 *buf, int q, AFrag &f) {
#pragma unroll
        for (int i = 0; i < WB; ++i)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                f.a[i][t] = __builtin_bit_cast(bf16x8, buf[((q * 2 + t) * 2 + h) * BT + 32 * i + l32]);
    };
    // sign operands of one step from its code word: B1 real signs, B2 imaginary signs
    struct BFrag {
        bf16x8 b1, b2;
    };
    auto make_b = [&](uint32_t w, BFrag &g) {
        constexpr uint32_t M = 0xC000C000u;
        const uint32_t r01 = w & M, r23 = (w << 2) & M, i01 = (w << 4) & M, i23 = (w << 6) & M;
        g.b1 = __builtin_bit_cast(bf16x8, make_uint4(r01, r23, r01, r23));
        g.b2 = __builtin_bit_cast(bf16x8, make_uint4(i01, i23, i01, i23));
    };
    auto mfma_step = [&](const AFrag &f, const BFrag &g) {
#pragma unroll
        for (int i = 0; i < WB; ++i) {
            acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][0], g.b1, acc[i][0], 0, 0, 0);
            acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][0], g.b2, acc[i][1], 0, 0, 0);
            acc[i][2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][1], g.b1, acc[i][2], 0, 0, 0);
            acc[i][3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][1], g.b2, acc[i][3], 0, 0, 0);
        }
    };
    auto word = [](const uint4 &c, int q) { return (q & 3) == 0 ? c.x : (q & 3) == 1 ? c.y : (q & 3) == 2 ? c.z : c.w; };

    AFrag fa[2];
    BFrag fb[2];
    uint4 cw[CW];
    auto stage = [&](auto cbc) {
        constexpr int CB = decltype(cbc)::value;
        // two LDS variables so the compiler tells the plane copy's target from the stage read
        const uint4 *cur = CB ? bufA1 : bufA0;
        uint4 *nxt = CB ? bufA0 : bufA1;
        if (!GEN) {
            uint4 *dst = nxt + __builtin_amdgcn_readfirstlane(wave) * 64;
#pragma unroll
            for (int k = 0; k < PLI; ++k)
                __builtin_amdgcn_global_load_lds(pl_src + k * NT,
                                                 (__attribute__((address_space(3))) void *)(dst + k * NT), 16, 0, 0);
            pl_src += STAGE_A;
        }
        uint4 cn[CW]; // the next stage's code words, each loaded as its slot here frees
        load_a(cur, 0, fa[0]);
        make_b(cw[0].x, fb[0]);
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if ((q & 3) == 0) cn[q >> 2] = code_load(cst + CW + (q >> 2));
            if (q + 1 < G) {
                load_a(cur, q + 1, fa[(q + 1) & 1]);
                make_b(word(cw[(q + 1) >> 2], q + 1), fb[(q + 1) & 1]);
            }
            // the next step's operands stay ahead of this step's matrix instructions (and
            // are made in registers those instructions do not read)
            __builtin_amdgcn_sched_barrier(0);
            mfma_step(fa[q & 1], fb[q & 1]);
            // GEN: the next stage's units while this step's matrix instructions run
            if (GEN) {
#pragma unroll
                for (int it = 0; it < UPT; ++it)
                    if ((it * G) / UPT == q) gen_unit(nxt, it);
            }
        }
#pragma unroll
        for (int c = 0; c < CW; ++c) cw[c] = cn[c];
        cst += CW;
        if (!GEN) asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); // plane block landed before the barrier
        __syncthreads();
    };

    if (npair > 0) {
        if (GEN) {
            gen(bufA0);
        } else {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(pl_src);
            u32x4 *dst = reinterpret_cast<u32x4 *>(bufA0) + tid;
#pragma unroll
            for (int k = 0; k < PLI; ++k) dst[k * NT] = src[k * NT];
            pl_src += STAGE_A;
        }
#pragma unroll
        for (int c = 0; c < CW; ++c) cw[c] = code_load(cst + c);
        __syncthreads();
        for (int p = 0; p < npair; ++p) {
            stage(std::integral_constant<int, 0>());
            stage(std::integral_constant<int, 1>());
        }
    }

    float4 *out = P.partial + (long long)kc * P.n_cols_pad * P.n_bases_pad;
    if (P.row0 && tile_b == 0 && h == 0) out[(long long)col * P.n_bases_pad] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int row = P.row0 + b0 + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
            float4 v;
            v.x = acc[i][0][e]; // U
            v.y = acc[i][3][e]; // V
            v.z = acc[i][1][e]; // X
            v.w = acc[i][2][e]; // Y
            out[(long long)col * P.n_bases_pad + row] = v;
        }
}

// ------------------------------------------------------------------------------------
// FP8 form of the D part (dsum8_kernel)
// ------------------------------------------------------------------------------------
// v_mfma_scale_f32_32x32x64_f8f6f4 with e4m3 operands: lane half h of a 32-sample K group
// holds 32 bytes per row, [term 2mm of samples 16h .. 16h+15, term 2mm+1 of the same
// samples], scaled by 2^(-4 (2mm)) and 2^(-4 (2mm+1)) (the E8M0 scale of the lane in half
// 0 applies to bytes 0-15 of every lane, that of half 1 to bytes 16-31). The twiddle W / 2
// is carried as four e4m3 terms (each rounds the remaining residual, scaled by 16^j), the
// lag signs as exact e4m3 +-2 / 0 (the code fields moved to bits 7:6 of a byte), so two
// instructions (mm = 0, 1) cover 32 samples. Within a dword the samples are in the order
// (2, 0, 3, 1) of their 4-sample code word, which the sign extraction gives for free.

// e4m3 +-2 / 0 bytes of the real (IM = 0) or imaginary (IM = 1) signs of a code word, in
// the byte order (k2, k0, k3, k1)
template <int IM>
__device__ __forceinline__ uint32_t f8_signs(uint32_t w)
{
    constexpr uint32_t M = 0xC000C000u;
    const uint32_t x = IM ? w << 4 : w;
    return (x & M) | (((x << 2) & M) >> 8);
}

// Four e4m3 terms of four values, each term a dword in the byte order (v2, v0, v3, v1):
// v = t0 + t1 / 16 + t2 / 256 + t3 / 4096 + O(2^-16 |v|).
__device__ __forceinline__ void f8_terms4(float v0, float v1, float v2, float v3, uint32_t t[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v2, v0, 0, false);
        const int d = __builtin_amdgcn_cvt_pk_fp8_f32(v3, v1, lo, true);
        t[j] = (uint32_t)d;
        if (j < 3) {
            v2 = (v2 - __builtin_amdgcn_cvt_f32_fp8(d, 0)) * 16.0f;
            v0 = (v0 - __builtin_amdgcn_cvt_f32_fp8(d, 1)) * 16.0f;
            v3 = (v3 - __builtin_amdgcn_cvt_f32_fp8(d, 2)) * 16.0f;
            v1 = (v1 - __builtin_amdgcn_cvt_f32_fp8(d, 3)) * 16.0f;
        }
    }
}

// Twiddle operands of one unit: base row b, samples k0 .. k0 + 15 (m = b k0 mod n), W / 2
// from the two-level table and the step W^b. o[tt][mm][half] is the uint4 half of the
// lane's 32 bytes for the real (tt = 0) or imaginary (tt = 1) part.
__device__ __forceinline__ void dsum8_unit(const float2 *coarse, const float2 *fine, int tb, int m, float2 wb,
                                           uint4 (&o)[2][2][2])
{
    const int mask = (1 << tb) - 1;
    float wr[16], wi[16];
    {
        const float2 a = coarse[m >> tb], c = fine[m & mask];
        wr[0] = fmaf(a.x, c.x, -a.y * c.y);
        wi[0] = fmaf(a.x, c.y, a.y * c.x);
    }
#pragma unroll
    for (int j = 1; j < 16; ++j) {
        wr[j] = fmaf(wr[j - 1], wb.x, -wi[j - 1] * wb.y);
        wi[j] = fmaf(wr[j - 1], wb.y, wi[j - 1] * wb.x);
    }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const float *v = tt ? wi : wr;
        uint32_t t[4][4]; // [dword d][term j]
#pragma unroll
        for (int d = 0; d < 4; ++d) f8_terms4(v[4 * d], v[4 * d + 1], v[4 * d + 2], v[4 * d + 3], t[d]);
#pragma unroll
        for (int j = 0; j < 4; ++j) o[tt][j >> 1][j & 1] = make_uint4(t[0][j], t[1][j], t[2][j], t[3][j]);
    }
}

// FP8 twiddle planes: [base tile][stage][32-sample group G][tt][mm][h][row][2] uint4.
template <int BT, int KS>
__global__ __launch_bounds__(256) void dplane8_build_kernel(DplaneParams Q)
{
    extern __shared__ float2 tables[];
    constexpr int NG = KS / 32;
    constexpr int STAGE_A = NG * 16 * BT; // uint4
    constexpr int UNITS = NG * 2 * BT;    // (G, h, row): 16 samples, both parts, all terms
    float2 *coarse = tables;
    float2 *fine = tables + Q.n_coarse;
    const int n = Q.n;
    build_twiddle_tables(coarse, fine, n, Q.tb, Q.n_coarse, threadIdx.x, 256, 0.5f); // W / 2
    __syncthreads();
    const long long s0 = (long long)blockIdx.x * Q.stages_per_block;
    const long long s1 = min(s0 + Q.stages_per_block, Q.plane_stages);
    for (int u = threadIdx.x; u < UNITS; u += 256) {
        const int row = u % BT, gh = u / BT, h = gh & 1, g = gh >> 1;
        const int b = base_of(Q.bm, blockIdx.y * BT + row);
        const float2 wb = twiddle_step(coarse, fine, Q.tb, b);
        int m = (int)(((long long)b * (s0 * KS + 32 * g + 16 * h)) % n);
        const int dm = (int)(((long long)b * KS) % n);
        uint4 *dst = Q.planes + ((long long)blockIdx.y * Q.plane_stages + s0) * STAGE_A;
        for (long long st = s0; st < s1; ++st) {
            uint4 o[2][2][2];
            dsum8_unit(coarse, fine, Q.tb, m, wb, o);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                    for (int hf = 0; hf < 2; ++hf)
                        dst[(((((g * 2 + tt) * 2 + mm) * 2 + h) * BT) + row) * 2 + hf] = o[tt][mm][hf];
            dst += STAGE_A;
            m = add_mod(m, dm, n);
        }
    }
}

// D part in the FP8 form: the structure of dsum_kernel (same blocks, stages of KS samples,
// twiddle planes copied to LDS by direct loads, code words of the next stage loaded as
// their slots free), with the K groups of 32 samples above.
template <int NW, int WB, int KS>
__global__ __launch_bounds__(64 * NW, 1) void dsum8_kernel(ContractParams P, const uint32_t *codes,
                                                          long long code_stages)
{
    using Cfg = DsumCfg<NW, WB, KS>;
    constexpr int NT = Cfg::NT, BT = Cfg::BT, LT = Cfg::LT, CW = Cfg::CW;
    constexpr int NG = KS / 32;
    constexpr int STAGE_A = NG * 16 * BT;
    constexpr int PLI = STAGE_A / NT;
    static_assert(STAGE_A % NT == 0, "plane stages split evenly");
    __shared__ uint4 bufA0[STAGE_A];
    __shared__ uint4 bufA1[STAGE_A];

    const int grp = blockIdx.x % P.grp_stride;
    const int tile_l = blockIdx.x / P.grp_stride;
    if (grp >= P.tiles_b * P.ksplit) return;
    const int tile_b = grp / P.ksplit, kc = grp % P.ksplit;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int b0 = tile_b * BT, c0 = tile_l * LT;
    const int k_begin = kc * P.kchunk;
    const int k_end = min(P.n, k_begin + P.kchunk);
    const int npair = k_end > k_begin ? (k_end - k_begin + 2 * KS - 1) / (2 * KS) : 0;
    const int col = c0 + wave * 32 + l32;

    const uint4 *pl_src = P.planes + ((long long)tile_b * P.plane_stages + k_begin / KS) * STAGE_A + tid;
    // code words of (stage, col) that lane half h needs: (h' = 0, 1) x (q = 2h, 2h + 1)
    const uint2 *cd = reinterpret_cast<const uint2 *>(codes);
    long long cst = k_begin / 32;
    auto code_load = [&](long long st, uint4 &w) { // w = words for dwords d = 0 .. 3
        st = min(st, code_stages - 1); // prefetch past the last stage reads a valid, unused one
        const long long base = (st * P.n_cols_pad + col) * 4 + h; // uint2 index of (h' = 0, q = 2h)
        const uint2 w0 = cd[base], w1 = cd[base + 2];              // h' = 0, h' = 1
        w = make_uint4(w0.x, w1.x, w0.y, w1.y);
    };

    f32x16 acc[WB][4];
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][t][e] = 0.0f;

    auto load_a = [&](const uint4 *buf, int g, int mm, i32x8 (&a)[WB][2]) {
#pragma unroll
        for (int i = 0; i < WB; ++i)
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int idx = ((((g * 2 + tt) * 2 + mm) * 2 + h) * BT + 32 * i + l32) * 2;
                const uint4 lo = buf[idx], hi = buf[idx + 1];
                a[i][tt] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
    };

    uint4 cw[CW];
    auto stage = [&](auto cbc) {
        constexpr int CB = decltype(cbc)::value;
        const uint4 *cur = CB ? bufA1 : bufA0;
        uint4 *nxt = CB ? bufA0 : bufA1;
        {
            uint4 *dst = nxt + __builtin_amdgcn_readfirstlane(wave) * 64;
#pragma unroll
            for (int k = 0; k < PLI; ++k)
                __builtin_amdgcn_global_load_lds(pl_src + k * NT,
                                                 (__attribute__((address_space(3))) void *)(dst + k * NT), 16, 0, 0);
            pl_src += STAGE_A;
        }
        uint4 cn[CW];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            code_load(cst + CW + g, cn[g]);
            const uint4 w = cw[g];
            const i32x8 b1 = i32x8{(int)f8_signs<0>(w.x), (int)f8_signs<0>(w.y), (int)f8_signs<0>(w.z),
                                   (int)f8_signs<0>(w.w), (int)f8_signs<0>(w.x), (int)f8_signs<0>(w.y),
                                   (int)f8_signs<0>(w.z), (int)f8_signs<0>(w.w)};
            const i32x8 b2 = i32x8{(int)f8_signs<1>(w.x), (int)f8_signs<1>(w.y), (int)f8_signs<1>(w.z),
                                   (int)f8_signs<1>(w.w), (int)f8_signs<1>(w.x), (int)f8_signs<1>(w.y),
                                   (int)f8_signs<1>(w.z), (int)f8_signs<1>(w.w)};
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
                i32x8 a[WB][2];
                load_a(cur, g, mm, a);
                const int scale_a = 127 - 4 * (2 * mm + h);
#pragma unroll
                for (int i = 0; i < WB; ++i) {
                    acc[i][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i][0], b1, acc[i][0], 0, 0, 0,
                                                                              scale_a, 0, 127);
                    acc[i][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i][0], b2, acc[i][1], 0, 0, 0,
                                                                              scale_a, 0, 127);
                    acc[i][2] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i][1], b1, acc[i][2], 0, 0, 0,
                                                                              scale_a, 0, 127);
                    acc[i][3] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i][1], b2, acc[i][3], 0, 0, 0,
                                                                              scale_a, 0, 127);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CW; ++c) cw[c] = cn[c];
        cst += CW;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); // plane block landed before the barrier
        __syncthreads();
    };

    if (npair > 0) {
        {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(pl_src);
            u32x4 *dst = reinterpret_cast<u32x4 *>(bufA0) + tid;
#pragma unroll
            for (int k = 0; k < PLI; ++k) dst[k * NT] = src[k * NT];
            pl_src += STAGE_A;
        }
#pragma unroll
        for (int c = 0; c < CW; ++c) code_load(cst + c, cw[c]);
        __syncthreads();
        for (int p = 0; p < npair; ++p) {
            stage(std::integral_constant<int, 0>());
            stage(std::integral_constant<int, 1>());
        }
    }

    float4 *out = P.partial + (long long)kc * P.n_cols_pad * P.n_bases_pad;
    if (P.row0 && tile_b == 0 && h == 0) out[(long long)col * P.n_bases_pad] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int row = P.row0 + b0 + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
            float4 v;
            v.x = acc[i][0][e]; // U
            v.y = acc[i][3][e]; // V
            v.z = acc[i][1][e]; // X
            v.w = acc[i][2][e]; // Y
            out[(long long)col * P.n_bases_pad + row] = v;
        }
}

} // namespace ndft
