// Sign-split contraction of the NDFT surface on gfx950 matrix cores.
//
// With z = lag product and sigma = csgn(z) (exact), one surface cell is (Eq. (7),
// Eq. (12a), identity a(x)b = csgn(a) b + a csgn(b)):
//     A[l][p] = sum_i S[p,i] z_l[i] + F[p,i] sigma_l[i],   S = csgn(F), F = W^{ip}.
// Writing S = Sc + j St, F = C + j T and pairing bin p with bin -p (S[-p,i] = conj
// S[p,i], F likewise), four real sums per (base bin b, delay l) give both bins:
//     U = sum Sc z_r + C s_r     X = sum Sc z_i + C s_i
//     Y = sum St z_r + T s_r     V = sum St z_i + T s_i
//     A[l][+b] = (U - V) + j (X + Y),   A[l][-b] = (U + V) + j (X - Y).
// As matrix products: rows A1 = (Sc, C), A2 = (St, T) per base; columns B1 = (z_r, s_r),
// B2 = (z_i, s_i) per delay; U = A1.B1, X = A1.B2, Y = A2.B1, V = A2.B2 with K = samples.
// Symmetric Doppler windows need half the multiply-adds of a complex GEMM over bins;
// one-sided windows need the same.
//
// A work-group owns BT bases x LT delays x one chunk of samples. Each stage of KS
// samples is generated cooperatively into LDS (twiddle rows from integer m = b i mod N,
// lag-product columns from s and r), then each wave multiplies its 32x32 blocks:
//   PREC_FP32:   v_mfma_f32_32x32x2_f32, K = (coef z, coef sigma) per sample.
//   PREC_BF16X2: v_mfma_f32_32x32x16_bf16, per sample 4 terms
//                (Sc, Sc, C_hi, C_lo) . (z_hi, z_lo, sigma, sigma); exact BF16 signs.
// Stages are double-buffered: one barrier per stage. Partial sums of each sample chunk
// go to the workspace; the reduce kernel adds the chunks in a fixed order.
#pragma once

#include "ndft_device.hpp"

namespace ndft {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

enum { PREC_FP32 = 0, PREC_BF16X2 = 1 };
enum { PROD_LAG = 0, PROD_IDENTITY = 1 };

// Ascending runs of base bins: index idx in [off[k], off[k+1]) is base start[k] + idx - off[k].
struct BaseMap {
    int nseg;
    int start[4];
    int off[5];
};

__device__ __forceinline__ int base_of(const BaseMap &bm, int idx)
{
    int b = bm.start[0]; // padding rows (idx >= total) compute a valid, discarded base
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < bm.nseg && idx >= bm.off[k] && idx < bm.off[k + 1]) b = bm.start[k] + (idx - bm.off[k]);
    return b;
}

struct ContractParams {
    const float2 *s;      // lag producer: surveillance [n]; identity producer: x [cols][n]
    const float2 *r;      // lag producer: reference [n]
    long long col_stride; // identity producer: elements between rows of x
    int n;
    int n_cols;           // delays (lag) or rows (identity)
    int tau0;             // first delay (lag)
    int n_bases;
    BaseMap bm;
    int tb, n_coarse;     // two-level twiddle table: fine size 2^tb, coarse entries
    int kchunk, ksplit;   // samples per chunk (multiple of KS), number of chunks
    int tiles_b, tiles_l;
    int n_bases_pad, n_cols_pad;
    float4 *partial;      // [ksplit][n_cols_pad][n_bases_pad] of (U, V, X, Y)
};

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    bf16x2v v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// bf16 of a value and of its remainder: v = hi + lo + O(2^-18 |v|).
__device__ __forceinline__ uint32_t split_bf16(float v)
{
    __bf16 h = (__bf16)v;
    __bf16 l = (__bf16)(v - (float)h);
    bf16x2v p = {h, l};
    return __builtin_bit_cast(uint32_t, p);
}

template <int PREC, int PROD, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
struct ContractCfg {
    static constexpr int NT = 64 * WAVES_B * WAVES_L;
    static constexpr int BT = WAVES_B * WB * 32;
    static constexpr int LT = WAVES_L * WL * 32;
    // stage buffers: KS samples x 2 types x 2 halves x rows x 4 bytes (FP32) or
    // KS/4 groups x 2 x 2 x rows x 16 bytes (BF16): the same byte count.
    static constexpr int STAGE_A_F4 = KS * BT; // float4 units
    static constexpr int STAGE_B_F4 = KS * LT;
    static constexpr int TW_UNITS = BT * KS / 2; // (row, sample pair) units per stage
    static constexpr int LG_UNITS = LT * KS / 2;
    static constexpr int TW_ITERS = (TW_UNITS + NT - 1) / NT;
    static constexpr int LG_ITERS = (LG_UNITS + NT - 1) / NT;
    static_assert(PREC != PREC_BF16X2 || KS % 4 == 0, "BF16 stage is whole 4-sample groups");
    static_assert(KS % 2 == 0, "pairs of samples");
};

template <int PREC, int PROD, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
__global__ __launch_bounds__(64 * WAVES_B * WAVES_L, 1) void contract_kernel(ContractParams P)
{
    using Cfg = ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>;
    constexpr int NT = Cfg::NT, BT = Cfg::BT, LT = Cfg::LT;

    __shared__ float4 bufA[2][Cfg::STAGE_A_F4];
    __shared__ float4 bufB[2][Cfg::STAGE_B_F4];
    extern __shared__ float2 tables[];
    float2 *coarse = tables;
    float2 *fine = tables + P.n_coarse;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wbi = wave % WAVES_B;
    const int wli = wave / WAVES_B;
    const int h = lane >> 5;
    const int l32 = lane & 31;

    int bid = blockIdx.x;
    const int kc = bid % P.ksplit;
    bid /= P.ksplit;
    const int tile_b = bid % P.tiles_b;
    const int tile_l = bid / P.tiles_b;
    const int b0 = tile_b * BT;
    const int c0 = tile_l * LT;
    const int n = P.n;
    const int k_begin = kc * P.kchunk;
    const int k_end = min(n, k_begin + P.kchunk);
    const int nst = (k_end - k_begin + KS - 1) / KS;

    build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, NT);

    // ---- producer state: twiddle units (row, pair) and lag units (col, pair) ----
    int tw_m[Cfg::TW_ITERS], tw_b[Cfg::TW_ITERS], tw_dm[Cfg::TW_ITERS];
#pragma unroll
    for (int it = 0; it < Cfg::TW_ITERS; ++it) {
        int u = tid + it * NT;
        int row = u % BT, pair = u / BT;
        int b = base_of(P.bm, b0 + row);
        long long i0 = (long long)k_begin + 2 * pair;
        tw_b[it] = b;
        tw_m[it] = (int)(((long long)b * i0) % n);
        tw_dm[it] = (int)(((long long)b * KS) % n);
    }

    f32x16 acc[WB][WL][4];
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WL; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][t][e] = 0.0f;

    __syncthreads(); // tables ready

    auto produce = [&](int st, int buf) {
        const int ibase = k_begin + st * KS;
        // twiddle rows
#pragma unroll
        for (int it = 0; it < Cfg::TW_ITERS; ++it) {
            int u = tid + it * NT;
            if (Cfg::TW_UNITS % NT == 0 || u < Cfg::TW_UNITS) {
                int row = u % BT, pair = u / BT;
                int m1 = tw_m[it];
                int m2 = m1 + tw_b[it];
                m2 = m2 >= n ? m2 - n : m2;
                TwSign g1 = twiddle_sign(m1, n), g2 = twiddle_sign(m2, n);
                float2 w1 = twiddle_value(coarse, fine, m1, P.tb, g1);
                float2 w2 = twiddle_value(coarse, fine, m2, P.tb, g2);
                if (PREC == PREC_FP32) {
                    float *A = reinterpret_cast<float *>(bufA[buf]);
                    int s1 = 2 * pair, s2 = 2 * pair + 1;
                    A[((s1 * 2 + 0) * 2 + 0) * BT + row] = (float)g1.c;
                    A[((s1 * 2 + 0) * 2 + 1) * BT + row] = w1.x;
                    A[((s1 * 2 + 1) * 2 + 0) * BT + row] = (float)g1.t;
                    A[((s1 * 2 + 1) * 2 + 1) * BT + row] = w1.y;
                    A[((s2 * 2 + 0) * 2 + 0) * BT + row] = (float)g2.c;
                    A[((s2 * 2 + 0) * 2 + 1) * BT + row] = w2.x;
                    A[((s2 * 2 + 1) * 2 + 0) * BT + row] = (float)g2.t;
                    A[((s2 * 2 + 1) * 2 + 1) * BT + row] = w2.y;
                } else {
                    uint4 *A = reinterpret_cast<uint4 *>(bufA[buf]);
                    int g = pair >> 1, hh = pair & 1;
                    float c1 = (float)g1.c, t1 = (float)g1.t, c2 = (float)g2.c, t2 = (float)g2.t;
                    uint4 a1, a2;
                    a1.x = pack_bf16x2(c1, c1);
                    a1.y = split_bf16(w1.x);
                    a1.z = pack_bf16x2(c2, c2);
                    a1.w = split_bf16(w2.x);
                    a2.x = pack_bf16x2(t1, t1);
                    a2.y = split_bf16(w1.y);
                    a2.z = pack_bf16x2(t2, t2);
                    a2.w = split_bf16(w2.y);
                    A[((g * 2 + 0) * 2 + hh) * BT + row] = a1;
                    A[((g * 2 + 1) * 2 + hh) * BT + row] = a2;
                }
                int mn = tw_m[it] + tw_dm[it];
                tw_m[it] = mn >= n ? mn - n : mn;
            }
        }
        // lag-product (or identity) columns
#pragma unroll
        for (int it = 0; it < Cfg::LG_ITERS; ++it) {
            int u = tid + it * NT;
            if (Cfg::LG_UNITS % NT == 0 || u < Cfg::LG_UNITS) {
                int col = u % LT, pair = u / LT;
                int c = c0 + col;
                int i1 = ibase + 2 * pair, i2 = i1 + 1;
                Lag z1, z2;
                const float2 zero = make_float2(0.0f, 0.0f);
                if (PROD == PROD_LAG) {
                    int d = P.tau0 + min(c, P.n_cols - 1);
                    float2 s1 = i1 < k_end ? P.s[i1] : zero;
                    float2 s2 = i2 < k_end ? P.s[i2] : zero;
                    float2 r1 = (i1 < k_end && i1 - d >= 0) ? P.r[i1 - d] : zero;
                    float2 r2 = (i2 < k_end && i2 - d >= 0) ? P.r[i2 - d] : zero;
                    z1 = lag_product(s1, r1);
                    z2 = lag_product(s2, r2);
                } else {
                    const float2 *x = P.s + (long long)min(c, P.n_cols - 1) * P.col_stride;
                    z1 = identity_entry(i1 < k_end ? x[i1] : zero);
                    z2 = identity_entry(i2 < k_end ? x[i2] : zero);
                }
                if (PREC == PREC_FP32) {
                    float *B = reinterpret_cast<float *>(bufB[buf]);
                    int s1 = 2 * pair, s2 = 2 * pair + 1;
                    B[((s1 * 2 + 0) * 2 + 0) * LT + col] = z1.zr;
                    B[((s1 * 2 + 0) * 2 + 1) * LT + col] = z1.sr;
                    B[((s1 * 2 + 1) * 2 + 0) * LT + col] = z1.zi;
                    B[((s1 * 2 + 1) * 2 + 1) * LT + col] = z1.si;
                    B[((s2 * 2 + 0) * 2 + 0) * LT + col] = z2.zr;
                    B[((s2 * 2 + 0) * 2 + 1) * LT + col] = z2.sr;
                    B[((s2 * 2 + 1) * 2 + 0) * LT + col] = z2.zi;
                    B[((s2 * 2 + 1) * 2 + 1) * LT + col] = z2.si;
                } else {
                    uint4 *B = reinterpret_cast<uint4 *>(bufB[buf]);
                    int g = pair >> 1, hh = pair & 1;
                    uint4 v1, v2;
                    v1.x = split_bf16(z1.zr);
                    v1.y = pack_bf16x2(z1.sr, z1.sr);
                    v1.z = split_bf16(z2.zr);
                    v1.w = pack_bf16x2(z2.sr, z2.sr);
                    v2.x = split_bf16(z1.zi);
                    v2.y = pack_bf16x2(z1.si, z1.si);
                    v2.z = split_bf16(z2.zi);
                    v2.w = pack_bf16x2(z2.si, z2.si);
                    B[((g * 2 + 0) * 2 + hh) * LT + col] = v1;
                    B[((g * 2 + 1) * 2 + hh) * LT + col] = v2;
                }
            }
        }
    };

    auto consume = [&](int buf) {
        const int rowA = wbi * WB * 32 + l32;
        const int colB = wli * WL * 32 + l32;
        if (PREC == PREC_FP32) {
            const float *A = reinterpret_cast<const float *>(bufA[buf]);
            const float *B = reinterpret_cast<const float *>(bufB[buf]);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                float a[WB][2], b[WL][2];
#pragma unroll
                for (int i = 0; i < WB; ++i)
#pragma unroll
                    for (int t = 0; t < 2; ++t) a[i][t] = A[((s * 2 + t) * 2 + h) * BT + rowA + 32 * i];
#pragma unroll
                for (int j = 0; j < WL; ++j)
#pragma unroll
                    for (int t = 0; t < 2; ++t) b[j][t] = B[((s * 2 + t) * 2 + h) * LT + colB + 32 * j];
#pragma unroll
                for (int i = 0; i < WB; ++i)
#pragma unroll
                    for (int j = 0; j < WL; ++j)
#pragma unroll
                        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
                            for (int tb = 0; tb < 2; ++tb)
                                acc[i][j][ta * 2 + tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                    a[i][ta], b[j][tb], acc[i][j][ta * 2 + tb], 0, 0, 0);
            }
        } else {
            const uint4 *A = reinterpret_cast<const uint4 *>(bufA[buf]);
            const uint4 *B = reinterpret_cast<const uint4 *>(bufB[buf]);
#pragma unroll
            for (int g = 0; g < KS / 4; ++g) {
                bf16x8 a[WB][2], b[WL][2];
#pragma unroll
                for (int i = 0; i < WB; ++i)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        a[i][t] = __builtin_bit_cast(bf16x8, A[((g * 2 + t) * 2 + h) * BT + rowA + 32 * i]);
#pragma unroll
                for (int j = 0; j < WL; ++j)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        b[j][t] = __builtin_bit_cast(bf16x8, B[((g * 2 + t) * 2 + h) * LT + colB + 32 * j]);
#pragma unroll
                for (int i = 0; i < WB; ++i)
#pragma unroll
                    for (int j = 0; j < WL; ++j)
#pragma unroll
                        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
                            for (int tb = 0; tb < 2; ++tb)
                                acc[i][j][ta * 2 + tb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    a[i][ta], b[j][tb], acc[i][j][ta * 2 + tb], 0, 0, 0);
            }
        }
    };

    if (nst > 0) {
        produce(0, 0);
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            if (st + 1 < nst) produce(st + 1, (st + 1) & 1);
            consume(st & 1);
            __syncthreads();
        }
    }

    // ---- partial sums of this chunk: lane holds rows 8*(e/4) + 4*h + e%4, column l32 ----
    float4 *out = P.partial + (long long)kc * P.n_cols_pad * P.n_bases_pad;
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            int col = c0 + wli * WL * 32 + 32 * j + l32;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                int row = b0 + wbi * WB * 32 + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
                float4 v;
                v.x = acc[i][j][0][e]; // U = A1.B1
                v.y = acc[i][j][3][e]; // V = A2.B2
                v.z = acc[i][j][1][e]; // X = A1.B2
                v.w = acc[i][j][2][e]; // Y = A2.B1
                out[(long long)col * P.n_bases_pad + row] = v;
            }
        }
}

struct ReduceParams {
    const float4 *partial;
    int ksplit, n_cols_pad, n_bases_pad;
    int n_cols, n_bases;
    BaseMap bm;
    int n, p0n, n_bins;
    float2 *out; // [n_cols][n_bins]
};

// Ordered sum of the chunk partials, then the +b / -b assembly into the output rows.
__global__ __launch_bounds__(256) void reduce_kernel(ReduceParams R)
{
    long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    long long total = (long long)R.n_cols * R.n_bases;
    if (idx >= total) return;
    int bi = (int)(idx % R.n_bases);
    int col = (int)(idx / R.n_bases);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    const long long plane = (long long)R.n_cols_pad * R.n_bases_pad;
    const float4 *p = R.partial + (long long)col * R.n_bases_pad + bi;
    for (int k = 0; k < R.ksplit; ++k) {
        float4 v = p[k * plane];
        a.x += v.x;
        a.y += v.y;
        a.z += v.z;
        a.w += v.w;
    }
    const int b = base_of(R.bm, bi);
    const int n = R.n;
    float2 *row = R.out + (long long)col * R.n_bins;
    int q = b - R.p0n;
    q = q < 0 ? q + n : q;
    if (q < R.n_bins) row[q] = make_float2(a.x - a.y, a.z + a.w);
    int pm = b == 0 ? 0 : n - b;
    if (pm != b) {
        int q2 = pm - R.p0n;
        q2 = q2 < 0 ? q2 + n : q2;
        if (q2 < R.n_bins) row[q2] = make_float2(a.x + a.y, a.z - a.w);
    }
}

} // namespace ndft
