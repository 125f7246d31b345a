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

enum { PREC_FP32 = 0, PREC_BF16X2 = 1, PREC_FP8 = 2 };
typedef int i32x8 __attribute__((ext_vector_type(8)));
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

// Zero samples after the end of every signed row (covers the reads of the last stages
// and the prefetch past them).
constexpr int kTailPad = 128;

struct ContractParams {
    const float4 *s4;     // signed samples (re, im, sign re, sign im), each row followed
                          // by kTailPad zeros: lag producer: surveillance [n + pad];
                          // identity producer: x [cols][col_stride]
    const float4 *r4;     // lag producer: signed reference with n zeros in front:
                          // r4[n + m] = r[m], r4[j < n] = 0 (so r[m < 0] reads 0)
    long long col_stride; // identity producer: elements between rows of x (>= n + pad)
    int n;
    int n_cols;           // delays (lag) or rows (identity)
    int tau0;             // first delay (lag)
    int n_bases;
    BaseMap bm;
    int tb, n_coarse;     // two-level twiddle table: fine size 2^tb, coarse entries
    int tw_exact;         // table reaches every quadrant point with fine index 0 (see
                          // ndft_surface_bf16.hpp): its products there are exact
    int kchunk, ksplit;   // samples per chunk (multiple of KS), number of chunks
    int tiles_b, tiles_l;
    int n_bases_pad, n_cols_pad;
    float4 *partial;      // [ksplit][n_cols_pad][n_bases_pad] of (U, V, X, Y)
    // FP8: the largest |re| + |im| of the surveillance (or identity rows) and of the
    // reference, as float bits (absmax_kernel); it fixes the data exponent of the e4m3 terms
    const unsigned *absmax;
    // precomputed twiddle operand (register-lag surface kernels with planes): per base
    // tile, `plane_stages` consecutive stage blocks in the LDS order of a stage
    const uint4 *planes;
    long long plane_stages;
    int grp_stride;       // block order: tile_l * grp_stride + (tile_b * ksplit + kc)
    // register-lag surface kernels: 1 when base 0 (twiddle 1 at every sample) is summed on
    // the vector units of the tiles with tile_b = 0 and stored in partial row 0; the matrix
    // rows (bm without base 0) then start at row 1
    int row0;
    // register-lag surface kernels read the complex64 inputs directly (signs are made
    // while a stage window is loaded): s_raw[n], r_raw[n]; batched launches set them from
    // the pools and these offsets
    const float2 *s_raw;
    const float2 *r_raw;
    long long s_raw_off, r_raw_off;
};

// Pack each complex sample with its exact component signs (read by the producers):
// rows of n samples from x (row stride n) go to out with row stride `ostride`, starting
// `lead` elements into each output row; every other output element is zero.
// Signs are scaled by g (1, or 1/2 for the register-lag surface kernel).
__global__ __launch_bounds__(256) void sign_prep_kernel(const float2 *__restrict__ x, float4 *__restrict__ out,
                                                        int n, long long rows, long long ostride, int lead, float g)
{
    long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= rows * ostride) return;
    long long row = k / ostride;
    long long j = k - row * ostride - lead;
    out[k] = (j >= 0 && j < n) ? with_signs(x[row * n + j], g) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Two single-row sign preps in one launch (blockIdx.y 0: x0 -> out0, 1: x1 -> out1), each as
// sign_prep_kernel with rows = 1: out[k] = x[k - lead] with its signs, zero outside [0, n).
struct PrepPair {
    const float2 *x[2];
    float4 *out[2];
    long long ostride[2];
    int lead[2];
};

__global__ __launch_bounds__(256) void sign_prep_pair_kernel(PrepPair Q, int n, float g)
{
    const int y = blockIdx.y;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= Q.ostride[y]) return;
    const long long j = k - Q.lead[y];
    Q.out[y][k] = (j >= 0 && j < n) ? with_signs(Q.x[y][j], g) : make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    bf16x2v v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// bf16 pairs of (a, b) and of their remainders: a = hi.x + lo.x + O(2^-18 |a|).
// (The high parts are read back from the packed word: a BF16 is the upper half of the
// FP32 with the same value.)
__device__ __forceinline__ void split_pair(float a, float b, uint32_t &hi, uint32_t &lo)
{
    bf16x2v h = {(__bf16)a, (__bf16)b};
    hi = __builtin_bit_cast(uint32_t, h);
    // the shift is written out so the compiler takes it from the packed word instead of
    // converting a again
    uint32_t ha_bits;
    asm("v_lshlrev_b32 %0, 16, %1" : "=v"(ha_bits) : "v"(hi));
    const float ha = __uint_as_float(ha_bits);
    const float hb = __uint_as_float(hi & 0xffff0000u);
    bf16x2v l = {(__bf16)(a - ha), (__bf16)(b - hb)};
    lo = __builtin_bit_cast(uint32_t, l);
}

// FP8 (e4m3) form: a value is carried as four e4m3 terms, v = t0 + t1/16 + t2/256 +
// t3/4096 + O(2^-16 |v|) (each term rounds the remaining residual, scaled by 16^j, to
// nearest). For two samples with signs (g1, g2) and values (v1, v2) this returns, per
// term j, the dword of bytes [g1, t_j(v1), g2, t_j(v2)] (SIGN_FIRST, twiddle side) or
// [t_j(v1), g1, t_j(v2), g2] (lag side), so that byte k of the two sides pairs a sign
// with a value; the signs are exact in e4m3.
template <bool SIGN_FIRST>
__device__ __forceinline__ void fp8_terms_pair(float g1, float v1, float g2, float v2, uint32_t d[4])
{
    const int sg = __builtin_amdgcn_cvt_pk_fp8_f32(g1, g2, 0, false);
    float r1 = v1, r2 = v2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int tv = __builtin_amdgcn_cvt_pk_fp8_f32(r1, r2, 0, false);
        d[j] = __builtin_amdgcn_perm((uint32_t)tv, (uint32_t)sg, SIGN_FIRST ? 0x05010400u : 0x01050004u);
        if (j < 3) {
            r1 = (r1 - __builtin_amdgcn_cvt_f32_fp8(tv, 0)) * 16.0f;
            r2 = (r2 - __builtin_amdgcn_cvt_f32_fp8(tv, 1)) * 16.0f;
        }
    }
}

// Data exponent of the FP8 form. Every data component is bounded by M: a lag component
// |z| <= max(|s_r| + |s_i|) + max(|r_r| + |r_i|) (each Eq. (1) operator is |a| + |b|), an
// identity entry by max(|x_r| + |x_i|). The lag side carries z 2^-e with e the exponent
// that puts M / 2^e in [32, 64), where the four-term split holds. In each K block a
// twiddle sign meets a lag value (that product needs weight 2^e) and a twiddle value meets
// a lag sign (weight 1), so e is spread over the operands: the twiddle signs are carried
// as +-2^ea (A side), the lag signs as +-2^-eb (B side), the twiddle values as terms of
// w 2^-x, and the MFMA scales the B block by 2^eb and the A block by 2^x (on top of the
// term weight), with ea + eb + x = e. The sign magnitudes stay exact e4m3 (2^-9 .. 2^8),
// so ea <= 8, eb <= 9; x > 0 (twiddle terms 2^x coarser) only when e > 17, up to 6: M <
// 2^29. Beyond, the data terms are made NaN so the surface is NaN, never silently wrong
// (the API documents the limit).
struct Fp8Exp {
    float a_sign; // 2^ea, twiddle-sign bytes
    float a_val;  // 2^-x, twiddle values
    float b_sign; // 2^-eb, lag-sign bytes
    float b_val;  // 2^-e, lag values (NaN when M is out of range)
    int scale_a;  // x, added to the E8M0 exponent of the term weight
    int scale_b;  // E8M0 exponent of 2^eb
};

__device__ __forceinline__ Fp8Exp fp8_exponent(const unsigned *absmax, bool two)
{
    const float m = __uint_as_float(absmax[0]) + (two ? __uint_as_float(absmax[1]) : 0.0f);
    int e = 0;
    if (m > 0.0f) {
        int ex;
        (void)frexpf(m, &ex); // m = f 2^ex, f in [0.5, 1)
        e = ex - 6;           // m / 2^e = f 2^6 in [32, 64)
    }
    const bool bad = !(m < 0x1p29f); // also NaN or infinity
    e = max(e, -17);
    const int x = min(max(e - 17, 0), 6);
    const int ea = min(max(e - x, -9), 8);
    const int eb = min(e - x - ea, 9);
    Fp8Exp f;
    f.a_sign = ldexpf(1.0f, ea);
    f.a_val = ldexpf(1.0f, -x);
    f.b_sign = ldexpf(1.0f, -eb);
    f.b_val = bad ? __builtin_nanf("") : ldexpf(1.0f, -(ea + eb + x));
    f.scale_a = x;
    f.scale_b = 127 + eb;
    return f;
}

// Largest |re| + |im| of `count` complex samples into *out (float bits; atomic maximum of
// non-negative floats compares as unsigned integers). *out must hold 0 beforehand.
__global__ __launch_bounds__(256) void absmax_kernel(const float2 *__restrict__ x, long long count,
                                                     unsigned *__restrict__ out)
{
    float m = 0.0f;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < count; k += (long long)gridDim.x * 256) {
        const float2 v = x[k];
        m = fmaxf(m, fabsf(v.x) + fabsf(v.y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

__global__ void absmax_zero_kernel(unsigned *out, int count)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) out[k] = 0u;
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
    // producer work per stage: twiddle units (base row, sample pair) and lag-product
    // units (column, sample pair); thread t takes units t, t + NT, ... of each kind
    static constexpr int TW_UNITS = BT * KS / 2;
    static constexpr int LG_UNITS = LT * KS / 2;
    static constexpr int TW_ITERS = (TW_UNITS + NT - 1) / NT;
    static constexpr int LG_ITERS = (LG_UNITS + NT - 1) / NT;
    static_assert(PREC != PREC_BF16X2 || KS % 4 == 0, "BF16 stage is whole 4-sample groups");
    static_assert(PREC != PREC_FP8 || KS % 16 == 0, "FP8 stage is whole 16-sample groups");
    static_assert(KS % 2 == 0, "pairs of samples");
    static_assert(KS <= kTailPad, "the last stage reads at most KS - 1 samples past the record");
};

struct LagIn {
    float4 s1, s2, r1, r2;
};

// Empty instruction that reads the four registers (no code is emitted).
__device__ __forceinline__ void mark_read(const float4 &v)
{
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// BF16 K order inside one lane's 8 elements (a pair of samples i, i+1):
//   A1 = [Sc_i, Sc_i+1, Sc_i, Sc_i+1, C_hi_i, C_hi_i+1, C_lo_i, C_lo_i+1]
//   B1 = [zr_hi_i, zr_hi_i+1, zr_lo_i, zr_lo_i+1, sr_i, sr_i+1, sr_i, sr_i+1]
// so A1.B1 = sum over the pair of Sc z_r + C sigma_r (U); A2 = (St, T) and B2 = (z_i,
// sigma_i) give X, Y, V the same way.
// One work item: the partial sums of BT bases x LT columns over sample chunk kc.
// LDS: two stage buffers for each operand and the twiddle table (caller-provided).
template <int PREC, int PROD, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
__device__ __forceinline__ void contract_tile(const ContractParams &P, const int kc, const int tile_b,
                                              const int tile_l,
                                              float4 (*bufA)[ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>::STAGE_A_F4],
                                              float4 (*bufB)[ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>::STAGE_B_F4],
                                              float2 *tables)
{
    using Cfg = ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>;
    constexpr int NT = Cfg::NT, BT = Cfg::BT, LT = Cfg::LT;
    constexpr int TWI = Cfg::TW_ITERS, LGI = Cfg::LG_ITERS;

    float2 *coarse = tables;
    float2 *fine = tables + P.n_coarse;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wbi = wave % WAVES_B;
    const int wli = wave / WAVES_B;
    const int h = lane >> 5;
    const int l32 = lane & 31;

    const int b0 = tile_b * BT;
    const int c0 = tile_l * LT;
    const int n = P.n;
    const int k_begin = kc * P.kchunk;
    const int k_end = min(n, k_begin + P.kchunk);
    const int nst = (k_end - k_begin + KS - 1) / KS;

    build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, NT);
    Fp8Exp fx;
    if (PREC == PREC_FP8) fx = fp8_exponent(P.absmax, PROD == PROD_LAG);

    // ---- twiddle slots: base row, sample pair, base b, m = b i mod n, step ----
    int tw_row[TWI], tw_pair[TWI], tw_b[TWI], tw_m[TWI], tw_dm[TWI];
#pragma unroll
    for (int it = 0; it < TWI; ++it) {
        int u = min(tid + it * NT, Cfg::TW_UNITS - 1);
        int row = u % BT, pair = u / BT;
        int b = base_of(P.bm, b0 + row);
        long long i0 = (long long)k_begin + 2 * pair;
        tw_row[it] = row;
        tw_pair[it] = pair;
        tw_b[it] = b;
        tw_m[it] = (int)(((long long)b * i0) % n);
        tw_dm[it] = (int)(((long long)b * KS) % n);
    }
    // ---- lag slots: column, sample pair, delay d, row pointer (identity) ----
    int lg_col[LGI], lg_pair[LGI], lg_d[LGI];
    const float4 *lg_x[LGI];
#pragma unroll
    for (int it = 0; it < LGI; ++it) {
        int u = min(tid + it * NT, Cfg::LG_UNITS - 1);
        int col = u % LT;
        int c = min(c0 + col, P.n_cols - 1); // padding columns repeat a valid one
        lg_col[it] = col;
        lg_pair[it] = u / LT;
        lg_d[it] = P.tau0 + c;
        lg_x[it] = PROD == PROD_LAG ? P.s4 : P.s4 + (long long)c * P.col_stride;
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

    // Lag slots load without a branch: padded rows make every address valid and
    // samples outside the record read as zero.
    auto load_lag = [&](int st, LagIn *in) {
        const int ibase = k_begin + st * KS;
#pragma unroll
        for (int it = 0; it < LGI; ++it) {
            int i1 = ibase + 2 * lg_pair[it];
            in[it].s1 = lg_x[it][i1];
            in[it].s2 = lg_x[it][i1 + 1];
            if (PROD == PROD_LAG) {
                const float4 *rr = P.r4 + (n + i1 - lg_d[it]);
                in[it].r1 = rr[0];
                in[it].r2 = rr[1];
            }
        }
    };

    auto produce = [&](int buf, const LagIn *in) {
        // ---- twiddle rows: signs from integer m, values from the table ----
#pragma unroll
        for (int it = 0; it < TWI; ++it) {
            if (Cfg::TW_UNITS % NT == 0 || tid + it * NT < Cfg::TW_UNITS) {
                const int row = tw_row[it], pair = tw_pair[it];
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
                } else if (PREC == PREC_FP8) {
                    // block (16-sample group g, type, term j): 8 dwords per row, dword pair%8
                    uint32_t *A = reinterpret_cast<uint32_t *>(bufA[buf]);
                    const int g = pair >> 3, dw = pair & 7;
                    uint32_t dc[4], dt[4];
                    fp8_terms_pair<true>((float)g1.c * fx.a_sign, w1.x * fx.a_val, (float)g2.c * fx.a_sign,
                                         w2.x * fx.a_val, dc);
                    fp8_terms_pair<true>((float)g1.t * fx.a_sign, w1.y * fx.a_val, (float)g2.t * fx.a_sign,
                                         w2.y * fx.a_val, dt);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        A[((((g * 2 + 0) * 4 + j) * BT) + row) * 8 + dw] = dc[j];
                        A[((((g * 2 + 1) * 4 + j) * BT) + row) * 8 + dw] = dt[j];
                    }
                } else {
                    uint4 *A = reinterpret_cast<uint4 *>(bufA[buf]);
                    int g = pair >> 1, hh = pair & 1;
                    uint4 a1, a2;
                    a1.x = pack_bf16x2((float)g1.c, (float)g2.c);
                    a1.y = a1.x;
                    split_pair(w1.x, w2.x, a1.z, a1.w);
                    a2.x = pack_bf16x2((float)g1.t, (float)g2.t);
                    a2.y = a2.x;
                    split_pair(w1.y, w2.y, a2.z, a2.w);
                    A[((g * 2 + 0) * 2 + hh) * BT + row] = a1;
                    A[((g * 2 + 1) * 2 + hh) * BT + row] = a2;
                }
                int mn = tw_m[it] + tw_dm[it];
                tw_m[it] = mn >= n ? mn - n : mn;
            }
        }
        // ---- lag-product (or identity) columns ----
#pragma unroll
        for (int it = 0; it < LGI; ++it) {
            // the prefetched registers count as read here on every path, so the next
            // prefetch into them never waits on newer loads
            mark_read(in[it].s1);
            mark_read(in[it].s2);
            if (PROD == PROD_LAG) {
                mark_read(in[it].r1);
                mark_read(in[it].r2);
            }
            if (Cfg::LG_UNITS % NT == 0 || tid + it * NT < Cfg::LG_UNITS) {
                const int col = lg_col[it], pair = lg_pair[it];
                Lag z1, z2;
                if (PROD == PROD_LAG) {
                    z1 = lag_product4(in[it].s1, in[it].r1);
                    z2 = lag_product4(in[it].s2, in[it].r2);
                } else {
                    z1 = identity_entry(in[it].s1);
                    z2 = identity_entry(in[it].s2);
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
                } else if (PREC == PREC_FP8) {
                    uint32_t *B = reinterpret_cast<uint32_t *>(bufB[buf]);
                    const int g = pair >> 3, dw = pair & 7;
                    uint32_t dr[4], di[4];
                    fp8_terms_pair<false>(z1.sr * fx.b_sign, z1.zr * fx.b_val, z2.sr * fx.b_sign, z2.zr * fx.b_val,
                                          dr);
                    fp8_terms_pair<false>(z1.si * fx.b_sign, z1.zi * fx.b_val, z2.si * fx.b_sign, z2.zi * fx.b_val,
                                          di);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        B[((((g * 2 + 0) * 4 + j) * LT) + col) * 8 + dw] = dr[j];
                        B[((((g * 2 + 1) * 4 + j) * LT) + col) * 8 + dw] = di[j];
                    }
                } else {
                    uint4 *B = reinterpret_cast<uint4 *>(bufB[buf]);
                    int g = pair >> 1, hh = pair & 1;
                    uint4 v1, v2;
                    split_pair(z1.zr, z2.zr, v1.x, v1.y);
                    v1.z = pack_bf16x2(z1.sr, z2.sr);
                    v1.w = v1.z;
                    split_pair(z1.zi, z2.zi, v2.x, v2.y);
                    v2.z = pack_bf16x2(z1.si, z2.si);
                    v2.w = v2.z;
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
        } else if (PREC == PREC_FP8) {
            // The f8f6f4 instruction scales the first 16 bytes of every lane with the E8M0
            // value of the lane in half 0 and the last 16 bytes with that of half 1. Lane
            // half h takes samples 8h .. 8h+7 of the 16-sample group: term j0 = 2 mm in
            // bytes 0-15, term j1 = 2 mm + 1 in bytes 16-31; scale 2^(-4 j) restores the term
            // weight on the twiddle side (the signs themselves are unscaled operands).
            const uint4 *A = reinterpret_cast<const uint4 *>(bufA[buf]);
            const uint4 *B = reinterpret_cast<const uint4 *>(bufB[buf]);
#pragma unroll
            for (int g = 0; g < KS / 16; ++g) {
#pragma unroll
                for (int mm = 0; mm < 2; ++mm) {
                    const int j0 = 2 * mm, j1 = 2 * mm + 1;
                    const int scale_a = 127 - 4 * (2 * mm + h) + fx.scale_a;
                    i32x8 a[WB][2], b[WL][2];
#pragma unroll
                    for (int i = 0; i < WB; ++i)
#pragma unroll
                        for (int tt = 0; tt < 2; ++tt) {
                            uint4 lo = A[(((g * 2 + tt) * 4 + j0) * BT + rowA + 32 * i) * 2 + h];
                            uint4 hi = A[(((g * 2 + tt) * 4 + j1) * BT + rowA + 32 * i) * 2 + h];
                            a[i][tt] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                                             (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                        }
#pragma unroll
                    for (int jj = 0; jj < WL; ++jj)
#pragma unroll
                        for (int tt = 0; tt < 2; ++tt) {
                            uint4 lo = B[(((g * 2 + tt) * 4 + j0) * LT + colB + 32 * jj) * 2 + h];
                            uint4 hi = B[(((g * 2 + tt) * 4 + j1) * LT + colB + 32 * jj) * 2 + h];
                            b[jj][tt] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                                              (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                        }
#pragma unroll
                    for (int i = 0; i < WB; ++i)
#pragma unroll
                        for (int jj = 0; jj < WL; ++jj)
#pragma unroll
                            for (int ta = 0; ta < 2; ++ta)
#pragma unroll
                                for (int tb = 0; tb < 2; ++tb)
                                    acc[i][jj][ta * 2 + tb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                        a[i][ta], b[jj][tb], acc[i][jj][ta * 2 + tb], 0, 0, 0, scale_a, 0,
                                        fx.scale_b);
                }
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

    // One pipeline step with compile-time buffer indices (so the generator's LDS
    // writes are known not to alias the multiply's LDS reads): inputs of stage st+1
    // are in `cur`; fetch stage st+2 into `nxt`, generate stage st+1 into buffer PB,
    // multiply stage st from buffer CB, then one barrier.
    LagIn inA[LGI], inB[LGI];
    __syncthreads(); // tables ready
    if (nst > 0) {
        load_lag(0, inB);
        if (nst > 1) load_lag(1, inA);
        produce(0, inB);
        __syncthreads();
        // Steady state: every step prefetches stage st+2, generates stage st+1 and
        // multiplies stage st; the scheduling barriers keep each prefetch ahead of the
        // generator so its registers stay separate from the stage being generated.
        int st = 0;
        for (; st + 3 < nst; st += 2) {
            load_lag(st + 2, inB);
            __builtin_amdgcn_sched_barrier(0);
            produce(1, inA);
            consume(0);
            __syncthreads();
            load_lag(st + 3, inA);
            __builtin_amdgcn_sched_barrier(0);
            produce(0, inB);
            consume(1);
            __syncthreads();
        }
        // the last one to three stages
        for (; st < nst; st += 2) {
            if (st + 2 < nst) load_lag(st + 2, inB);
            if (st + 1 < nst) produce(1, inA);
            consume(0);
            __syncthreads();
            if (st + 1 < nst) {
                if (st + 2 < nst) produce(0, inB);
                consume(1);
                __syncthreads();
            }
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

// One tile per work-group: blockIdx.x = (tile_l * tiles_b + tile_b) * ksplit + kc.
template <int PREC, int PROD, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
__global__ __launch_bounds__(64 * WAVES_B * WAVES_L, 1) void contract_kernel(ContractParams P)
{
    using Cfg = ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>;
    __shared__ float4 bufA[2][Cfg::STAGE_A_F4];
    __shared__ float4 bufB[2][Cfg::STAGE_B_F4];
    extern __shared__ float2 tables[];
    int bid = blockIdx.x;
    const int kc = bid % P.ksplit;
    bid /= P.ksplit;
    contract_tile<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>(P, kc, bid % P.tiles_b, bid / P.tiles_b, bufA, bufB,
                                                            tables);
}

// Header at the start of a batched workspace (written by the prepare call).
struct BatchHeader {
    int counter;      // work-item queue, reset to 0 before each run
    int n_items;
    int n_cpi;
    int plan_id;
    unsigned long long tag; // identifies the prepare call that wrote the tables
    int status;             // device planner: 0, or why the batch did not run (ndft_status)
    int pad;
};

// Persistent form for a batch of surfaces: each work-group takes items (cpi, tile_b,
// tile_l, kc) from an atomic counter until the list is exhausted. Items are ordered by
// decreasing sample count so the longest chunks start first. Every work-group leaves
// the loop once the counter passes n_items; a header written by another prepare call
// (tag or plan mismatch) makes the kernel do nothing.
template <int PREC, int PROD, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
__global__ __launch_bounds__(64 * WAVES_B * WAVES_L, 1) void contract_batched_kernel(
    BatchHeader *hdr, const ContractParams *params, const int4 *items, unsigned long long tag, int plan_id)
{
    using Cfg = ContractCfg<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>;
    __shared__ float4 bufA[2][Cfg::STAGE_A_F4];
    __shared__ float4 bufB[2][Cfg::STAGE_B_F4];
    __shared__ int s_item;
    extern __shared__ float2 tables[];
    if (hdr->tag != tag || hdr->plan_id != plan_id) return;
    const int n_items = hdr->n_items;
    for (;;) {
        __syncthreads(); // every thread has read s_item and finished with the LDS buffers
        if (threadIdx.x == 0) s_item = atomicAdd(&hdr->counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item); // uniform: scalar loads below
        if (it >= n_items) break;
        const int4 w = items[it];
        const ContractParams P = params[__builtin_amdgcn_readfirstlane(w.x)];
        contract_tile<PREC, PROD, WAVES_B, WAVES_L, WB, WL, KS>(P, w.w, w.y, w.z, bufA, bufB, tables);
    }
}

// Resets the work queue and the FP8 data maxima of the surfaces (absmax: count words,
// may be null).
__global__ void batch_reset_kernel(BatchHeader *hdr, unsigned *absmax, int count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) hdr->counter = 0;
    if (absmax)
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) absmax[k] = 0u;
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
__device__ __forceinline__ void reduce_element(const ReduceParams &R, long long idx)
{
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

__global__ __launch_bounds__(256) void reduce_kernel(ReduceParams R)
{
    reduce_element(R, (long long)blockIdx.x * 256 + threadIdx.x);
}

// Batched: blockIdx.y selects the surface; its rows start at out_off[y] in out_pool.
__global__ __launch_bounds__(256) void reduce_batched_kernel(const BatchHeader *hdr, const ReduceParams *rp,
                                                             const long long *out_off, float2 *out_pool,
                                                             unsigned long long tag)
{
    if (hdr->tag != tag) return;
    ReduceParams R = rp[blockIdx.y];
    R.out = out_pool + out_off[blockIdx.y];
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < (long long)R.n_cols * R.n_bases;
         idx += (long long)gridDim.x * 256)
        reduce_element(R, idx);
}

// Batched sign prep: blockIdx.y selects the surface; x and out rows as sign_prep_kernel.
struct PrepDesc {
    long long src_off; // offset of the input row in its pool (complex elements)
    float4 *out;
    int n, lead;
    long long ostride;
    float g;          // sign scale
    unsigned *absmax; // FP8 plans: the row's largest |re| + |im| (float bits), else null
};

__global__ __launch_bounds__(256) void prep_batched_kernel(const BatchHeader *hdr, const PrepDesc *pd,
                                                           const float2 *pool_s, const float2 *pool_r,
                                                           unsigned long long tag)
{
    if (hdr->tag != tag) return;
    const PrepDesc D = pd[blockIdx.y];
    const float2 *x = (blockIdx.y & 1) ? pool_r : pool_s; // even: surveillance, odd: reference
    x += D.src_off;
    float m = 0.0f;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < D.ostride; k += (long long)gridDim.x * 256) {
        long long j = k - D.lead;
        const float2 v = (j >= 0 && j < D.n) ? x[j] : make_float2(0.f, 0.f);
        m = fmaxf(m, fabsf(v.x) + fabsf(v.y));
        D.out[k] = (j >= 0 && j < D.n) ? with_signs(v, D.g) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (D.absmax) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(D.absmax, __float_as_uint(m));
    }
}

} // namespace ndft
