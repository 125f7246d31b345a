// Split-BF16 surface kernel with the lag-product operand built in registers.
//
// The sums are those of the shared-operand contraction (ndft_contract.hpp): for base bin
// b and delay l, U = A1.B1, X = A1.B2, Y = A2.B1, V = A2.B2 over the samples, with twiddle
// rows A1 = (Sc, C), A2 = (St, T) and lag columns B1 = (z_r, sigma_r), B2 = (z_i, sigma_i)
// (Eq. (12a) through the identity a(x)b = csgn(a) b + a csgn(b)). What changes is where
// the operands live:
//   * a work-group is NW waves; wave w owns delays c0 + 32 WL w .. and ALL BT = 32 WB
//     bases of the tile, so a lag-product column is used by exactly one wave: each lane
//     computes its own B fragment (two samples of one delay) in registers, straight from
//     the signed inputs, and never writes it to LDS;
//   * the twiddle operand (shared by every wave) is generated cooperatively into a
//     double-buffered LDS stage, one stage of KS samples ahead of the matrix cores.
// LDS traffic per matrix instruction is then one A fragment (the B side needs none),
// and every lane does the same operand work.
//
// Signs. A lag component z (FP32, one rounding of the exact sum of two Eq. (1)
// operators) carries the exact sign whenever it is non-zero. The kernel takes the sign
// operand from the rounded BF16 high part of z (a few bit operations per pair): exact
// wherever that high part is non-zero. Lanes where a high part is zero (z = 0 or below
// the BF16 range) are flagged per 4-sample group; after the stage, flagged groups are
// recomputed with the exact comparison of the two operator magnitudes (FP64 TwoSum) and
// the difference of the sign operands is added with extra matrix instructions.
// Differences are 0 or +-2 (see Scaling), exact in BF16, and columns that are exactly zero get exact
// zeros (the difference is zero, nothing is added).
//
// Twiddle values come from the two-level table. With TWX (exact table) the table is
// chosen so that every quadrant point m in {0, N/4, N/2, 3N/4} that is an integer is
// reached with a fine index of 0; the table product is then exactly 0 / +-1 there, and
// elsewhere its error (a few FP32 ulp) is far below the smallest non-zero |cos|, |sin|
// (about 1.5 / N; the host allows TWX for N <= 2^20), so the sign operands again come
// from the rounded high parts. Without TWX, signs come from integer quadrant tests.
#pragma once

#include <type_traits>

#include "ndft_contract.hpp"

namespace ndft {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4))); // plain 16-byte loads/stores

// Scaling. Both operands carry their sign terms as +-2 and their value terms halved:
// the stage windows hold input signs as +-1/2 (so every Eq. (1) operator, hence z, comes out
// exactly halved) and the fine twiddle table holds W^r / 2. Products Sc' z' = (2 Sc)(z/2)
// and C' sigma' = (C/2)(2 sigma) are the exact terms. The point is the BF16 pattern of
// +-2, 0x4000: it is one bit of the rounded high part moved into place.

// Sign operands of a BF16 pair v: +-2 where a half is non-zero, +-0 where it is zero.
// The return value's bits 15 and 31 flag the non-zero halves.
__device__ __forceinline__ uint32_t bf16_signs2(uint32_t v, uint32_t &sig)
{
    // a half in [1, 0x7fff] plus 0x7fff sets its bit 15 (no carry between halves)
    const uint32_t t = (v & 0x7fff7fffu) + 0x7fff7fffu;
    sig = ((t >> 1) & 0x40004000u) | (v & 0x80008000u);
    return t;
}

// Twiddle operands of base row b for the sample pair (i, i + 1), m1 = b i mod N,
// m2 = b (i + 1) mod N, from the four table entries (coarse and fine of m1 and m2; the
// fine table holds W / 2): A1 = (Sc pair, Sc pair, C hi pair, C lo pair) and A2 = (St
// pair, St pair, T hi pair, T lo pair), sign operands +-2 (see Scaling).
template <bool TWX>
__device__ __forceinline__ void twiddle_pair_operands(float2 a1, float2 b1, float2 a2, float2 b2, int m1, int m2,
                                                      int n, uint4 &A1, uint4 &A2)
{
    float2 w1 = make_float2(fmaf(a1.x, b1.x, -a1.y * b1.y), fmaf(a1.x, b1.y, a1.y * b1.x));
    float2 w2 = make_float2(fmaf(a2.x, b2.x, -a2.y * b2.y), fmaf(a2.x, b2.y, a2.y * b2.x));
    if (TWX) {
        split_pair(w1.x, w2.x, A1.z, A1.w);
        (void)bf16_signs2(A1.z, A1.x);
        split_pair(w1.y, w2.y, A2.z, A2.w);
        (void)bf16_signs2(A2.z, A2.x);
    } else {
        const TwSign g1 = twiddle_sign(m1, n), g2 = twiddle_sign(m2, n);
        w1.x = g1.c ? w1.x : 0.0f;
        w1.y = g1.t ? w1.y : 0.0f;
        w2.x = g2.c ? w2.x : 0.0f;
        w2.y = g2.t ? w2.y : 0.0f;
        A1.x = pack_bf16x2(2.0f * (float)g1.c, 2.0f * (float)g2.c);
        split_pair(w1.x, w2.x, A1.z, A1.w);
        A2.x = pack_bf16x2(2.0f * (float)g1.t, 2.0f * (float)g2.t);
        split_pair(w1.y, w2.y, A2.z, A2.w);
    }
    A1.y = A1.x;
    A2.y = A2.x;
}

// Lag products of two samples from half-signed inputs (z/2, the operations of
// lag_product4) in the split-BF16 column layout: B1 = (z_r hi pair, z_r lo pair, sign
// pair, sign pair), B2 likewise for z_i. Returns bits 15 and 31 set when all four high
// parts are non-zero.
__device__ __forceinline__ uint32_t lag_pair_operands(const float4 &s1, const float4 &s2, const float4 &r1,
                                                      const float4 &r2, uint4 &B1, uint4 &B2)
{
    const float zr1 = fmaf(s1.x, r1.z, r1.x * s1.z) + fmaf(s1.y, r1.w, r1.y * s1.w);
    const float zi1 = fmaf(s1.y, r1.z, r1.x * s1.w) - fmaf(r1.y, s1.z, s1.x * r1.w);
    const float zr2 = fmaf(s2.x, r2.z, r2.x * s2.z) + fmaf(s2.y, r2.w, r2.y * s2.w);
    const float zi2 = fmaf(s2.y, r2.z, r2.x * s2.w) - fmaf(r2.y, s2.z, s2.x * r2.w);
    split_pair(zr1, zr2, B1.x, B1.y);
    const uint32_t tr = bf16_signs2(B1.x, B1.z);
    B1.w = B1.z;
    split_pair(zi1, zi2, B2.x, B2.y);
    const uint32_t ti = bf16_signs2(B2.x, B2.z);
    B2.w = B2.z;
    return tr & ti;
}

// Sign-operand corrections of a flagged pair: exact sign operands (2 csgn z) minus the
// ones taken from the high parts, as BF16 pairs in {0, +-2} (only the sign dwords are
// non-zero). Returns whether any is non-zero.
__device__ __forceinline__ bool lag_pair_sign_fix(const float4 &s1, const float4 &s2, const float4 &r1,
                                                  const float4 &r2, uint4 &D1, uint4 &D2)
{
    const Lag e1 = lag_product4(s1, r1); // values z/2, exact signs
    const Lag e2 = lag_product4(s2, r2);
    uint32_t hr, lr, hi, li, gr, gi;
    split_pair(e1.zr, e2.zr, hr, lr);
    split_pair(e1.zi, e2.zi, hi, li);
    (void)bf16_signs2(hr, gr);
    (void)bf16_signs2(hi, gi);
    const float dr1 = 2.0f * e1.sr - __uint_as_float(gr << 16);
    const float dr2 = 2.0f * e2.sr - __uint_as_float(gr & 0xffff0000u);
    const float di1 = 2.0f * e1.si - __uint_as_float(gi << 16);
    const float di2 = 2.0f * e2.si - __uint_as_float(gi & 0xffff0000u);
    const uint32_t pr = pack_bf16x2(dr1, dr2), pi = pack_bf16x2(di1, di2);
    D1 = make_uint4(0u, 0u, pr, pr);
    D2 = make_uint4(0u, 0u, pi, pi);
    return (dr1 != 0.0f) | (dr2 != 0.0f) | (di1 != 0.0f) | (di2 != 0.0f);
}

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// Empty instructions that read and redefine a whole register tuple (no code is emitted):
// arithmetic on the value stays after them. Instruction selection would otherwise hoist
// the arithmetic of a later pipeline slot up to the load that feeds it.
__device__ __forceinline__ void pin(float4 &v)
{
    f32x4v t = __builtin_bit_cast(f32x4v, v);
    asm volatile("" : "+v"(t));
    v = __builtin_bit_cast(float4, t);
}
__device__ __forceinline__ void pin(float2 &v)
{
    f32x2v t = __builtin_bit_cast(f32x2v, v);
    asm volatile("" : "+v"(t));
    v = __builtin_bit_cast(float2, t);
}

// (a + b) mod n for 0 <= a, b < n < 2^31: the unsigned minimum of x and x - n.
__device__ __forceinline__ int add_mod(int a, int b, int n)
{
    const unsigned x = (unsigned)(a + b);
    return (int)min(x, x - (unsigned)n);
}

template <int NW, int WB, int WL, int KS, int PF>
struct SurfCfg {
    static constexpr int NT = 64 * NW;
    static constexpr int BT = 32 * WB;
    static constexpr int LT = 32 * WL * NW;
    static constexpr int G = KS / 4;             // 4-sample matrix steps per stage
    static constexpr int STAGE_A = KS * BT;      // uint4 per stage buffer
    static constexpr int TW_UNITS = BT * KS / 2; // (base row, sample pair) per stage
    static constexpr int TWI = (TW_UNITS + NT - 1) / NT;
    // input windows of a stage in LDS: surveillance samples k0 .. k0 + KS + 7 and the
    // reference samples every delay of the tile needs for them
    static constexpr int WS = KS + 8;
    static constexpr int WR = KS + 8 + LT - 1;
    static constexpr int WIN = WS + WR;
    static constexpr int WIN_ITERS = (WIN + NT - 1) / NT;
    static_assert(KS % 8 == 0, "a stage is an even number of 4-sample steps");
    static_assert(TWI <= G, "at most one twiddle unit per step");
    static_assert(2 * KS + 8 <= kTailPad, "the last stage pair and its window stay in the zero tail");
};

// Twiddle source of a tile: generated in the kernel from the table with integer signs
// (TW_GEN) or with signs from the exact table (TW_GEN_EXACT), or copied from planes
// precomputed by plane_build_kernel (TW_PLANES).
enum { TW_GEN = 0, TW_GEN_EXACT = 1, TW_PLANES = 2 };

// Z0: this tile also sums base 0 (see ContractParams::row0). With W^0 = 1 every Eq. (6)
// product is z + csgn z, so the row is the column sum of the lag operands weighted like
// a twiddle row (2 on the value parts, 1/2 on the sign parts: the scaling above), done
// with BF16 dot products on the operands the matrix step consumes.
template <int NW, int WB, int WL, int KS, int PF, int TWM, bool Z0>
__device__ __forceinline__ void surface_bf16_tile(const ContractParams &P, const int kc, const int tile_b,
                                                  const int tile_l,
                                                  uint4 *bufA0, uint4 *bufA1,
                                                  float4 (*win)[SurfCfg<NW, WB, WL, KS, PF>::WIN], float2 *tables,
                                                  const float2 *s_raw, const float2 *r_raw)
{
    using Cfg = SurfCfg<NW, WB, WL, KS, PF>;
    constexpr int NT = Cfg::NT, BT = Cfg::BT, LT = Cfg::LT, G = Cfg::G;
    constexpr bool TWX = TWM == TW_GEN_EXACT;
    constexpr bool PLANES = TWM == TW_PLANES;
    constexpr int TWI = PLANES ? 0 : Cfg::TWI;  // generated twiddle units per thread
    constexpr int PLI = Cfg::STAGE_A / NT;       // plane uint4 per thread per stage
    static_assert(!PLANES || Cfg::STAGE_A % NT == 0, "plane stages split evenly");
    // vector instructions per slot (lag operands ~45 per column block, a twiddle unit
    // ~35) spread over the slot's matrix instructions
    constexpr int VALU_PER_MFMA = (45 * WL + 35 * TWI / G + (Z0 ? 6 * WL : 0) + 4 * WB * WL - 1) / (4 * WB * WL);

    float2 *coarse = tables;
    float2 *fine = PLANES ? nullptr : tables + P.n_coarse;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    const int l32 = lane & 31;
    const int n = P.n;
    const int b0 = tile_b * BT;
    const int c0 = tile_l * LT;
    const int k_begin = kc * P.kchunk;
    const int k_end = min(n, k_begin + P.kchunk);
    // chunks are whole stage pairs except the last one of the record, which reads the
    // zero tail past n
    const int npair = k_end > k_begin ? (k_end - k_begin + 2 * KS - 1) / (2 * KS) : 0;

    if (!PLANES) build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, NT, 0.5f); // W / 2

    // ---- twiddle units: (base row, sample pair) -> LDS slot, base, m of the pair ----
    int tw_off[TWI > 0 ? TWI : 1], tw_b[TWI > 0 ? TWI : 1], tw_m[TWI > 0 ? TWI : 1], tw_dm[TWI > 0 ? TWI : 1];
#pragma unroll
    for (int it = 0; it < TWI; ++it) {
        const int u = min(tid + it * NT, Cfg::TW_UNITS - 1);
        const int row = u % BT, pair = u / BT;
        tw_off[it] = (((pair >> 1) * 2) * 2 + (pair & 1)) * BT + row; // A1; A2 at + 2 BT
        const int b = base_of(P.bm, b0 + row);
        tw_b[it] = b;
        tw_m[it] = (int)(((long long)b * (k_begin + 2 * pair)) % n);
        tw_dm[it] = (int)(((long long)b * KS) % n);
    }

    // ---- lag operand sources: lane (h, l32), column block j: delay d_j ----
    // sample i (pair i, i + 1; i = k0 + 4q + 2h in step q of the stage starting at k0):
    // s[i] and r[i - d_j] (zero outside [0, n)), read from the stage window as Ws[i - k0]
    // and Wr[i - k0 + (dmax - d_j)]
    const int dmax = P.tau0 + min(c0 + LT - 1, P.n_cols - 1);
    int roff[WL], valid0[WL];
#pragma unroll
    for (int j = 0; j < WL; ++j) {
        const int col = min(c0 + (wave * WL + j) * 32 + l32, P.n_cols - 1); // padding repeats
        roff[j] = Cfg::WS + dmax - (P.tau0 + col) + 2 * h;
        valid0[j] = k_begin + 2 * h + 1 - (P.tau0 + col); // >= -sfirst: pair reaches the delay
    }
    // One complex64 load per lane per stage: entry e < WS is s[k0 + e], else r[m] with
    // m = k0 - dmax + e - WS; samples outside [0, n) are zero (r[m < 0] = 0, s past the
    // record), so the loaded index is clamped and the value replaced. Indices past WIN
    // repeat the last entry and are not stored. The store adds the half-scaled signs.
    auto win_load = [&](int k0, float2 (&wv)[Cfg::WIN_ITERS]) {
#pragma unroll
        for (int it = 0; it < Cfg::WIN_ITERS; ++it) {
            const int e = min(tid + it * NT, Cfg::WIN - 1);
            const bool is_s = e < Cfg::WS;
            const int idx = is_s ? k0 + e : k0 - dmax + (e - Cfg::WS);
            const float2 v = (is_s ? s_raw : r_raw)[min(max(idx, 0), n - 1)];
            wv[it] = (idx >= 0 && idx < n) ? v : make_float2(0.0f, 0.0f);
        }
    };
    auto win_store = [&](float4 *w, const float2 (&wv)[Cfg::WIN_ITERS]) {
#pragma unroll
        for (int it = 0; it < Cfg::WIN_ITERS; ++it)
            if (Cfg::WIN % NT == 0 || tid + it * NT < Cfg::WIN) w[tid + it * NT] = with_signs(wv[it], 0.5f);
    };

    // planes of this base tile, from the first stage of this chunk
    const u32x4 *pl_src =
        PLANES ? reinterpret_cast<const u32x4 *>(P.planes) + ((long long)tile_b * P.plane_stages + k_begin / KS) * Cfg::STAGE_A + tid
               : nullptr;

    f32x16 acc[WB][WL][4];
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WL; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][t][e] = 0.0f;

    // A twiddle unit is fetched (four table entries, issued together at the start of a
    // stage so their LDS latency is hidden) and later finished (operands to LDS).
    struct TwFetch {
        float2 a1, b1, a2, b2; // coarse and fine entries of m1 and m2
        int m2;
    };
    TwFetch twf[TWI > 0 ? TWI : 1];
    auto tw_fetch = [&](int it) {
        const int m1 = tw_m[it];
        const int m2 = add_mod(m1, tw_b[it], n);
        const int mask = (1 << P.tb) - 1;
        twf[it].a1 = coarse[m1 >> P.tb];
        twf[it].b1 = fine[m1 & mask];
        twf[it].a2 = coarse[m2 >> P.tb];
        twf[it].b2 = fine[m2 & mask];
        twf[it].m2 = m2;
    };
    auto tw_finish = [&](uint4 *buf, int it) {
        if (Cfg::TW_UNITS % NT == 0 || tid + it * NT < Cfg::TW_UNITS) {
            TwFetch &f = twf[it];
            pin(f.a1);
            pin(f.b1);
            pin(f.a2);
            pin(f.b2);
            const int m1 = tw_m[it];
            uint4 a1, a2;
            twiddle_pair_operands<TWX>(f.a1, f.b1, f.a2, f.b2, m1, f.m2, n, a1, a2);
            buf[tw_off[it]] = a1;
            buf[tw_off[it] + 2 * BT] = a2;
            tw_m[it] = add_mod(m1, tw_dm[it], n);
        }
    };

    struct In {
        float4 s1, s2, r1[WL], r2[WL];
    };
    In in[2];
    auto read_in = [&](const float4 *w, In &x, int q) { // step q of the window's stage
        x.s1 = w[4 * q + 2 * h];
        x.s2 = w[4 * q + 2 * h + 1];
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            x.r1[j] = w[roff[j] + 4 * q];
            x.r2[j] = w[roff[j] + 4 * q + 1];
        }
    };

    // A fragments of one 4-sample step: base block i, operand t (A1, A2)
    struct AFrag {
        bf16x8 a[WB][2];
    };
    auto load_a = [&](const uint4 *buf, int g, AFrag &f) {
#pragma unroll
        for (int i = 0; i < WB; ++i)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                f.a[i][t] = __builtin_bit_cast(bf16x8, buf[((g * 2 + t) * 2 + h) * BT + 32 * i + l32]);
    };
    auto mfma_step = [&](const AFrag &f, const uint4 (&B1)[WL], const uint4 (&B2)[WL]) {
#pragma unroll
        for (int i = 0; i < WB; ++i)
#pragma unroll
            for (int j = 0; j < WL; ++j) {
                const bf16x8 b1 = __builtin_bit_cast(bf16x8, B1[j]);
                const bf16x8 b2 = __builtin_bit_cast(bf16x8, B2[j]);
                acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][0], b1, acc[i][j][0], 0, 0, 0);
                acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][0], b2, acc[i][j][1], 0, 0, 0);
                acc[i][j][2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][1], b1, acc[i][j][2], 0, 0, 0);
                acc[i][j][3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][1], b2, acc[i][j][3], 0, 0, 0);
            }
    };

    // base-0 row: per column block, U (real lag parts) and X (imaginary), over the lane's
    // samples; the two halves h are added at the end
    float z0u[WL], z0x[WL];
#pragma unroll
    for (int j = 0; j < WL; ++j) z0u[j] = z0x[j] = 0.0f;
    const bf16x2v w_val = {(__bf16)2.0f, (__bf16)2.0f}, w_sgn = {(__bf16)0.5f, (__bf16)0.5f};
    auto dot2 = [](uint32_t v, bf16x2v w, float c) {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, v), w, c, false);
    };
    auto z0_step = [&](const uint4 (&B1)[WL], const uint4 (&B2)[WL]) {
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            z0u[j] = dot2(B1[j].z, w_sgn, dot2(B1[j].y, w_val, dot2(B1[j].x, w_val, z0u[j])));
            z0x[j] = dot2(B2[j].z, w_sgn, dot2(B2[j].y, w_val, dot2(B2[j].x, w_val, z0x[j])));
        }
    };

    // Lag operands of one step from its inputs; returns 1 when some lane needs repair.
    struct BFrag {
        uint4 b1[WL], b2[WL];
    };
    // A lane's pair lies wholly before its delay when i + 1 < d: then r reads the zero
    // padding, z = 0 exactly and no repair is needed; such lanes are not flagged (i is the
    // pair's first sample, `sfirst` the step's first sample relative to k_begin).
    auto lag_step = [&](In &x, BFrag &f, int sfirst) -> uint32_t {
        pin(x.s1);
        pin(x.s2);
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            pin(x.r1[j]);
            pin(x.r2[j]);
        }
        uint64_t flag = 0; // lanes (as ballots, so the test stays in scalar registers)
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            const uint32_t nz = lag_pair_operands(x.s1, x.s2, x.r1[j], x.r2[j], f.b1[j], f.b2[j]);
            flag |= __builtin_amdgcn_ballot_w64((nz & 0x80008000u) != 0x80008000u) &
                    __builtin_amdgcn_ballot_w64(sfirst + valid0[j] >= 0);
        }
        return flag != 0 ? 1u : 0u;
    };

    // Exact-sign repair of the flagged steps of one stage (rare: zero lag components), from
    // the stage's input window.
    auto repair = [&](const uint4 *buf, const float4 *w, uint32_t bits) {
        while (bits) {
            const int g = __builtin_ctz(bits);
            bits &= bits - 1;
            In x;
            read_in(w, x, g);
            BFrag D;
            bool any = false;
#pragma unroll
            for (int j = 0; j < WL; ++j)
                any |= lag_pair_sign_fix(x.s1, x.s2, x.r1[j], x.r2[j], D.b1[j], D.b2[j]);
            if (__builtin_amdgcn_ballot_w64(any)) {
                AFrag f;
                load_a(buf, g, f);
                mfma_step(f, D.b1, D.b2);
                if (Z0) z0_step(D.b1, D.b2); // value parts of D are 0
            }
        }
    };

    // Software pipeline over the 4-sample steps g of a stage (slot g): read the inputs of
    // step g + 2 from the stage window (LDS), read the A fragments of step g + 1, build the
    // lag operands of step g + 1, emit a twiddle unit of the next stage, and run the matrix
    // step g on operands prepared in slot g - 1. The next stage's window is fetched from
    // global memory at the start of the stage (one load per lane) and stored at its end.
    // Scheduling barriers keep each slot's reads at its start.
    AFrag fa[2];
    BFrag fb[2];
    uint32_t rare_next = 0; // repair flag of step 0 of the next stage
    int kpair = 0;          // first sample of the current stage pair, from k_begin
    auto stage = [&](auto cbc, auto kstc) {
        constexpr int CB = decltype(cbc)::value;
        constexpr int KST = decltype(kstc)::value;
        // two LDS variables (not one array) so the compiler can tell the buffer the plane
        // copy writes from the one the stage reads
        uint4 *cur = CB ? bufA1 : bufA0;
        uint4 *nxt = CB ? bufA0 : bufA1;
        const float4 *curw = win[CB];
        uint32_t rare = rare_next;
        load_a(cur, 0, fa[0]);
        float2 wv[Cfg::WIN_ITERS]; // next stage's window
        win_load(k_begin + KST + KS + kpair, wv);
        if (PLANES) {
            // next stage's plane block straight into LDS (no registers): the 16 bytes of
            // lane i of a wave land at dst + 16 i, dst wave-uniform
            uint4 *dst = nxt + __builtin_amdgcn_readfirstlane(wave) * 64;
#pragma unroll
            for (int k = 0; k < PLI; ++k)
                __builtin_amdgcn_global_load_lds(pl_src + k * NT,
                                                 (__attribute__((address_space(3))) void *)(dst + k * NT), 16, 0, 0);
            pl_src += Cfg::STAGE_A;
        }
        // twiddle unit it is finished in slot (it G) / TWI and its table entries are read
        // one slot earlier (unit 0: here)
#pragma unroll
        for (int it = 0; it < TWI; ++it)
            if ((it * G) / TWI == 0) tw_fetch(it);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            read_in(curw, in[g & 1], g + 2); // steps G, G + 1 are in this window too
            if (g + 1 < G) load_a(cur, g + 1, fa[(g + 1) & 1]);
#pragma unroll
            for (int it = 0; it < TWI; ++it)
                if ((it * G) / TWI == g + 1) tw_fetch(it);
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t r = lag_step(in[(g + 1) & 1], fb[(g + 1) & 1], kpair + KST + 4 * (g + 1));
            if (g + 1 < G)
                rare |= r << (g + 1);
            else
                rare_next = r;
#pragma unroll
            for (int it = 0; it < TWI; ++it)
                if ((it * G) / TWI == g) tw_finish(nxt, it);
            mfma_step(fa[g & 1], fb[g & 1].b1, fb[g & 1].b2);
            if (Z0) z0_step(fb[g & 1].b1, fb[g & 1].b2);
            // order inside the slot: each matrix instruction followed by a run of vector
            // instructions (the matrix core works while they issue)
#pragma unroll
            for (int k = 0; k < 4 * WB * WL; ++k) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0); // MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, VALU_PER_MFMA, 0); // VALU
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        win_store(win[CB ^ 1], wv);
        if (rare) repair(cur, curw, rare);
        // the plane copy has landed before the barrier publishes it
        if (PLANES) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    };

    __syncthreads(); // tables ready
    if (npair > 0) {
#pragma unroll
        for (int it = 0; it < TWI; ++it) {
            tw_fetch(it);
            tw_finish(bufA0, it);
        }
        if (PLANES) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(bufA0) + tid;
#pragma unroll
            for (int k = 0; k < PLI; ++k) dst[k * NT] = pl_src[k * NT];
            pl_src += Cfg::STAGE_A;
        }
        {
            float2 wv[Cfg::WIN_ITERS];
            win_load(k_begin, wv);
            win_store(win[0], wv);
        }
        __syncthreads();
        read_in(win[0], in[0], 0);
        read_in(win[0], in[1], 1);
        rare_next = lag_step(in[0], fb[0], 0);
        for (int p = 0; p < npair; ++p) {
            stage(std::integral_constant<int, 0>(), std::integral_constant<int, 0>());
            stage(std::integral_constant<int, 1>(), std::integral_constant<int, KS>());
            kpair += 2 * KS;
        }
    }

    // ---- partial sums of this chunk: lane holds rows 8*(e/4) + 4*h + e%4, column l32 ----
    float4 *out = P.partial + (long long)kc * P.n_cols_pad * P.n_bases_pad;
    if (Z0) {
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            const float u = z0u[j] + __shfl_xor(z0u[j], 32);
            const float x = z0x[j] + __shfl_xor(z0x[j], 32);
            const int col = c0 + (wave * WL + j) * 32 + l32;
            if (h == 0) out[(long long)col * P.n_bases_pad] = make_float4(u, 0.0f, x, 0.0f);
        }
    }
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            const int col = c0 + (wave * WL + j) * 32 + l32;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = P.row0 + b0 + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
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
template <int NW, int WB, int WL, int KS, int PF>
__global__ __launch_bounds__(64 * NW, 1) void surface_bf16_kernel(ContractParams P)
{
    using Cfg = SurfCfg<NW, WB, WL, KS, PF>;
    __shared__ uint4 bufA0[Cfg::STAGE_A];
    __shared__ uint4 bufA1[Cfg::STAGE_A];
    __shared__ float4 win[2][Cfg::WIN];
    extern __shared__ float2 tables[];
    int bid = blockIdx.x;
    const int kc = bid % P.ksplit;
    bid /= P.ksplit;
    const int tile_b = bid % P.tiles_b, tile_l = bid / P.tiles_b;
    if (P.row0 && tile_b == 0) {
        if (P.tw_exact)
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN_EXACT, true>(P, kc, tile_b, tile_l, bufA0, bufA1, win, tables,
                                                                      P.s_raw, P.r_raw);
        else
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN, true>(P, kc, tile_b, tile_l, bufA0, bufA1, win, tables, P.s_raw,
                                                                P.r_raw);
    } else {
        if (P.tw_exact)
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN_EXACT, false>(P, kc, tile_b, tile_l, bufA0, bufA1, win, tables,
                                                                       P.s_raw, P.r_raw);
        else
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN, false>(P, kc, tile_b, tile_l, bufA0, bufA1, win, tables,
                                                                 P.s_raw, P.r_raw);
    }
}

// Twiddle operand from planes. Block order keeps the delay tiles that share a plane
// stream on one XCD (blocks are dealt to the XCDs in turn, so blockIdx mod 8 picks it):
// blockIdx = tile_l * grp_stride + (tile_b * ksplit + kc), grp_stride a multiple of 8;
// indices past the last group exit at once.
template <int NW, int WB, int WL, int KS, int PF>
__global__ __launch_bounds__(64 * NW, 1) void surface_bf16_planes_kernel(ContractParams P)
{
    using Cfg = SurfCfg<NW, WB, WL, KS, PF>;
    __shared__ uint4 bufA0[Cfg::STAGE_A];
    __shared__ uint4 bufA1[Cfg::STAGE_A];
    __shared__ float4 win[2][Cfg::WIN];
    const int grp = blockIdx.x % P.grp_stride;
    const int tile_l = blockIdx.x / P.grp_stride;
    if (grp >= P.tiles_b * P.ksplit) return;
    const int tile_b = grp / P.ksplit;
    if (P.row0 && tile_b == 0)
        surface_bf16_tile<NW, WB, WL, KS, PF, TW_PLANES, true>(P, grp % P.ksplit, tile_b, tile_l, bufA0, bufA1, win,
                                                               nullptr, P.s_raw, P.r_raw);
    else
        surface_bf16_tile<NW, WB, WL, KS, PF, TW_PLANES, false>(P, grp % P.ksplit, tile_b, tile_l, bufA0, bufA1, win,
                                                                nullptr, P.s_raw, P.r_raw);
}

// Precompute the twiddle planes: thread t of a block owns units (row, pair) t, t + 256,
// ... of the stage layout and walks `stages_per_block` consecutive stages of base tile
// blockIdx.y, so m = b i mod N advances by b KS mod N per stage.
struct PlaneBuildParams {
    uint4 *planes;
    long long plane_stages;
    int n, tb, n_coarse, tw_exact;
    int stages_per_block;
    BaseMap bm;
};

template <int BT, int KS>
__global__ __launch_bounds__(256) void plane_build_kernel(PlaneBuildParams Q)
{
    extern __shared__ float2 tables[];
    constexpr int STAGE_A = KS * BT;
    constexpr int UNITS = BT * KS / 2;
    float2 *coarse = tables;
    float2 *fine = tables + Q.n_coarse;
    const int n = Q.n;
    build_twiddle_tables(coarse, fine, n, Q.tb, Q.n_coarse, threadIdx.x, 256, 0.5f);
    __syncthreads();
    const long long s0 = (long long)blockIdx.x * Q.stages_per_block;
    const long long s1 = min(s0 + Q.stages_per_block, Q.plane_stages);
    const int mask = (1 << Q.tb) - 1;
    for (int u = threadIdx.x; u < UNITS; u += 256) {
        const int row = u % BT, pair = u / BT;
        const int off = (((pair >> 1) * 2) * 2 + (pair & 1)) * BT + row;
        const int b = base_of(Q.bm, blockIdx.y * BT + row);
        int m1 = (int)(((long long)b * (s0 * KS + 2 * pair)) % n);
        const int dm = (int)(((long long)b * KS) % n);
        uint4 *dst = Q.planes + ((long long)blockIdx.y * Q.plane_stages + s0) * STAGE_A + off;
        for (long long st = s0; st < s1; ++st) {
            const int m2 = add_mod(m1, b, n);
            uint4 a1, a2;
            if (Q.tw_exact)
                twiddle_pair_operands<true>(coarse[m1 >> Q.tb], fine[m1 & mask], coarse[m2 >> Q.tb], fine[m2 & mask],
                                            m1, m2, n, a1, a2);
            else
                twiddle_pair_operands<false>(coarse[m1 >> Q.tb], fine[m1 & mask], coarse[m2 >> Q.tb], fine[m2 & mask],
                                             m1, m2, n, a1, a2);
            dst[0] = a1;
            dst[2 * BT] = a2;
            dst += STAGE_A;
            m1 = add_mod(m1, dm, n);
        }
    }
}

// Persistent form over a batch (same queue protocol as contract_batched_kernel); the
// inputs come straight from the pools (no sign-prep pass).
template <int NW, int WB, int WL, int KS, int PF>
__global__ __launch_bounds__(64 * NW, 1) void surface_bf16_batched_kernel(BatchHeader *hdr,
                                                                          const ContractParams *params,
                                                                          const int4 *items,
                                                                          unsigned long long tag, int plan_id,
                                                                          const float2 *pool_s, const float2 *pool_r)
{
    using Cfg = SurfCfg<NW, WB, WL, KS, PF>;
    __shared__ uint4 bufA0[Cfg::STAGE_A];
    __shared__ uint4 bufA1[Cfg::STAGE_A];
    __shared__ float4 win[2][Cfg::WIN];
    __shared__ int s_item;
    extern __shared__ float2 tables[];
    if (hdr->tag != tag || hdr->plan_id != plan_id) return;
    const int n_items = hdr->n_items;
    for (;;) {
        __syncthreads(); // every thread has read s_item and finished with the LDS buffers
        if (threadIdx.x == 0) s_item = atomicAdd(&hdr->counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int4 w = items[it];
        const ContractParams P = params[__builtin_amdgcn_readfirstlane(w.x)];
        const float2 *s_raw = pool_s + P.s_raw_off, *r_raw = pool_r + P.r_raw_off;
        if (P.tw_exact)
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN_EXACT, false>(P, w.w, w.y, w.z, bufA0, bufA1, win, tables, s_raw,
                                                                       r_raw);
        else
            surface_bf16_tile<NW, WB, WL, KS, PF, TW_GEN, false>(P, w.w, w.y, w.z, bufA0, bufA1, win, tables, s_raw, r_raw);
    }
}

} // namespace ndft
