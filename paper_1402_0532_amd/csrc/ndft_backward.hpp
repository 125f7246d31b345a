// Adjoint of the Eq. (12a) surface with respect to the reference and surveillance
// inputs, with the almost-everywhere derivative d(x (x) y)/dx = sign(y) at every
// operator node (the sign functions are held constant).
//
// With G[l][q] = dL/dRe A + j dL/dIm A, the outer operator of Eq. (6) gives
//     dz[l][i] = sum_q conj(S[p_q, i]) G[l][q],        S = csgn(W^{i p}),
// and the lag product z = s (x) conj(r) gives
//     grad_r[m] = sum_l conj(dz[l][m + d_l]) csgn(s[m + d_l]),
//     grad_s[i] = sum_l dz[l][i] csgn(r[i - d_l]).
// No lag-product value enters. Bins p and -p share S up to conjugation, so per base
// bin b, with Gp = G[l][bin +b] and Gm = G[l][bin -b] (0 when not requested):
//     dz[l][i] = sum_b Sc[b,i] E[l][b] + St[b,i] O[l][b],  E = Gp + Gm,  O = j (Gm - Gp),
// a real matrix product whose second operand (Sc, St) is exactly ternary.
#pragma once

#include "ndft_contract.hpp"

namespace ndft {

// E/O operand per (base index, delay), zero for padding bases:
// eo[bi][l] = (E_r, E_i, O_r, O_i).
__global__ __launch_bounds__(256) void adj_prep_kernel(const float2 *__restrict__ G, int n_tau, int n_dop,
                                                       int n, int p0n, BaseMap bm, int n_bases, int n_bases_pad,
                                                       float4 *__restrict__ eo)
{
    long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= (long long)n_bases_pad * n_tau) return;
    int bi = (int)(k / n_tau);
    int l = (int)(k % n_tau);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (bi < n_bases) {
        int b = base_of(bm, bi);
        float2 gp = make_float2(0.f, 0.f), gm = make_float2(0.f, 0.f);
        int q = b - p0n;
        q = q < 0 ? q + n : q;
        if (q < n_dop) gp = G[(long long)l * n_dop + q];
        int bm2 = b == 0 ? 0 : n - b;
        if (bm2 != b) {
            int q2 = bm2 - p0n;
            q2 = q2 < 0 ? q2 + n : q2;
            if (q2 < n_dop) gm = G[(long long)l * n_dop + q2];
        }
        v.x = gp.x + gm.x;
        v.y = gp.y + gm.y;
        v.z = -(gm.y - gp.y);
        v.w = gm.x - gp.x;
    }
    eo[k] = v;
}

struct AdjParams {
    const float4 *eo; // [n_bases_pad][n_tau]
    BaseMap bm;
    int n, n_tau, n_bases_pad;
    double inv_n; // 1 / n rounded
    float2 *dz;   // [n_tau][n]
};

// dz tile: 64 delays x 64 samples per work-group (4 waves of 32 x 32), K = bases.
//   PREC_FP32:   v_mfma_f32_32x32x2_f32, one base per step: k = (E term, O term).
//   PREC_BF16X2: v_mfma_f32_32x32x16_bf16, lane k order for bases (b, b+1):
//                [E_hi_b, E_hi_b+1, E_lo_b, E_lo_b+1, O_hi_b, O_hi_b+1, O_lo_b, O_lo_b+1]
//                against [Sc_b, Sc_b+1, Sc_b, Sc_b+1, St_b, St_b+1, St_b, St_b+1].
template <int PREC>
__global__ __launch_bounds__(256, 2) void adj_contract_kernel(AdjParams P)
{
    constexpr int LT = 64, IT = 64, KB = 16, JB = IT / 64; // delays, samples, bases per stage
    constexpr int AIT = KB * LT / 256;        // E/O loads per thread and stage
    __shared__ float4 sA[KB][LT];             // E/O of the stage's bases
    __shared__ float2 sB[KB][IT];             // (Sc, St) of the stage's bases
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int wl = wave & 1, wi = wave >> 1; // wave tile: 32 delays x 32 JB samples
    const int tiles_l = (P.n_tau + LT - 1) / LT;
    const int l0 = (blockIdx.x % tiles_l) * LT;
    const int i0 = (blockIdx.x / tiles_l) * IT;
    const int n = P.n;

    f32x16 acc[JB][2]; // [sample block][re, im]
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[j][c][e] = 0.0f;

    // E/O rows of a stage (64 delays x 16 bases, zero past the delays and padded bases),
    // loaded into registers one stage ahead
    auto load_eo = [&](int kb0, float4 (&v)[AIT]) {
#pragma unroll
        for (int t = 0; t < AIT; ++t) {
            const int u = tid + 256 * t, k = u / LT, l = u % LT;
            v[t] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (kb0 + k < P.n_bases_pad && l0 + l < P.n_tau) v[t] = P.eo[(long long)(kb0 + k) * P.n_tau + l0 + l];
        }
    };
    float4 pre[AIT];
    load_eo(0, pre);
    for (int kb0 = 0; kb0 < P.n_bases_pad; kb0 += KB) {
#pragma unroll
        for (int t = 0; t < AIT; ++t) {
            const int u = tid + 256 * t;
            sA[u / LT][u % LT] = pre[t];
        }
        // sign columns (16 bases x 64 samples; a thread takes 4 consecutive samples of one
        // base); padding bases meet zero E/O rows
        static_assert(KB * IT == 4 * 256, "four signs per thread");
        {
            const int k = tid / (IT / 4), c = (tid % (IT / 4)) * 4;
            const int b = base_of(P.bm, min(kb0 + k, P.n_bases_pad - 1));
            const int i = min(i0 + c, n - 1);
            // m = b i mod n: the product (< 2^48) and the remainder are exact in FP64, the
            // quotient from the rounded reciprocal is off by at most one either way
            const double prod = (double)b * (double)i;
            double rem = fma(-floor(prod * P.inv_n), (double)n, prod);
            rem = rem < 0.0 ? rem + (double)n : (rem >= (double)n ? rem - (double)n : rem);
            int m = (int)rem;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                TwSign g = twiddle_sign(m, n);
                sB[k][c + e] = make_float2((float)g.c, (float)g.t);
                // next sample (clamped at the last one like i): m + b mod n
                if (i0 + c + e + 1 < n) {
                    m += b;
                    m = m >= n ? m - n : m;
                }
            }
        }
        __syncthreads();
        if (kb0 + KB < P.n_bases_pad) load_eo(kb0 + KB, pre); // in flight during the products
        if (PREC == PREC_FP32) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                float4 e = sA[k][wl * 32 + l32];
                float ar = h ? e.z : e.x; // E_r or O_r
                float ai = h ? e.w : e.y; // E_i or O_i
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    float2 sg = sB[k][wi * 32 * JB + 32 * j + l32];
                    float bv = h ? sg.y : sg.x; // Sc or St
                    acc[j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bv, acc[j][0], 0, 0, 0);
                    acc[j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bv, acc[j][1], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < KB; k += 4) {
                // lane half h takes bases k + 2h, k + 2h + 1
                float4 e1 = sA[k + 2 * h][wl * 32 + l32];
                float4 e2 = sA[k + 2 * h + 1][wl * 32 + l32];
                uint4 ar, ai;
                split_pair(e1.x, e2.x, ar.x, ar.y);
                split_pair(e1.z, e2.z, ar.z, ar.w);
                split_pair(e1.y, e2.y, ai.x, ai.y);
                split_pair(e1.w, e2.w, ai.z, ai.w);
                bf16x8 va = __builtin_bit_cast(bf16x8, ar), vi = __builtin_bit_cast(bf16x8, ai);
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    float2 s1 = sB[k + 2 * h][wi * 32 * JB + 32 * j + l32];
                    float2 s2 = sB[k + 2 * h + 1][wi * 32 * JB + 32 * j + l32];
                    uint4 bv;
                    bv.x = pack_bf16x2(s1.x, s2.x);
                    bv.y = bv.x;
                    bv.z = pack_bf16x2(s1.y, s2.y);
                    bv.w = bv.z;
                    bf16x8 vb = __builtin_bit_cast(bf16x8, bv);
                    acc[j][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va, vb, acc[j][0], 0, 0, 0);
                    acc[j][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vi, vb, acc[j][1], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // rows = delays 8*(e/4) + 4*h + e%4, column = sample l32
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        int i = i0 + wi * 32 * JB + 32 * j + l32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int l = l0 + wl * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
            if (l < P.n_tau && i < n) P.dz[(long long)l * n + i] = make_float2(acc[j][0][e], acc[j][1][e]);
        }
    }
}

// grad_r[m] = sum_l conj(dz[l][m + d_l]) csgn(s[m + d_l]); grad_s[i] = sum_l dz[l][i] csgn(r[i - d_l]).
// A block takes kAdjBandOut consecutive outputs; its kAdjBandGroups thread groups each sum
// one range of delays (ascending), and the group sums are added in group order, so the
// result does not depend on the launch. Lanes of a group read consecutive samples.
constexpr int kAdjBandOut = 32, kAdjBandGroups = 16;

__global__ __launch_bounds__(kAdjBandOut * kAdjBandGroups) void adj_band_kernel(
    const float2 *__restrict__ dz, const float2 *__restrict__ s, const float2 *__restrict__ r, int n, int tau0,
    int n_tau, float2 *__restrict__ grad_r, float2 *__restrict__ grad_s)
{
    __shared__ float4 part[kAdjBandGroups][kAdjBandOut];
    const int lane = threadIdx.x % kAdjBandOut, grp = threadIdx.x / kAdjBandOut;
    const int k = blockIdx.x * kAdjBandOut + lane;
    const int per = (n_tau + kAdjBandGroups - 1) / kAdjBandGroups;
    const int l0 = min(n_tau, grp * per), l1 = min(n_tau, l0 + per);
    float gr = 0.f, gi = 0.f, hr = 0.f, hi = 0.f; // grad_r, grad_s partial sums
    if (k < n) {
        for (int l = l0; l < l1; ++l) {
            const int i = k + tau0 + l; // grad_r: sample i = m + d_l
            if (i < n) {
                const float2 z = dz[(long long)l * n + i];
                const float2 sv = s[i];
                const float sr = sgnf(sv.x), si = sgnf(sv.y);
                gr += z.x * sr + z.y * si;
                gi += z.x * si - z.y * sr;
            }
            const int m = k - tau0 - l; // grad_s: reference index m = i - d_l
            if (grad_s && m >= 0) {
                const float2 z = dz[(long long)l * n + k];
                const float2 rv = r[m];
                const float rr = sgnf(rv.x), ri = sgnf(rv.y);
                hr += z.x * rr - z.y * ri;
                hi += z.x * ri + z.y * rr;
            }
        }
    }
    part[grp][lane] = make_float4(gr, gi, hr, hi);
    __syncthreads();
    if (grp == 0 && k < n) {
        float4 t = part[0][lane];
#pragma unroll
        for (int g = 1; g < kAdjBandGroups; ++g) {
            const float4 u = part[g][lane];
            t.x += u.x;
            t.y += u.y;
            t.z += u.z;
            t.w += u.w;
        }
        grad_r[k] = make_float2(t.x, t.y);
        if (grad_s) grad_s[k] = make_float2(t.z, t.w);
    }
}

} // namespace ndft
