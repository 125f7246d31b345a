// Decimated DFT of the lag-product rows for transform length L = 512 (N a multiple of 512,
// at most 1024 requested bins): the fast path of dft12b_kernel (same sum, same readings):
//   A[l][p] = sum_{m < M} W^{m p} Y_m[p mod 512],  Y_m[k] = sum_{t < 512} z[m + M t] W_512^{t k},
// N = 512 M, z the lag products of delay d (DFT_LAG: the Eq. (12b) surface) or their exact
// signs (DFT_CODES: the twiddle half of the Eq. (12a) and Eq. (12c) sign-split forms, bin
// p = 0 left out, see ndft_dft12b.hpp).
//
// One work-group of 256 threads owns a whole delay row at a time and keeps its bins in
// registers, so no partial surfaces are written. DFT_LAG reads the inputs with their exact
// signs (a sign-prep pass: s4[n], and r4[2 n] with n zeros in front, so a delayed reference
// needs no bounds test); DFT_CODES reads the 2-bit sign codes the twiddle-sign kernel wrote
// for the same call in the packed layout (half a byte a sample instead of 32 bytes, a delay
// row contiguous, and no lag arithmetic). Both go
// through buffer loads whose scalar offset carries the stride of the samples a lane takes.
// The phases go in groups of 16; each 512-point transform is done as 32 x 16 (t = 16 a + b,
// k = c + 32 e):
//   pass 1: thread (j, b) loads the 32 samples a of transform j with residue b, makes their
//           lag products (or decodes their signs), takes the 32-point DFT over a in registers
//           and turns output c by W_512^{b c};
//   pass 2: after one exchange through LDS, thread (j, c) takes the 16-point DFT over b for
//           two columns c, giving Y_j[c + 32 e];
//   bins:   after a second exchange, each thread adds W^{m0 p} sum_j (W^p)^j Y_j[p mod 512]
//           for its bins, the inner sum by Horner's rule (four fused multiply-adds a phase),
//           the group's factor W^{m0 p} from the table.
// Two LDS exchanges and four barriers per 8192 samples, no inner-twiddle passes over LDS.
//
// LDS: pass-1 buffer at (c 16 + b) 17 + j (the 16 lanes of a row j are consecutive, the
// four b of a wave 17 apart); pass-2 buffer at j 513 + k (the 16 lanes of one column c
// write rows j 2 banks apart: 513 float2 is 1026 words, 2 more than a multiple of 32). The W_N
// table is the two-level one of ndft_device.hpp; W_512^k is a table of its own.
#pragma once

#include "ndft_contract.hpp"
#include "ndft_dft12b.hpp"

namespace ndft {

// The twiddle-sign half's partial planes (DFT_CODES): [ksplit][cols_pad][bases_pad] float4
// (U, V, X, Y) sums over sample ranges, rows in the order of bm. The whole-row kernel adds
// them to its bins itself (the ordered sum and +b / -b assembly of reduce_element), so the
// surface is written once. part == nullptr: no planes (the surface is written or added to
// as P.accumulate says).
struct TsumParams {
    const float4 *part;
    int ksplit, cols_pad, bases_pad;
    BaseMap bm;
};

// Row of base b in a base map (b is one of its bases).
__device__ __forceinline__ int row_of_base(const BaseMap &bm, int b)
{
    int r = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < bm.nseg && b >= bm.start[k] && b - bm.start[k] < bm.off[k + 1] - bm.off[k])
            r = bm.off[k] + (b - bm.start[k]);
    return r;
}

constexpr int kD5Threads = 256;
constexpr int kD5Group = 16;      // transforms per group
constexpr int kD5MaxBins = 1024;  // requested bins (4 per thread)
constexpr int kD5X = 32 * 16 * 17;
constexpr int kD5YS = 513;

// o times W_32^e = e^{-2 pi j e / 32} (e a constant after unrolling; 0 <= e < 32).
__device__ __forceinline__ float2 mul_w32(float2 o, int e)
{
    // cos and sin of 2 pi k / 32, k = 0 .. 8
    constexpr float C[9] = {1.0f,
                            0.98078528040323044913f,
                            0.92387953251128675613f,
                            0.83146961230254523708f,
                            0.70710678118654752440f,
                            0.55557023301960222474f,
                            0.38268343236508977173f,
                            0.19509032201612826785f,
                            0.0f};
    float sg = 1.0f;
    if (e >= 16) { // W_32^{e} = -W_32^{e - 16}
        e -= 16;
        sg = -1.0f;
    }
    if (e == 0) return make_float2(sg * o.x, sg * o.y);
    if (e == 8) return make_float2(sg * o.y, -sg * o.x); // -j
    if (e == 4) {
        const float h = sg * C[4];
        return make_float2(h * (o.x + o.y), h * (o.y - o.x));
    }
    if (e == 12) {
        const float h = sg * C[4];
        return make_float2(h * (o.y - o.x), -h * (o.x + o.y));
    }
    // e in 1..15: cos = C[e] (e <= 8) or -C[16 - e]; sin = C[8 - e] (e <= 8) or C[e - 8]
    const float cs = sg * (e <= 8 ? C[e] : -C[16 - e]);
    const float sn = sg * (e <= 8 ? C[8 - e] : C[e - 8]);
    return make_float2(fmaf(o.x, cs, o.y * sn), fmaf(o.y, cs, -(o.x * sn)));
}

// In-register DFT of 16 points (4 x 4) and of 32 points (8 x 4): input a = R2 a1 + a2,
// output c = c1 + R1 c2, X[c] = sum_a2 W_N^{a2 c1} W_R2^{a2 c2} sum_a1 u[R2 a1 + a2] W_R1^{a1 c1}.
__device__ __forceinline__ void reg_dft16(float2 (&u)[16])
{
    float2 v[4][4];
#pragma unroll
    for (int a2 = 0; a2 < 4; ++a2) {
        v[a2][0] = u[a2];
        v[a2][1] = u[4 + a2];
        v[a2][2] = u[8 + a2];
        v[a2][3] = u[12 + a2];
        dft4(v[a2][0], v[a2][1], v[a2][2], v[a2][3]);
#pragma unroll
        for (int c1 = 1; c1 < 4; ++c1) v[a2][c1] = mul_w32(v[a2][c1], 2 * a2 * c1); // W_16^{a2 c1}
    }
#pragma unroll
    for (int c1 = 0; c1 < 4; ++c1) {
        float2 t0 = v[0][c1], t1 = v[1][c1], t2 = v[2][c1], t3 = v[3][c1];
        dft4(t0, t1, t2, t3);
        u[c1] = t0;
        u[c1 + 4] = t1;
        u[c1 + 8] = t2;
        u[c1 + 12] = t3;
    }
}

__device__ __forceinline__ void reg_dft32(float2 (&u)[32])
{
    float2 v[4][8];
#pragma unroll
    for (int a2 = 0; a2 < 4; ++a2) {
#pragma unroll
        for (int a1 = 0; a1 < 8; ++a1) v[a2][a1] = u[4 * a1 + a2];
        small_dft<8>(v[a2]);
#pragma unroll
        for (int c1 = 1; c1 < 8; ++c1) v[a2][c1] = mul_w32(v[a2][c1], a2 * c1);
    }
#pragma unroll
    for (int c1 = 0; c1 < 8; ++c1) {
        float2 t0 = v[0][c1], t1 = v[1][c1], t2 = v[2][c1], t3 = v[3][c1];
        dft4(t0, t1, t2, t3);
        u[c1] = t0;
        u[c1 + 8] = t1;
        u[c1 + 16] = t2;
        u[c1 + 24] = t3;
    }
}

// The two signs of a code field pair as values: the 2-bit field at bits pr + 1 : pr (real
// part) and pr - 3 : pr - 4 (imaginary part) read as a signed integer, 01 -> 1, 11 -> -1,
// 00 -> 0.
__device__ __forceinline__ float2 code_pair(unsigned w, int pr)
{
    // the builtin's result is typed unsigned: the sign-extended field is read back as int
    const int re = (int)__builtin_amdgcn_sbfe(w, (unsigned)pr, 2u), im = (int)__builtin_amdgcn_sbfe(w, (unsigned)(pr - 4), 2u);
    return make_float2((float)re, (float)im);
}

// Inner phase sums of a whole group (kD5Group phases) for a thread's first NU bins,
// sum_j (W^p)^j Y_j[p mod 512] by Horner's rule from the last phase down: the NU chains side
// by side and unrolled, so the reads are issued ahead of the multiply-adds. A bin of the
// last NU past the window runs on a valid column and is dropped by the caller.
template <int NU>
__device__ __forceinline__ void group_horner(const float2 *X, const int (&bp)[4], const float2 (&bstep)[4],
                                             float2 (&hs)[4])
{
#pragma unroll
    for (int u = 0; u < NU; ++u) hs[u] = X[(kD5Group - 1) * kD5YS + (bp[u] & 511)];
#pragma unroll
    for (int jj = kD5Group - 2; jj >= 0; --jj) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const float2 yv = X[jj * kD5YS + (bp[u] & 511)], w = bstep[u];
            hs[u] = make_float2(fmaf(hs[u].x, w.x, fmaf(-hs[u].y, w.y, yv.x)),
                                fmaf(hs[u].x, w.y, fmaf(hs[u].y, w.x, yv.y)));
        }
    }
}

// Grid: x strides over the delays. Dynamic LDS: the two-level table of W_N.
template <int SRC>
__global__ __launch_bounds__(kD5Threads, 2) void dft512_kernel(Dft12bParams P, TsumParams T)
{
    static_assert(SRC == DFT_LAG || SRC == DFT_CODES, "lag products or their sign codes");
    __shared__ float2 X[kD5X];
    __shared__ float2 w512[512];
    extern __shared__ float2 tab[];
    float2 *coarse = tab, *fine = tab + P.n_coarse;
    const int tid = threadIdx.x;
    const int n = P.n, M = P.M;
    build_twiddle_tables(coarse, fine, n, P.tb, P.n_coarse, tid, kD5Threads);
    __syncthreads();
    for (int k = tid; k < 512; k += kD5Threads) w512[k] = table_twiddle(coarse, fine, k * M, P.tb); // k M < n
    __syncthreads();

    const int j = tid & 15, hb = tid >> 4; // pass 1: residue b = hb; pass 2: columns hb, hb + 16
    // buffer views of the signed inputs: s4[n], r4[2 n] (bounded: reads past them give 0)
    const __amdgpu_buffer_rsrc_t srs =
        __builtin_amdgcn_make_buffer_rsrc((void *)P.s4, (short)0, n * 16, 0x00020000);
    const __amdgpu_buffer_rsrc_t rrs =
        __builtin_amdgcn_make_buffer_rsrc((void *)P.r4, (short)0, 2 * n * 16, 0x00020000);
    // and of the sign codes (DFT_CODES)
    const __amdgpu_buffer_rsrc_t crs =
        __builtin_amdgcn_make_buffer_rsrc((void *)P.codes, (short)0, (int)P.code_bytes, 0x00020000);
    // this thread's bins: q = tid + 256 u
    int bq[4], bp[4], bjump[4];
    float2 bstep[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = tid + kD5Threads * u;
        bq[u] = q < P.n_dop ? q : -1;
        int p = P.p0n + (q < P.n_dop ? q : 0);
        p = p >= n ? p - n : p;
        bp[u] = p;
        bstep[u] = table_twiddle(coarse, fine, p, P.tb);
        bjump[u] = (int)(((long long)kD5Group * p) % n); // the group factor's step: W^{16 p}
    }
    // twiddle-sign planes: the row of each bin's base (bin p: base min(p, n - p)), and the
    // planes' stride
    // bins in use per thread (the same for the whole work-group)
    const int nu = min(4, (P.n_dop + kD5Threads - 1) / kD5Threads);
    int trow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) trow[u] = row_of_base(T.bm, bp[u] <= (n >> 1) ? bp[u] : n - bp[u]);
    const long long tplane = (long long)T.cols_pad * T.bases_pad;
    const bool tsum = SRC == DFT_CODES && T.part != nullptr;

    // DFT_LAG: rows in an XCD-aware order (work-groups are dealt to the 8 XCDs in turn; with
    // a grid that is a multiple of 8 the work-groups of one XCD take consecutive delays,
    // whose reference windows nearly coincide: measured 2% faster). DFT_CODES: rows in grid
    // order (each row's packed codes are contiguous; the XCD order measured 2% slower).
    const int G = (int)gridDim.x;
    const int v = SRC == DFT_LAG && (G & 7) == 0 ? (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3)
                                                 : (int)blockIdx.x;
    for (int l = v; l < P.n_tau; l += G) {
        const int d = P.tau0 + l;
        float2 acc[4];
        int bv[4]; // (m0 p) mod n of the current group
        // the twiddle-sign half of the bins: plane g is read during group g (its load in
        // flight through the group's transforms) and the planes are added in order
        float4 tacc[4], tv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc[u] = make_float2(0.0f, 0.0f);
            bv[u] = 0;
            tacc[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const float4 *trow_l = tsum ? T.part + (long long)l * T.bases_pad : nullptr;
        for (int m0 = 0; m0 < M; m0 += kD5Group) {
            const int mb = min(kD5Group, M - m0);
            const int tg = m0 / kD5Group; // the plane this group reads
            const bool tload = tsum && tg < T.ksplit;
            if (tload) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (bq[u] >= 0) tv[u] = trow_l[tg * tplane + trow[u]];
            }
            // ---- pass 1: the 32 samples a of transform j, residue hb; 32-point DFT; W_512^{b c} ----
            // lanes past the group's last phase (a short last group) repeat that phase's
            // loads: their transforms are never read
            const int jl = min(j, mb - 1);
            float2 x[32];
            if constexpr (SRC == DFT_CODES) {
                // sample idx = base + 16 M a is field idx mod 8 of packed word idx / 8 of row
                // l: the field stays put for all a (16 M a is a multiple of 8) and the word
                // steps by 2 M, which goes in the scalar offset
                const int base = m0 + jl + M * hb;
                const unsigned vo = ((unsigned)l * (unsigned)P.code_wpc + (unsigned)(base >> 3)) * 4u;
                const unsigned step = 8u * (unsigned)M;
                const int e = base & 7;
                const int pr = ((e & 1) ? 30 : 14) - 2 * ((e >> 1) & 1) - ((e & 4) ? 0 : 8);
#pragma unroll
                for (int a = 0; a < 32; ++a) {
                    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(crs, vo, step * (unsigned)a, 0);
                    x[a] = code_pair(w, pr);
                }
            } else {
                // sample idx = m0 + j + M (16 a + hb): one vector offset per lane, the step
                // of a (16 M samples) in the scalar offset of each load
                const unsigned vs = (unsigned)(m0 + jl + M * hb) * 16u;
                const unsigned vr = (unsigned)(n + m0 + jl + M * hb - d) * 16u;
                const unsigned step = 256u * (unsigned)M;
#pragma unroll
                for (int a = 0; a < 32; ++a) {
                    const float4 sv = __builtin_bit_cast(
                        float4, __builtin_amdgcn_raw_buffer_load_b128(srs, vs, step * (unsigned)a, 0));
                    const float4 rv = __builtin_bit_cast(
                        float4, __builtin_amdgcn_raw_buffer_load_b128(rrs, vr, step * (unsigned)a, 0));
                    x[a] = lag_value_signed(sv, rv);
                }
            }
            reg_dft32(x);
#pragma unroll
            for (int c = 1; c < 32; ++c) x[c] = cmulf(x[c], w512[hb * c]); // hb c < 512
            __syncthreads(); // the previous group's bin reads are done
#pragma unroll
            for (int c = 0; c < 32; ++c) X[(c * 16 + hb) * 17 + j] = x[c];
            __syncthreads();
            // ---- pass 2: 16-point DFTs over b for columns hb and hb + 16 ----
            float2 y[2][16];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < 16; ++b) y[h][b] = X[((hb + 16 * h) * 16 + b) * 17 + j];
            __syncthreads(); // the pass-1 buffer is read; it becomes the pass-2 buffer
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                reg_dft16(y[h]);
#pragma unroll
                for (int e = 0; e < 16; ++e) X[j * kD5YS + hb + 16 * h + 32 * e] = y[h][e];
            }
            __syncthreads();
            // ---- bins: sum_j W^{(m0 + j) p} Y_j[p mod 512] = W^{m0 p} sum_j (W^p)^j Y_j, the
            // inner sum by Horner's rule from the group's last phase down ----
            float2 hs[4] = {};
            if (mb == kD5Group) {
                if (nu == 1)
                    group_horner<1>(X, bp, bstep, hs);
                else if (nu == 2)
                    group_horner<2>(X, bp, bstep, hs);
                else if (nu == 3)
                    group_horner<3>(X, bp, bstep, hs);
                else
                    group_horner<4>(X, bp, bstep, hs);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= nu) break;
                    const int k = bp[u] & 511;
                    const float2 w = bstep[u];
                    float2 h = X[(mb - 1) * kD5YS + k];
                    for (int jj = mb - 2; jj >= 0; --jj) {
                        const float2 yv = X[jj * kD5YS + k];
                        h = make_float2(fmaf(h.x, w.x, fmaf(-h.y, w.y, yv.x)), fmaf(h.x, w.y, fmaf(h.y, w.x, yv.y)));
                    }
                    hs[u] = h;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u >= nu) break;
                const float2 g = table_twiddle(coarse, fine, bv[u], P.tb), h = hs[u];
                acc[u] = make_float2(fmaf(g.x, h.x, fmaf(-g.y, h.y, acc[u].x)), fmaf(g.x, h.y, fmaf(g.y, h.x, acc[u].y)));
                bv[u] += bjump[u]; // both below n
                bv[u] = bv[u] >= n ? bv[u] - n : bv[u];
            }
            if (tload) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (bq[u] >= 0) {
                        tacc[u].x += tv[u].x;
                        tacc[u].y += tv[u].y;
                        tacc[u].z += tv[u].z;
                        tacc[u].w += tv[u].w;
                    }
            }
        }
        float2 *dst = P.out + (size_t)l * P.n_dop;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (bq[u] < 0) continue;
            float2 a = acc[u];
            if (SRC == DFT_CODES && bp[u] == 0) a = make_float2(0.0f, 0.0f);
            if (tsum) {
                // planes past the row's groups, then the +b (p <= n / 2) or -b assembly
                float4 t = tacc[u];
                for (int k = (M + kD5Group - 1) / kD5Group; k < T.ksplit; ++k) {
                    const float4 v = trow_l[k * tplane + trow[u]];
                    t.x += v.x;
                    t.y += v.y;
                    t.z += v.z;
                    t.w += v.w;
                }
                a = caddf(a, bp[u] <= (n >> 1) ? make_float2(t.x - t.y, t.z + t.w)
                                                : make_float2(t.x + t.y, t.z - t.w));
            } else if (P.accumulate) {
                a = caddf(a, dst[bq[u]]);
            }
            dst[bq[u]] = a;
        }
    }
}

} // namespace ndft
