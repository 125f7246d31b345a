// Layout of a batched workspace (many CPIs, one persistent launch), shared by the host
// planner (ndft_caf_batched_prepare) and the device planner (ndft_caf_batched_dev, whose
// CPI descriptors live in device memory).
//
// Workspace: [256 B header][ContractParams x n_cpi][ReduceParams x n_cpi][out offsets x
// n_cpi][PrepDesc x 2 n_cpi][FP8 data maxima, 2 words x n_cpi][work items][per CPI: signed
// surveillance, signed reference, split-K partial sums], every region 256-byte aligned.
// A surface is split into (base tile, delay tile, sample chunk) work items; a chunk is
// `chunk` samples (a multiple of the plan's stage), the last one of a CPI ragged.
#pragma once

#include "ndft.h"
#include "ndft_contract.hpp"

namespace ndft {

__host__ __device__ inline long long bdiv(long long a, long long b) { return (a + b - 1) / b; }
__host__ __device__ inline size_t balign(size_t b) { return (b + 255) / 256 * 256; }
__host__ __device__ inline long long bmod(long long a, long long n)
{
    const long long r = a % n;
    return r < 0 ? r + n : r;
}

// Base bins: every requested bin p in {p0 + q mod n} is served by base min(p, n - p); the
// set of bases is a union of at most four ascending runs.
__host__ __device__ inline BaseMap base_map(long long n, long long p0, long long n_bins, int *total)
{
    const long long a = bmod(p0, n);
    long long px[2], py[2];
    int np = 0;
    if (a + n_bins <= n) {
        px[np] = a;
        py[np++] = a + n_bins;
    } else {
        px[np] = a;
        py[np++] = n;
        px[np] = 0;
        py[np++] = a + n_bins - n;
    }
    const long long h = n / 2; // bins [0, h] are their own base; bins (h, n) map to n - p
    long long ix[4], iy[4];
    int ni = 0;
    for (int k = 0; k < np; ++k) {
        const long long x = px[k], y = py[k];
        if (x < h + 1) {
            ix[ni] = x;
            iy[ni++] = y < h + 1 ? y : h + 1;
        }
        if (y > h + 1) {
            const long long xx = x > h + 1 ? x : h + 1;
            ix[ni] = n - y + 1;
            iy[ni++] = n - xx + 1;
        }
    }
    // sort the (at most four) intervals by start, then merge
    for (int k = 1; k < ni; ++k)
        for (int m = k; m > 0 && (ix[m] < ix[m - 1] || (ix[m] == ix[m - 1] && iy[m] < iy[m - 1])); --m) {
            const long long tx = ix[m], ty = iy[m];
            ix[m] = ix[m - 1];
            iy[m] = iy[m - 1];
            ix[m - 1] = tx;
            iy[m - 1] = ty;
        }
    long long mx[4], my[4];
    int nm = 0;
    for (int k = 0; k < ni; ++k) {
        if (ix[k] >= iy[k]) continue;
        if (nm > 0 && ix[k] <= my[nm - 1]) {
            if (iy[k] > my[nm - 1]) my[nm - 1] = iy[k];
        } else {
            mx[nm] = ix[k];
            my[nm++] = iy[k];
        }
    }
    BaseMap bm;
    bm.nseg = nm;
    int off = 0;
    for (int k = 0; k < 4; ++k) {
        bm.start[k] = k < nm ? (int)mx[k] : 0;
        bm.off[k] = off;
        if (k < nm) off += (int)(my[k] - mx[k]);
    }
    bm.off[4] = off;
    *total = off;
    return bm;
}

// Two-level table for length n within max_bytes of LDS: fine size 2^tb >= sqrt(n) by
// default. The exact form needs every quadrant point m in {n/4, n/2, 3n/4} that is an
// integer to have m mod 2^tb = 0 (2^tb divides n/4, resp. n/2 for n = 2 mod 4; any tb
// for odd n) and n <= 2^20; tb is lowered to get it when the coarse table still fits.
__host__ __device__ inline void table_choice(long long n, int max_bytes, int *tb_out, int *n_coarse_out,
                                             int *exact_out)
{
    int tb = 0;
    while ((1LL << (2 * tb)) < n) ++tb;
    int exact = 0;
    if (n <= (1 << 20)) {
        int v = 0;
        while (((n >> v) & 1) == 0) ++v;
        const int cap = n % 4 == 0 ? v - 2 : (n % 2 == 0 ? v - 1 : 62);
        const int t = tb < cap ? tb : cap;
        if ((bdiv(n, 1LL << t) + (1LL << t)) * (long long)sizeof(float2) <= max_bytes) {
            tb = t;
            exact = 1;
        }
    }
    *tb_out = tb;
    *n_coarse_out = (int)bdiv(n, 1LL << tb);
    *exact_out = exact;
}

// What the layout needs from the tile plan.
struct BatchPlanGeom {
    int bt, lt;      // bases and delays per tile
    int max_dynamic; // LDS left for the twiddle table
    float sign_scale;
    int fp8;         // data maxima for the e4m3 data exponent
};

constexpr int kMaxBatch = 16384;
constexpr int kDefaultChunk = 4096;

__host__ __device__ inline bool cpi_valid(const ndft_cpi &c)
{
    return c.n >= 1 && c.n <= NDFT_MAX_N && c.tau0 >= 0 && c.n_tau >= 1 && c.tau0 + c.n_tau <= c.n &&
           c.n_dop >= 1 && c.n_dop <= c.n && c.surv_off >= 0 && c.ref_off >= 0 && c.out_off >= 0;
}

// One CPI's tables and buffer sizes at a given chunk; false when the CPI is invalid or its
// twiddle table does not fit the plan's LDS.
struct CpiLayout {
    ContractParams C; // pointers left null
    ReduceParams R;   // partial / out left null
    int table_bytes;
    long long items, full_items; // work items, those with a whole chunk
    size_t s4_bytes, r4_bytes, part_bytes;
};

__host__ __device__ inline bool cpi_layout(const ndft_cpi &d, const BatchPlanGeom &g, int chunk, CpiLayout &o)
{
    if (!cpi_valid(d)) return false;
    ContractParams &C = o.C;
    ReduceParams &R = o.R;
    C = ContractParams{};
    R = ReduceParams{};
    int nb;
    C.bm = base_map(d.n, d.p0, d.n_dop, &nb);
    C.n = (int)d.n;
    C.n_cols = (int)d.n_tau;
    C.tau0 = (int)d.tau0;
    C.n_bases = nb;
    table_choice(d.n, g.max_dynamic, &C.tb, &C.n_coarse, &C.tw_exact);
    o.table_bytes = (int)((C.n_coarse + (1 << C.tb)) * sizeof(float2));
    if (o.table_bytes > g.max_dynamic) return false;
    C.kchunk = chunk;
    C.ksplit = (int)bdiv(d.n, chunk);
    C.tiles_b = (int)bdiv(nb, g.bt);
    C.tiles_l = (int)bdiv(d.n_tau, g.lt);
    C.n_bases_pad = C.tiles_b * g.bt;
    C.n_cols_pad = C.tiles_l * g.lt;
    C.s_raw_off = d.surv_off;
    C.r_raw_off = d.ref_off;
    R.ksplit = C.ksplit;
    R.n_cols_pad = C.n_cols_pad;
    R.n_bases_pad = C.n_bases_pad;
    R.n_cols = C.n_cols;
    R.n_bases = nb;
    R.bm = C.bm;
    R.n = C.n;
    R.p0n = (int)bmod(d.p0, d.n);
    R.n_bins = (int)d.n_dop;
    const long long tiles = (long long)C.tiles_b * C.tiles_l;
    o.items = tiles * C.ksplit;
    o.full_items = tiles * (d.n / chunk);
    o.s4_bytes = balign(sizeof(float4) * (size_t)(d.n + kTailPad));
    o.r4_bytes = balign(sizeof(float4) * (size_t)(2 * d.n + kTailPad));
    o.part_bytes = balign(sizeof(float4) * (size_t)C.ksplit * C.n_cols_pad * C.n_bases_pad);
    return true;
}

// Offsets of the fixed regions (they depend on n_cpi only).
struct BatchRegions {
    size_t params, red, outoff, prep, absmax, items;
};

__host__ __device__ inline BatchRegions batch_regions(int n_cpi)
{
    BatchRegions r;
    size_t off = 256; // header
    r.params = off;
    off = balign(off + sizeof(ContractParams) * n_cpi);
    r.red = off;
    off = balign(off + sizeof(ReduceParams) * n_cpi);
    r.outoff = off;
    off = balign(off + sizeof(long long) * n_cpi);
    r.prep = off;
    off = balign(off + sizeof(PrepDesc) * 2 * n_cpi);
    r.absmax = off;
    off = balign(off + sizeof(unsigned) * 2 * n_cpi);
    r.items = off;
    return r;
}

// Device planner of ndft_caf_batched_dev: one work-group of kPlanThreads reads the CPI
// descriptors from device memory, lays out the workspace exactly as the host planner does
// for the same chunk (doubling the chunk while the partial sums do not fit ws_bytes), and
// writes every table the batched kernels read. Work items go whole chunks first, then the
// ragged last chunks, each part in CPI order. An invalid descriptor, a table that does
// not fit or a workspace that is too small even with one chunk per surface leaves the tag
// at 0 and the status at NDFT_E_INVAL / NDFT_E_WORKSPACE: the kernels that follow do
// nothing then.
constexpr int kPlanThreads = 1024;
constexpr int kMaxDevBatch = 4096; // CPIs of one device-planned batch (LDS prefix sums)

struct DevPlanArgs {
    const ndft_cpi *cpis;
    int n_cpi;
    BatchPlanGeom g;
    int chunk;         // starting chunk (a multiple of the plan's stage)
    int kgran;         // the plan's stage
    char *ws;
    size_t ws_bytes;
    unsigned long long tag;
    int plan_id;
};

__device__ inline void block_exclusive_scan(unsigned long long *v, int count, unsigned long long *total,
                                            unsigned long long *tmp)
{
    // per-thread contiguous ranges, then a scan of the thread sums (kPlanThreads entries)
    const int tid = threadIdx.x;
    const int per = (count + kPlanThreads - 1) / kPlanThreads;
    const int lo = min(count, tid * per), hi = min(count, lo + per);
    unsigned long long s = 0;
    for (int k = lo; k < hi; ++k) s += v[k];
    tmp[tid] = s;
    __syncthreads();
    if (tid == 0) {
        unsigned long long run = 0;
        for (int k = 0; k < kPlanThreads; ++k) {
            const unsigned long long t = tmp[k];
            tmp[k] = run;
            run += t;
        }
        *total = run;
    }
    __syncthreads();
    unsigned long long run = tmp[tid];
    for (int k = lo; k < hi; ++k) {
        const unsigned long long t = v[k];
        v[k] = run;
        run += t;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(DevPlanArgs A)
{
    __shared__ unsigned long long s_bytes[kMaxDevBatch]; // per CPI buffer bytes -> offsets
    __shared__ unsigned long long s_full[kMaxDevBatch];  // whole-chunk items -> first index
    __shared__ unsigned long long s_tail[kMaxDevBatch];  // ragged items -> first index
    __shared__ unsigned long long s_tmp[kPlanThreads];
    __shared__ unsigned long long s_tot[3];
    __shared__ int s_bad;
    const int tid = threadIdx.x, n_cpi = A.n_cpi;
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(A.ws);
    const BatchRegions rg = batch_regions(n_cpi);
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int chunk = A.chunk;
    bool fits = false;
    for (int attempt = 0; attempt < 32 && !fits; ++attempt) {
        long long max_n = 1;
        for (int c = tid; c < n_cpi; c += kPlanThreads) {
            const ndft_cpi d = A.cpis[c];
            CpiLayout o;
            if (!cpi_layout(d, A.g, chunk, o)) {
                s_bad = NDFT_E_INVAL;
                s_bytes[c] = s_full[c] = s_tail[c] = 0;
                continue;
            }
            s_bytes[c] = o.s4_bytes + o.r4_bytes + o.part_bytes;
            s_full[c] = o.full_items;
            s_tail[c] = o.items - o.full_items;
            max_n = d.n > max_n ? d.n : max_n;
        }
        __syncthreads();
        if (s_bad) break;
        block_exclusive_scan(s_bytes, n_cpi, &s_tot[0], s_tmp);
        block_exclusive_scan(s_full, n_cpi, &s_tot[1], s_tmp);
        block_exclusive_scan(s_tail, n_cpi, &s_tot[2], s_tmp);
        const unsigned long long n_items = s_tot[1] + s_tot[2];
        const size_t bufs = balign(rg.items + sizeof(int4) * (size_t)n_items);
        fits = n_items < (1ULL << 30) && bufs + s_tot[0] <= A.ws_bytes;
        // the largest n of the batch bounds the useful chunk
        s_tmp[tid] = (unsigned long long)max_n;
        __syncthreads();
        for (int st = kPlanThreads / 2; st > 0; st >>= 1) {
            if (tid < st && s_tmp[tid + st] > s_tmp[tid]) s_tmp[tid] = s_tmp[tid + st];
            __syncthreads();
        }
        const long long big = (long long)s_tmp[0];
        __syncthreads();
        if (!fits) {
            if (chunk >= big) break; // one chunk per surface already
            chunk *= 2;
        }
    }
    if (s_bad || !fits) {
        if (tid == 0) {
            hdr->tag = 0ULL;
            hdr->status = s_bad ? s_bad : (int)NDFT_E_WORKSPACE;
            hdr->n_items = 0;
            hdr->counter = 0;
        }
        return;
    }
    const size_t bufs = balign(rg.items + sizeof(int4) * (size_t)(s_tot[1] + s_tot[2]));
    ContractParams *params = reinterpret_cast<ContractParams *>(A.ws + rg.params);
    ReduceParams *red = reinterpret_cast<ReduceParams *>(A.ws + rg.red);
    long long *outoff = reinterpret_cast<long long *>(A.ws + rg.outoff);
    PrepDesc *prep = reinterpret_cast<PrepDesc *>(A.ws + rg.prep);
    unsigned *absmax = reinterpret_cast<unsigned *>(A.ws + rg.absmax);
    int4 *items = reinterpret_cast<int4 *>(A.ws + rg.items);
    const unsigned long long full_total = s_tot[1];
    for (int c = tid; c < n_cpi; c += kPlanThreads) {
        const ndft_cpi d = A.cpis[c];
        CpiLayout o;
        cpi_layout(d, A.g, chunk, o);
        char *base = A.ws + bufs + s_bytes[c];
        float4 *s4 = reinterpret_cast<float4 *>(base);
        float4 *r4 = reinterpret_cast<float4 *>(base + o.s4_bytes);
        float4 *part = reinterpret_cast<float4 *>(base + o.s4_bytes + o.r4_bytes);
        o.C.s4 = s4;
        o.C.r4 = r4;
        o.C.partial = part;
        o.C.absmax = A.g.fp8 ? absmax + 2 * c : nullptr;
        o.R.partial = part;
        params[c] = o.C;
        red[c] = o.R;
        outoff[c] = d.out_off;
        prep[2 * c] = PrepDesc{d.surv_off, s4, (int)d.n, 0, (long long)(d.n + kTailPad), A.g.sign_scale,
                               A.g.fp8 ? absmax + 2 * c : nullptr};
        prep[2 * c + 1] = PrepDesc{d.ref_off, r4, (int)d.n, (int)d.n, (long long)(2 * d.n + kTailPad),
                                   A.g.sign_scale, A.g.fp8 ? absmax + 2 * c + 1 : nullptr};
        // items: (cpi, tile_b, tile_l, chunk); whole chunks first, then the ragged one
        const int whole = (int)(d.n / chunk);
        unsigned long long fi = s_full[c], ti = full_total + s_tail[c];
        for (int tl = 0; tl < o.C.tiles_l; ++tl)
            for (int tbi = 0; tbi < o.C.tiles_b; ++tbi)
                for (int kc = 0; kc < o.C.ksplit; ++kc) {
                    const int4 w = make_int4(c, tbi, tl, kc);
                    if (kc < whole)
                        items[fi++] = w;
                    else
                        items[ti++] = w;
                }
    }
    __syncthreads();
    if (tid == 0) {
        hdr->counter = 0;
        hdr->n_items = (int)(s_tot[1] + s_tot[2]);
        hdr->n_cpi = n_cpi;
        hdr->plan_id = A.plan_id;
        hdr->status = 0;
        __threadfence();
        hdr->tag = A.tag;
    }
}

// Copies the planner's status word (0 when the batch ran) to a caller int32.
__global__ void batch_status_kernel(const BatchHeader *hdr, int *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = hdr->status;
}

} // namespace ndft
