// libndft.so: C ABI of the NDFT hot path (declarations and conventions in include/ndft.h).
// Host side: argument validation, base-bin segments, tile plans, workspace layout,
// kernel launches on the caller's stream and optional hipEvent timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <chrono>
#include <map>
#include <utility>
#include <vector>

#include "ndft.h"
#include "ndft_backward.hpp"
#include "ndft_batch.hpp"
#include "ndft_contract.hpp"
#include "ndft_debug.hpp"
#include "ndft_dft12b.hpp"
#include "ndft_dft512.hpp"
#include "ndft_fast.hpp"
#include "ndft_nfft.hpp"
#include "ndft_signsplit.hpp"
#include "ndft_surface_bf16.hpp"

using namespace ndft;

namespace {

// ------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------
inline int64_t mod_n(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// Base bins: every requested bin p in {p0 + q mod n} is served by base min(p, n - p);
// the set of bases is a union of at most four ascending runs.
BaseMap make_base_map(int64_t n, int64_t p0, int64_t n_bins, int *total)
{
    int64_t a = mod_n(p0, n);
    std::vector<std::pair<int64_t, int64_t>> pieces;
    if (a + n_bins <= n) {
        pieces.push_back({a, a + n_bins});
    } else {
        pieces.push_back({a, n});
        pieces.push_back({0, a + n_bins - n});
    }
    const int64_t h = n / 2; // bins [0, h] are their own base; bins (h, n) map to n - p
    std::vector<std::pair<int64_t, int64_t>> iv;
    for (auto &pc : pieces) {
        int64_t x = pc.first, y = pc.second;
        if (x < h + 1) iv.push_back({x, std::min(y, h + 1)});
        if (y > h + 1) {
            int64_t xx = std::max(x, h + 1);
            iv.push_back({n - y + 1, n - xx + 1});
        }
    }
    std::sort(iv.begin(), iv.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (auto &v : iv) {
        if (v.first >= v.second) continue;
        if (!merged.empty() && v.first <= merged.back().second)
            merged.back().second = std::max(merged.back().second, v.second);
        else
            merged.push_back(v);
    }
    BaseMap bm;
    std::memset(&bm, 0, sizeof(bm));
    bm.nseg = (int)merged.size();
    int off = 0;
    for (int k = 0; k < bm.nseg; ++k) {
        bm.start[k] = (int)merged[k].first;
        bm.off[k] = off;
        off += (int)(merged[k].second - merged[k].first);
    }
    for (int k = bm.nseg; k < 5; ++k) bm.off[k] = off;
    *total = off;
    return bm;
}

// ------------------------------------------------------------------------------------
// tile plans
// ------------------------------------------------------------------------------------
struct Plan {
    const char *name;
    int bt, lt, ks, nt;
    int kgran;               // sample chunks are multiples of this
    int static_lds;
    const void *kfn[2];      // [PROD_LAG, PROD_IDENTITY]; nullptr: no such form
    const void *kfn_batched; // persistent lag-product kernel
    double cost_scale;       // relative cost per padded cell in the built-in choice
    double row_cost_cols;    // per padded base row, in cells (the plane builder's pass)
    float sign_scale;        // scale of the input signs the kernels read (1 or 1/2)
    const void *planes_kfn;  // twiddle plane builder (nullptr: twiddles made in the kernel)
    bool raw_inputs;         // reads complex64 inputs itself (no sign-prep launches)
    const void *lag_kfn;     // sign-split plans: the lag / twiddle-sign kernel (lsum_kernel)
    const void *lag_kfn_lin; // the same for the Eq. (12c) surface (ordinary lag product)
    int stage_a;             // plane uint4 per stage (plane plans)
    bool fft_d;              // sign-split with the twiddle half as a decimated FFT (no matrix kernel)
    bool fastx = false;      // the fast exact transform (every bin; N a power of two, ndft_fast.hpp)
};

template <int PREC, int WAVES_B, int WAVES_L, int WB, int WL, int KS>
Plan make_plan(const char *name)
{
    using Cfg = ContractCfg<PREC, PROD_LAG, WAVES_B, WAVES_L, WB, WL, KS>;
    Plan p;
    p.name = name;
    p.bt = Cfg::BT;
    p.lt = Cfg::LT;
    p.ks = KS;
    p.nt = Cfg::NT;
    p.kgran = KS;
    p.static_lds = 2 * (Cfg::STAGE_A_F4 + Cfg::STAGE_B_F4) * 16;
    p.kfn[0] = reinterpret_cast<const void *>(&contract_kernel<PREC, PROD_LAG, WAVES_B, WAVES_L, WB, WL, KS>);
    p.kfn[1] = reinterpret_cast<const void *>(&contract_kernel<PREC, PROD_IDENTITY, WAVES_B, WAVES_L, WB, WL, KS>);
    p.kfn_batched =
        reinterpret_cast<const void *>(&contract_batched_kernel<PREC, PROD_LAG, WAVES_B, WAVES_L, WB, WL, KS>);
    p.cost_scale = 1.0 + 64.0 / Cfg::BT + 64.0 / Cfg::LT;
    p.row_cost_cols = 0.0;
    p.sign_scale = 1.0f;
    p.planes_kfn = nullptr;
    p.raw_inputs = false;
    p.lag_kfn = nullptr;
    p.lag_kfn_lin = nullptr;
    p.fft_d = false;
    p.stage_a = 0;
    return p;
}

// Split-BF16 surface plans with register-built lag operands (lag products only); with
// PLANES the twiddle operand is precomputed into the workspace by a builder kernel.
template <int NW, int WB, int WL, int KS, int PF, bool PLANES = false>
Plan make_surface_plan(const char *name)
{
    using Cfg = SurfCfg<NW, WB, WL, KS, PF>;
    Plan p;
    p.name = name;
    p.bt = Cfg::BT;
    p.lt = Cfg::LT;
    p.ks = KS;
    p.nt = Cfg::NT;
    p.kgran = 2 * KS;
    p.static_lds = 2 * Cfg::STAGE_A * 16 + 2 * Cfg::WIN * 16 + 16;
    p.kfn[0] = PLANES ? reinterpret_cast<const void *>(&surface_bf16_planes_kernel<NW, WB, WL, KS, PF>)
                      : reinterpret_cast<const void *>(&surface_bf16_kernel<NW, WB, WL, KS, PF>);
    p.kfn[1] = nullptr;
    p.kfn_batched =
        PLANES ? nullptr : reinterpret_cast<const void *>(&surface_bf16_batched_kernel<NW, WB, WL, KS, PF>);
    // lag operands are built once per base tile; twiddles once per delay tile (6% more
    // per cell, measured) or once into planes (a builder pass worth ~100 delay columns)
    p.cost_scale = 0.25 * (1.0 + 24.0 / Cfg::BT) * (PLANES ? 1.0 : 1.06);
    p.row_cost_cols = PLANES ? 100.0 : 0.0;
    p.sign_scale = 0.5f;
    p.planes_kfn = PLANES ? reinterpret_cast<const void *>(&plane_build_kernel<Cfg::BT, KS>) : nullptr;
    p.raw_inputs = true;
    p.lag_kfn = nullptr;
    p.lag_kfn_lin = nullptr;
    p.fft_d = false;
    p.stage_a = Cfg::STAGE_A;
    return p;
}

// Sign-split split-BF16 plans: lsum_kernel (twiddle-sign part, lag sign codes, base 0) and
// dsum_kernel (twiddles against the lag signs), its twiddle operands from planes or (GEN)
// made in the kernel.
template <int NW, int WB, int KS, bool GEN>
Plan make_split_plan(const char *name, double rel_cost)
{
    using Cfg = DsumCfg<NW, WB, KS>;
    Plan p;
    p.name = name;
    p.bt = Cfg::BT;
    p.lt = Cfg::LT;
    p.ks = KS;
    p.nt = Cfg::NT;
    p.kgran = 2 * KS;
    p.static_lds = 2 * Cfg::STAGE_A * 16;
    p.kfn[0] = reinterpret_cast<const void *>(&dsum_kernel<NW, WB, KS, GEN>);
    p.kfn[1] = nullptr;
    p.kfn_batched = nullptr;
    // half the matrix work of the combined form; the twiddle-sign part costs in proportion
    // to the sign runs (see split_cost)
    // half the matrix work of the combined form, times the plan's measured cost per padded
    // cell relative to the best (whole call, N = 65536 surface: work-groups per compute
    // unit and waves per SIMD differ between the tile shapes)
    p.cost_scale = 0.25 * 0.5 * rel_cost;
    p.row_cost_cols = GEN ? 0.0 : 50.0;
    p.sign_scale = 0.5f;
    p.planes_kfn = GEN ? nullptr : reinterpret_cast<const void *>(&dplane_build_kernel<Cfg::BT, KS>);
    p.raw_inputs = true;
    p.lag_kfn = reinterpret_cast<const void *>(&lsum_kernel<false, false>);
    p.lag_kfn_lin = reinterpret_cast<const void *>(&lsum_kernel<true, false>);
    p.fft_d = false;
    p.stage_a = Cfg::STAGE_A;
    return p;
}

// FP32 form of the sign-split plans: lsum_kernel for the twiddle-sign half (and base 0), and
// the twiddle half D = sum_k W^{pk} csgn(z_k), an ordinary DFT of the exact lag signs, by the
// decimated FFT kernel of the Eq. (12b) surface (dft12b_kernel<., true>), in FP32.
Plan make_fftd_plan(const char *name)
{
    Plan p = make_split_plan<8, 2, 128, true>(name, 1.0);
    p.kfn[0] = nullptr;
    p.fft_d = true; // lag_kfn_lin kept: the Eq. (12c) surface in FP32 the same way
    // the sign codes in the packed layout the FFT kernel reads (half the bytes)
    p.lag_kfn = reinterpret_cast<const void *>(&lsum_kernel<false, true>);
    p.lag_kfn_lin = reinterpret_cast<const void *>(&lsum_kernel<true, true>);
    p.cost_scale = 0.05; // far below the FP32 contraction wherever it is eligible
    return p;
}

// FP8 form of the sign-split plans: the same lsum_kernel, dsum8_kernel with four-term e4m3
// twiddle planes against exact e4m3 lag signs.
template <int NW, int WB, int KS>
Plan make_split8_plan(const char *name, double rel_cost)
{
    Plan p = make_split_plan<NW, WB, KS, false>(name, rel_cost);
    p.kfn[0] = reinterpret_cast<const void *>(&dsum8_kernel<NW, WB, KS>);
    p.planes_kfn = reinterpret_cast<const void *>(&dplane8_build_kernel<DsumCfg<NW, WB, KS>::BT, KS>);
    return p;
}

// FP32 fast exact transform (ndft_fast.hpp): every bin of a row from FFTs and cyclic
// correlations over the odd residues, N a power of two in [kFastMinN, kFastMaxN]; no matrix
// kernel. In the built-in choice its cost is a per-row count independent of the window.
Plan make_fast_plan(const char *name)
{
    Plan p;
    std::memset(&p, 0, sizeof(p));
    p.name = name;
    p.bt = 1;
    p.lt = 1;
    p.ks = 1;
    p.nt = kFastThreads;
    p.kgran = 1;
    p.cost_scale = 1.0;
    p.sign_scale = 1.0f;
    p.fastx = true;
    return p;
}

bool fast_ok(int64_t n) { return n >= kFastMinN && n <= kFastMaxN && (n & (n - 1)) == 0; }

// Built-in cost of the fast transform per row, in the contraction's units (padded cell x
// cost_scale): ~2 log2(N)^2 cells (its work is O(N log N) a row against O(N) a cell, and
// its ~log2(N)^2 barrier-separated steps bound it at these lengths).
double fast_row_cost(int64_t n)
{
    int lg = 0;
    while ((1LL << lg) < n) ++lg;
    return 2.0 * lg * lg;
}

const std::vector<Plan> &plans(int prec)
{
    // name: bases x delays per work-group, waves, samples per stage
    static const std::vector<Plan> f32 = {
        make_plan<PREC_FP32, 2, 4, 2, 1, 8>("fp32_b128_l128_w8_ks8"),
        make_plan<PREC_FP32, 1, 8, 2, 1, 8>("fp32_b64_l256_w8_ks8"),
        make_plan<PREC_FP32, 4, 2, 2, 1, 8>("fp32_b256_l64_w8_ks8"),
        make_plan<PREC_FP32, 3, 4, 1, 1, 8>("fp32_b96_l128_w12_ks8"),
        make_fftd_plan("fp32s_fftd_b64_l256"),
        make_fast_plan("fp32x_fast_exact"),
    };
    static const std::vector<Plan> fp8 = {
        make_plan<PREC_FP8, 2, 4, 2, 1, 16>("fp8_b128_l128_w8_ks16"),
        make_plan<PREC_FP8, 3, 4, 1, 1, 16>("fp8_b96_l128_w12_ks16"),
        make_split8_plan<8, 2, 128>("fp8s_b64_l256_w8_ks128", 0.85),
    };
    static const std::vector<Plan> bf16 = {
        make_plan<PREC_BF16X2, 2, 4, 2, 1, 8>("bf16x2_b128_l128_w8_ks8"),
        make_plan<PREC_BF16X2, 1, 8, 2, 1, 8>("bf16x2_b64_l256_w8_ks8"),
        make_plan<PREC_BF16X2, 4, 2, 2, 1, 8>("bf16x2_b256_l64_w8_ks8"),
        make_plan<PREC_BF16X2, 3, 4, 1, 1, 8>("bf16x2_b96_l128_w12_ks8"),
        make_surface_plan<4, 3, 1, 32, 4>("bf16x2r_b96_l128_w4_ks32"),
        make_surface_plan<4, 3, 1, 16, 4>("bf16x2r_b96_l128_w4_ks16"),
        make_surface_plan<4, 4, 1, 16, 4>("bf16x2r_b128_l128_w4_ks16"),
        make_surface_plan<4, 3, 1, 16, 4, true>("bf16x2p_b96_l128_w4_ks16"),
        make_surface_plan<4, 3, 1, 32, 4, true>("bf16x2p_b96_l128_w4_ks32"),
        make_surface_plan<4, 4, 1, 16, 4, true>("bf16x2p_b128_l128_w4_ks16"),
        make_split_plan<4, 4, 32, false>("bf16x2s_b128_l128_w4_ks32", 1.12),
        make_split_plan<4, 3, 32, false>("bf16x2s_b96_l128_w4_ks32", 1.07),
        make_split_plan<8, 2, 32, false>("bf16x2s_b64_l256_w8_ks32", 1.10),
        make_split_plan<8, 3, 32, false>("bf16x2s_b96_l256_w8_ks32", 1.10),
        make_split_plan<8, 2, 32, true>("bf16x2g_b64_l256_w8_ks32", 1.09),
        make_split_plan<4, 4, 32, true>("bf16x2g_b128_l128_w4_ks32", 1.11),
        make_split_plan<8, 3, 32, true>("bf16x2g_b96_l256_w8_ks32", 1.03),
        make_split_plan<4, 2, 32, true>("bf16x2g_b64_l128_w4_ks32", 1.0),
        make_split_plan<4, 2, 32, false>("bf16x2s_b64_l128_w4_ks32", 0.95),
        make_split_plan<4, 2, 64, false>("bf16x2s_b64_l128_w4_ks64", 0.96),
        make_split_plan<8, 2, 64, false>("bf16x2s_b64_l256_w8_ks64", 0.97),
        make_split_plan<8, 2, 128, false>("bf16x2s_b64_l256_w8_ks128", 0.85),
        make_split_plan<8, 2, 128, true>("bf16x2g_b64_l256_w8_ks128", 0.8),
    };
    return prec == NDFT_FP8 ? fp8 : (prec == NDFT_BF16X2 ? bf16 : f32);
}

std::mutex g_plan_mu;
int g_plan_override[3] = {-1, -1, -1};
int g_ksplit_override[3] = {0, 0, 0};

// Largest twiddle-table size (N = 2^24: 4096 coarse + 4096 fine entries).
constexpr int kMaxTableBytes = 8192 * 8;
// LDS per work-group on gfx950.
constexpr int kLdsBytes = 160 * 1024;

// Dynamic LDS a plan can take next to its static stage buffers.
int plan_max_dynamic(const Plan &p) { return std::min(kMaxTableBytes, kLdsBytes - p.static_lds - 256); }

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

void set_kernel_attributes()
{
    for (const void *fn : {reinterpret_cast<const void *>(&fast_ndft_kernel<FAST_X>),
                           reinterpret_cast<const void *>(&fast_ndft_kernel<FAST_LAG>),
                           reinterpret_cast<const void *>(&fast_ndft_kernel<FAST_LIN>)}) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           fast_lds_bytes(kFastMaxN, 2 * 64));
        if (e != hipSuccess && g_attr_err == hipSuccess) g_attr_err = e;
    }
    for (int prec = 0; prec < 3; ++prec)
        for (const Plan &p : plans(prec))
            for (int k = 0; k < 4; ++k) {
                const void *fn = k < 2 ? p.kfn[k] : (k == 2 ? p.kfn_batched : p.planes_kfn);
                if (!fn) continue;
                hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, plan_max_dynamic(p));
                if (e != hipSuccess && g_attr_err == hipSuccess) g_attr_err = e;
            }
}

struct Dft12bLaunch {
    int lb, M, MB, n_mg, tb, n_coarse;
    int fast;         // L = 512: dft512_kernel (a work-group per delay row, no partials)
    int codes;        // a sign half: the fast kernel reads the twiddle-sign kernel's codes
    size_t dyn_bytes; // the twiddle table (dynamic LDS)
    size_t ws_bytes;  // partial surfaces when a delay takes more than one work-group
};

struct Launch {
    const Plan *plan;
    int prec;
    int ksplit, kchunk;
    int tiles_b, tiles_l;
    int n_bases, n_bases_pad, n_cols_pad;
    int tb, n_coarse, tw_exact;
    BaseMap bm;        // every base, in partial-row order (reduction)
    BaseMap bm_tile;   // bases of the matrix rows: bm without base 0 when row0 = 1
    int row0;          // 1: base 0 is summed on the vector units into partial row 0
    int ksT;           // sign-split: lsum_kernel chunks (partial planes after the ksplit ones)
    long long kchunkT; // sign-split: samples per lsum_kernel chunk
    long long k_codes; // sign-split: samples covered by the sign codes (n rounded up)
    size_t code_off;   // sign-split: offset of the sign codes in the workspace
    size_t code_bytes; // sign-split: their bytes (the packed layout for fft_d plans)
    size_t part_bytes; // split-K partials
    size_t ws_bytes;   // partials + signed copies of the inputs (+ twiddle planes)
    long long plane_stages; // planes: stage blocks per base tile
    size_t plane_bytes;
    size_t plane_off;       // offset of the planes in the workspace
    int grp_stride;
    int lin;           // sign-split: the Eq. (12c) lag product (lag_kfn_lin)
    int fits;          // the twiddle table fits the plan's dynamic LDS (else NDFT_E_UNSUPPORTED)
    Dft12bLaunch dft;  // fft_d plans: the twiddle half's decimated FFT
    size_t dft_off;    // fft_d plans: offset of its partial surfaces in the workspace
    size_t absmax_off; // FP8 combined plans: two words of data maxima (0: none)
};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Split-K count: minimises the rounds of work-groups over the compute units per unit of
// tile work, times 1 + k/256 for the partial sums each chunk adds (written, then read by
// the reduction); the smaller count on ties.
int pick_ksplit(int tiles, int64_t n, int ks, int cus)
{
    int max_k = (int)std::max<int64_t>(1, cdiv(n, 8LL * ks)); // at least ~8 stages per chunk
    int best = 1;
    double best_cost = -1.0;
    for (int k = 1; k <= max_k; ++k) {
        const double rounds = (double)cdiv((int64_t)tiles * k, cus);
        const double cost = rounds / k * (1.0 + k / 256.0);
        if (best_cost < 0.0 || cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = k;
        }
    }
    return best;
}

// Two-level table for length n within max_bytes of LDS: fine size 2^tb >= sqrt(n) by
// default. The exact form needs every quadrant point m in {n/4, n/2, 3n/4} that is an
// integer to have m mod 2^tb = 0 (2^tb divides n/4, resp. n/2 for n = 2 mod 4; any tb
// for odd n) and n <= 2^20; tb is lowered to get it when the coarse table still fits.
void choose_table(int64_t n, int max_bytes, int *tb_out, int *n_coarse_out, int *exact_out)
{
    int tb = 0;
    while ((1LL << (2 * tb)) < n) ++tb;
    int exact = 0;
    if (n <= (1 << 20)) {
        int v = 0;
        while (((n >> v) & 1) == 0) ++v;
        const int cap = n % 4 == 0 ? v - 2 : (n % 2 == 0 ? v - 1 : 62);
        const int t = std::min(tb, cap);
        if ((cdiv(n, 1LL << t) + (1LL << t)) * (int64_t)sizeof(float2) <= max_bytes) {
            tb = t;
            exact = 1;
        }
    }
    *tb_out = tb;
    *n_coarse_out = (int)cdiv(n, 1LL << tb);
    *exact_out = exact;
}

// Work-groups of a plan's main kernel that fit one compute unit together (register and
// LDS use of the built kernel, from the runtime); 1 when it cannot be queried.
int plan_occupancy(const Plan &p, int prod, size_t dyn_shmem)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, size_t>, int> cache;
    const void *fn = p.kfn[prod];
    if (!fn) return 1;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, dyn_shmem});
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, p.nt, dyn_shmem) != hipSuccess || nb < 1) nb = 1;
    cache[{fn, dyn_shmem}] = nb;
    return nb;
}

// Largest base of a base map (bases ascend).
int max_base(const BaseMap &bm, int n_bases)
{
    if (bm.nseg == 0) return 0;
    const int k = bm.nseg - 1;
    return bm.start[k] + (n_bases - bm.off[k]) - 1;
}

// Base 0 goes to the vector units (partial row 0) when the register-lag kernels run the
// lag product, base 0 is in the set and the other bases fill whole tiles: one base would
// otherwise cost a whole padded tile row.
int zero_row(const Plan &p, int prod, const BaseMap &bm, int n_bases)
{
    if (p.lag_kfn) return bm.nseg > 0 && bm.start[0] == 0 ? 1 : 0; // base 0 always apart
    return p.raw_inputs && prod == PROD_LAG && bm.nseg > 0 && bm.start[0] == 0 && n_bases > 1 &&
                   (n_bases - 1) % p.bt == 0
               ? 1
               : 0;
}

BaseMap drop_first_base(const BaseMap &bm)
{
    BaseMap r = bm;
    if (bm.off[1] - bm.off[0] == 1) { // first run is the single base: remove the run
        r.nseg = bm.nseg - 1;
        for (int k = 0; k < 4; ++k) r.start[k] = k + 1 < 4 ? bm.start[k + 1] : 0;
        for (int k = 0; k < 5; ++k) r.off[k] = k + 1 < 5 ? bm.off[k + 1] - 1 : bm.off[4] - 1;
    } else {
        r.start[0] = bm.start[0] + 1;
        for (int k = 1; k < 5; ++k) r.off[k] = bm.off[k] - 1;
    }
    return r;
}

// lsum_kernel base groups (blockIdx.z): kLsumBases base rows each, after row 0 when base 0
// is present (summed apart)
int64_t lsum_groups(const Launch &L)
{
    const int has0 = L.bm.nseg > 0 && L.bm.start[0] == 0;
    return std::max<int64_t>(1, cdiv(L.n_bases - has0, kLsumBases));
}

// ------------------------------------------------------------------------------------
// the Eq. (12b) surface: decimated DFT of the lag-product rows
// ------------------------------------------------------------------------------------

// whole_rows: allow the whole-row kernel (the Eq. (12c) signs stay on the phase-group
// kernel, which measured faster for them)
Dft12bLaunch plan_dft12b(int64_t n, int64_t n_tau, int64_t n_dop, size_t code_bytes = 0)
{
    Dft12bLaunch L;
    std::memset(&L, 0, sizeof(L));
    while (L.lb < kDftMaxLog && n % (2LL << L.lb) == 0) ++L.lb; // L = 2^lb, the largest power of two dividing n
    L.M = (int)(n >> L.lb);
    L.MB = std::min(kDftTile >> L.lb, L.M);
    L.n_mg = (int)cdiv(L.M, L.MB);
    int exact = 0;
    choose_table(n, 65536, &L.tb, &L.n_coarse, &exact);
    L.dyn_bytes = (size_t)(L.n_coarse + (1 << L.tb)) * sizeof(float2);
    // the whole-row kernel wherever it has enough rows to fill the device (or a row is a
    // single group of transforms anyway); the sign halves (code_bytes > 0) read the sign
    // codes through 32-bit buffer offsets
    L.fast = L.lb == 9 && n_dop <= kD5MaxBins && (n_tau >= 128 || L.M <= kD5Group) &&
                     code_bytes < (size_t(1) << 31)
                 ? 1
                 : 0;
    L.codes = code_bytes > 0 ? 1 : 0;
    if (L.fast) L.n_mg = 1;
    // whole-row kernel on the lag products: the signed inputs s4[n], r4[2 n]; else the
    // partial surfaces
    L.ws_bytes = L.fast ? (L.codes ? 0 : align256((size_t)n * sizeof(float4)) + align256((size_t)2 * n * sizeof(float4)))
                        : (L.n_mg > 1 ? align256((size_t)L.n_mg * n_tau * n_dop * sizeof(float2)) : 0);
    return L;
}

// lin: the Eq. (12c) surface, which only the sign-split plans compute; L.plan is nullptr
// when the precision has none.
Launch plan_launch(int prec, int prod, int64_t n, int64_t n_cols, int64_t p0, int64_t n_bins,
                   int64_t signed_elems, bool lin = false)
{
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.prec = prec;
    L.lin = lin ? 1 : 0;
    L.bm = make_base_map(n, p0, n_bins, &L.n_bases);
    int pi, ko;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        pi = g_plan_override[prec];
        ko = g_ksplit_override[prec];
    }
    const std::vector<Plan> &ps = plans(prec);
    // the fast exact transform takes either lag product; where it can, the sign-split plans
    // keep the walk short for the Eq. (12c) surface too
    bool fast_here = false;
    for (const Plan &q : ps) fast_here = fast_here || (q.fastx && fast_ok(n));
    auto usable = [&](int k) {
        if (ps[k].fastx) return fast_ok(n);
        if (lin) return ps[k].lag_kfn_lin != nullptr;
        return ps[k].kfn[prod] != nullptr || (prod == PROD_LAG && ps[k].fft_d);
    };
    if (pi < 0 || pi >= (int)ps.size() || !usable(pi)) {
        // built-in choice: padded matrix-core work times the plan's operand-generation
        // overhead, then the earlier plan
        double best = -1.0;
        pi = lin ? -1 : 0;
        for (int k = 0; k < (int)ps.size(); ++k) {
            if (!usable(k)) continue;
            // sign-split: the twiddle-sign part walks 2 b C / N sign changes per base b, part
            // and chunk of C samples; taken while that stays at most 2 (b C <= N) for the
            // matrix-core plans, whose twiddle half is dense in the bases anyway, and at most
            // 8 (b C / 4 <= N) for the FP32 plan, whose FFT half costs the same for any
            // window (the Eq. (12c) surface has no other form: the walk is exact for any base)
            const int64_t runs_c = ps[k].fft_d ? kLsumChunk / 4 : kLsumChunk;
            if ((!lin || fast_here) && ps[k].lag_kfn && (int64_t)max_base(L.bm, L.n_bases) * runs_c > n) continue;
            // the FFT of the twiddle half wants a power-of-two factor of at least 64 in n
            if (!lin && ps[k].fft_d && n % 64 != 0) continue;
            const int r0 = ps[k].fastx ? 0 : zero_row(ps[k], prod, L.bm, L.n_bases);
            double rows = (double)(cdiv(L.n_bases - r0, ps[k].bt) * ps[k].bt);
            double cols = (double)(cdiv(n_cols, ps[k].lt) * ps[k].lt);
            double cost = ps[k].fastx ? cols * fast_row_cost(n)
                                      : rows * (cols + ps[k].row_cost_cols) * ps[k].cost_scale;
            if (best < 0 || cost < best * 0.999) {
                best = cost;
                pi = k;
            }
        }
    }
    if (pi < 0) return L; // L.plan stays nullptr
    L.plan = &ps[pi];
    if (L.plan->fastx) {
        // tables of the call: the group order, its inverse, the correlation spectra
        choose_table(n, kMaxTableBytes, &L.tb, &L.n_coarse, &L.tw_exact);
        L.fits = 1;
        L.ws_bytes = 2 * align256((size_t)(n / 2) * sizeof(int)) +
                     align256((size_t)std::max(1, fast_spec_entries((int)n)) * sizeof(float2));
        return L;
    }
    L.row0 = zero_row(*L.plan, prod, L.bm, L.n_bases);
    L.bm_tile = L.row0 ? drop_first_base(L.bm) : L.bm;
    L.tiles_b = (int)cdiv(L.n_bases - L.row0, L.plan->bt);
    L.tiles_l = (int)cdiv(n_cols, L.plan->lt);
    L.n_bases_pad = L.row0 + L.tiles_b * L.plan->bt;
    L.n_cols_pad = L.tiles_l * L.plan->lt;
    const int gran = L.plan->kgran;
    int max_split = (int)std::max<int64_t>(1, cdiv(n, gran));
    const int cus = device_cu_count();
    choose_table(n, plan_max_dynamic(*L.plan), &L.tb, &L.n_coarse, &L.tw_exact);
    L.fits = (int64_t)(L.n_coarse + (1 << L.tb)) * (int64_t)sizeof(float2) <= plan_max_dynamic(*L.plan) ? 1 : 0;
    // work-group slots: compute units times the plan's work-groups per unit
    const size_t dyn = L.plan->lag_kfn && !L.plan->planes_kfn ? (size_t)(L.n_coarse + (1 << L.tb)) * sizeof(float2) : 0;
    const int slots = cus * (L.plan->lag_kfn ? plan_occupancy(*L.plan, prod, dyn) : 1);
    L.ksplit = ko > 0 ? std::min(ko, max_split) : pick_ksplit(L.tiles_b * L.tiles_l, n, gran, slots);
    L.kchunk = (int)(cdiv(cdiv(n, L.ksplit), gran) * gran);
    L.ksplit = (int)cdiv(n, L.kchunk); // no empty chunks
    if (L.tiles_b == 0) L.ksplit = 0;  // sign-split with base 0 only: no matrix part
    if (L.plan->fft_d) L.ksplit = 0;   // the twiddle half is not a matrix contraction
    if (L.plan->lag_kfn) {
        // lsum_kernel: blocks of kLsumDelays delays x kLsumBases bases x a sample range of
        // whole chunks; about two blocks per compute unit
        L.k_codes = cdiv(n, kLsumChunk) * kLsumChunk;
        const int64_t nck = L.k_codes / kLsumChunk;
        const int64_t blocks = cdiv(n_cols, kLsumDelays) * lsum_groups(L);
        int64_t ks = std::min<int64_t>(nck, std::max<int64_t>(1, cdiv(2LL * cus, blocks)));
        L.kchunkT = cdiv(nck, ks) * kLsumChunk;
        L.ksT = (int)cdiv(L.k_codes, L.kchunkT);
    }
    L.part_bytes = align256((size_t)(L.ksplit + L.ksT) * L.n_cols_pad * L.n_bases_pad * sizeof(float4));
    L.ws_bytes = L.part_bytes + align256((size_t)signed_elems * sizeof(float4));
    if (L.plan->planes_kfn) {
        // every stage a chunk can reach, the one after the last included (prefetch)
        L.plane_stages = L.plan->lag_kfn ? L.k_codes / L.plan->ks + 1 : 2 * cdiv(n, 2LL * L.plan->ks) + 1;
        L.plane_bytes = align256((size_t)L.tiles_b * L.plane_stages * L.plan->stage_a * sizeof(uint4));
        L.plane_off = L.ws_bytes;
        L.ws_bytes += L.plane_bytes;
        L.grp_stride = (int)(cdiv((int64_t)L.tiles_b * L.ksplit, 8) * 8);
    }
    if (L.plan->lag_kfn) {
        L.grp_stride = (int)(cdiv((int64_t)L.tiles_b * L.ksplit, 8) * 8);
        L.code_off = L.ws_bytes;
        // one byte per delay and sample in the matrix kernels' layout, half a byte packed
        L.code_bytes = (size_t)L.k_codes * L.n_cols_pad / (L.plan->fft_d ? 2 : 1);
        L.ws_bytes += align256(L.code_bytes);
    }
    if (L.plan->fft_d) {
        L.dft = plan_dft12b(n, n_cols, n_bins, L.code_bytes);
        L.dft_off = L.ws_bytes;
        L.ws_bytes += L.dft.ws_bytes;
    }
    if (prec == NDFT_FP8 && !L.plan->lag_kfn) { // the e4m3 data exponent of the combined kernel
        L.absmax_off = L.ws_bytes;
        L.ws_bytes += 256;
    }
    return L;
}

// ------------------------------------------------------------------------------------
// profiling events
// ------------------------------------------------------------------------------------
std::mutex g_prof_mu;
bool g_prof_on = false;
// set for the duration of an ndft_caf_noalloc call on this thread: no event records
thread_local bool t_no_prof = false;
// slot 0: the contraction (or its FFT) kernel; slot 1: the twiddle-sign kernel
constexpr int kProfSlots = 2;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pending[kProfSlots];
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache write-back) when the event completes, so
    // the records do not slow the kernels between them
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    int slot;
    explicit ProfScope(hipStream_t st, int sl = 0) : s(st), slot(sl)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on || t_no_prof) return;
        a = take_event();
        b = take_event();
        if (a && b) (void)hipEventRecord(a, s);
    }
    void stop()
    {
        if (!(a && b)) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending[slot].push_back({a, b});
        a = b = nullptr;
    }
};

ndft_status check_launch()
{
    return hipGetLastError() == hipSuccess ? NDFT_OK : NDFT_E_HIP;
}

ndft_status launch_prep(const float2 *x, float4 *out, int64_t n, int64_t rows, int64_t ostride, int64_t lead,
                        float g, hipStream_t stream)
{
    int64_t count = rows * ostride;
    if (count == 0) return NDFT_OK;
    hipLaunchKernelGGL(sign_prep_kernel, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, stream, x, out, (int)n,
                       (long long)rows, (long long)ostride, (int)lead, g);
    return check_launch();
}

// The surveillance and the reference rows with their signs in one launch: s -> s4 (s_len
// entries, s from 0), r -> r4 (r_len entries, r from r_lead).
ndft_status launch_prep_pair(const float2 *s, float4 *s4, int64_t s_len, const float2 *r, float4 *r4, int64_t r_len,
                             int64_t r_lead, int64_t n, float g, hipStream_t stream)
{
    PrepPair Q;
    Q.x[0] = s;
    Q.x[1] = r;
    Q.out[0] = s4;
    Q.out[1] = r4;
    Q.ostride[0] = s_len;
    Q.ostride[1] = r_len;
    Q.lead[0] = 0;
    Q.lead[1] = (int)r_lead;
    const int64_t len = std::max(s_len, r_len);
    if (len == 0) return NDFT_OK;
    hipLaunchKernelGGL(sign_prep_pair_kernel, dim3((unsigned)cdiv(len, 256), 2), dim3(256), 0, stream, Q, (int)n, g);
    return check_launch();
}

// FP8 combined kernel: the largest |re| + |im| of each input (one word each) into the
// workspace slot, cleared first by a kernel of its own (no memset in the stream).
ndft_status launch_absmax(unsigned *w, const float2 *a, int64_t na, const float2 *b, int64_t nb, hipStream_t s)
{
    hipLaunchKernelGGL(absmax_zero_kernel, dim3(1), dim3(64), 0, s, w, 2);
    const auto grid = [](int64_t c) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(c, 256), 1024))); };
    hipLaunchKernelGGL(absmax_kernel, grid(na), dim3(256), 0, s, a, (long long)na, w);
    if (b) hipLaunchKernelGGL(absmax_kernel, grid(nb), dim3(256), 0, s, b, (long long)nb, w + 1);
    return check_launch();
}

ndft_status launch_contract(const Launch &L, int prod, const float4 *s4, const float4 *r4, long long col_stride,
                            int64_t n, int64_t n_cols, int64_t tau0, float4 *partial, hipStream_t stream,
                            uint4 *planes = nullptr, const float2 *s_raw = nullptr, const float2 *r_raw = nullptr,
                            const unsigned *absmax = nullptr)
{
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    ContractParams P;
    std::memset(&P, 0, sizeof(P));
    P.s4 = s4;
    P.r4 = r4;
    P.s_raw = s_raw;
    P.r_raw = r_raw;
    P.col_stride = col_stride;
    P.n = (int)n;
    P.n_cols = (int)n_cols;
    P.tau0 = (int)tau0;
    P.n_bases = L.n_bases - L.row0;
    P.bm = L.bm_tile;
    P.row0 = L.row0;
    P.tb = L.tb;
    P.n_coarse = L.n_coarse;
    P.tw_exact = L.tw_exact;
    P.kchunk = L.kchunk;
    P.ksplit = L.ksplit;
    P.tiles_b = L.tiles_b;
    P.tiles_l = L.tiles_l;
    P.n_bases_pad = L.n_bases_pad;
    P.n_cols_pad = L.n_cols_pad;
    P.partial = partial;
    P.absmax = absmax;
    if (L.prec == NDFT_FP8 && !absmax) return NDFT_E_INVAL;
    void *args[] = {&P};
    size_t shmem = (size_t)(L.n_coarse + (1 << L.tb)) * sizeof(float2);
    if ((int)shmem > plan_max_dynamic(*L.plan)) return NDFT_E_UNSUPPORTED; // FP8 stages leave less LDS
    if (!L.plan->kfn[prod]) return NDFT_E_UNSUPPORTED;
    dim3 grid((unsigned)((int64_t)L.tiles_b * L.tiles_l * L.ksplit));
    dim3 block((unsigned)L.plan->nt);
    if (L.plan->planes_kfn) {
        if (!planes) return NDFT_E_INVAL;
        P.planes = planes;
        P.plane_stages = L.plane_stages;
        P.grp_stride = L.grp_stride;
        PlaneBuildParams Q;
        std::memset(&Q, 0, sizeof(Q));
        Q.planes = planes;
        Q.plane_stages = L.plane_stages;
        Q.n = (int)n;
        Q.tb = L.tb;
        Q.n_coarse = L.n_coarse;
        Q.tw_exact = L.tw_exact;
        // about two work-groups per compute unit (each builds its own twiddle table)
        Q.stages_per_block =
            (int)std::max<int64_t>(1, cdiv((int64_t)L.plane_stages * L.tiles_b, 2LL * device_cu_count()));
        Q.bm = L.bm_tile;
        void *qargs[] = {&Q};
        dim3 qgrid((unsigned)cdiv(L.plane_stages, Q.stages_per_block), (unsigned)L.tiles_b);
        if (hipLaunchKernel(L.plan->planes_kfn, qgrid, dim3(256), qargs, shmem, stream) != hipSuccess)
            return NDFT_E_HIP;
        grid = dim3((unsigned)((int64_t)L.tiles_l * L.grp_stride));
        shmem = 0;
    }
    ProfScope prof(stream);
    hipError_t e = hipLaunchKernel(L.plan->kfn[prod], grid, block, args, shmem, stream);
    prof.stop();
    if (e != hipSuccess) return NDFT_E_HIP;
    return check_launch();
}

// Sign-split form: twiddle planes, lsum_kernel (twiddle-sign part, sign codes, base 0),
// dsum_kernel (twiddles against the lag signs); the reduction follows.
// lsum_only: the lag kernel alone (no planes, no matrix part), for the sign test hook.
ndft_status launch_split(const Launch &L, const float2 *surv, const float2 *ref, int64_t n, int64_t n_cols,
                         int64_t tau0, float4 *partial, void *ws, hipStream_t stream, bool lsum_only = false)
{
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    uint32_t *codes = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + L.code_off);
    uint4 *planes = reinterpret_cast<uint4 *>(static_cast<char *>(ws) + L.plane_off);
    const size_t shmem = (size_t)(L.n_coarse + (1 << L.tb)) * sizeof(float2);
    if ((int)shmem > plan_max_dynamic(*L.plan)) return NDFT_E_UNSUPPORTED;
    if (!lsum_only && L.tiles_b > 0 && L.plan->planes_kfn) {
        DplaneParams Q;
        std::memset(&Q, 0, sizeof(Q));
        Q.planes = planes;
        Q.plane_stages = L.plane_stages;
        Q.n = (int)n;
        Q.tb = L.tb;
        Q.n_coarse = L.n_coarse;
        // about two work-groups per compute unit (each builds its own twiddle table)
        Q.stages_per_block =
            (int)std::max<int64_t>(1, cdiv((int64_t)L.plane_stages * L.tiles_b, 2LL * device_cu_count()));
        Q.bm = L.bm_tile;
        void *qargs[] = {&Q};
        dim3 qgrid((unsigned)cdiv(L.plane_stages, Q.stages_per_block), (unsigned)L.tiles_b);
        if (hipLaunchKernel(L.plan->planes_kfn, qgrid, dim3(256), qargs, shmem, stream) != hipSuccess)
            return NDFT_E_HIP;
    }
    {
        LsumParams T;
        std::memset(&T, 0, sizeof(T));
        T.s = surv;
        T.r = ref;
        T.n = (int)n;
        T.n_cols = (int)n_cols;
        T.tau0 = (int)tau0;
        T.bm = L.bm;
        T.n_bases = L.n_bases;
        T.n_bases_pad = L.n_bases_pad;
        T.n_cols_pad = L.n_cols_pad;
        T.kchunk = L.kchunkT;
        T.k_end = L.k_codes;
        T.codes = codes;
        T.code_wpc = L.k_codes / 8;
        T.part = partial + (size_t)L.ksplit * L.n_cols_pad * L.n_bases_pad;
        void *targs[] = {&T};
        dim3 tgrid((unsigned)cdiv(n_cols, kLsumDelays), (unsigned)L.ksT, (unsigned)lsum_groups(L));
        const void *tfn = L.lin ? L.plan->lag_kfn_lin : L.plan->lag_kfn;
        ProfScope tprof(stream, 1);
        const hipError_t te = hipLaunchKernel(tfn, tgrid, dim3(256), targs, 0, stream);
        tprof.stop();
        if (te != hipSuccess) return NDFT_E_HIP;
    }
    ndft_status st = check_launch();
    if (st != NDFT_OK || lsum_only || L.tiles_b == 0 || L.plan->fft_d) return st; // fft_d: the FFT runs after the reduction
    ContractParams P;
    std::memset(&P, 0, sizeof(P));
    P.n = (int)n;
    P.n_cols = (int)n_cols;
    P.tau0 = (int)tau0;
    P.n_bases = L.n_bases - L.row0;
    P.bm = L.bm_tile;
    P.row0 = L.row0;
    P.kchunk = L.kchunk;
    P.ksplit = L.ksplit;
    P.tiles_b = L.tiles_b;
    P.tiles_l = L.tiles_l;
    P.n_bases_pad = L.n_bases_pad;
    P.n_cols_pad = L.n_cols_pad;
    P.partial = partial;
    P.planes = planes;
    P.plane_stages = L.plane_stages;
    P.grp_stride = L.grp_stride;
    P.tb = L.tb;
    P.n_coarse = L.n_coarse;
    const uint32_t *ccodes = codes;
    long long code_stages = L.k_codes / 32;
    void *args[] = {&P, &ccodes, &code_stages};
    ProfScope prof(stream);
    hipError_t e = hipLaunchKernel(L.plan->kfn[PROD_LAG], dim3((unsigned)((int64_t)L.tiles_l * L.grp_stride)),
                                   dim3((unsigned)L.plan->nt), args, L.plan->planes_kfn ? 0 : shmem, stream);
    prof.stop();
    if (e != hipSuccess) return NDFT_E_HIP;
    return check_launch();
}

ndft_status launch_reduce(const Launch &L, const float4 *partial, int64_t n, int64_t n_cols, int64_t p0,
                          int64_t n_bins, float2 *out, hipStream_t stream)
{
    ReduceParams R;
    std::memset(&R, 0, sizeof(R));
    R.partial = partial;
    R.ksplit = L.ksplit + L.ksT; // sign-split: lsum_kernel's planes follow the matrix ones
    R.n_cols_pad = L.n_cols_pad;
    R.n_bases_pad = L.n_bases_pad;
    R.n_cols = (int)n_cols;
    R.n_bases = L.n_bases;
    R.bm = L.bm;
    R.n = (int)n;
    R.p0n = (int)mod_n(p0, n);
    R.n_bins = (int)n_bins;
    R.out = out;
    int64_t total = n_cols * (int64_t)L.n_bases;
    if (total == 0) return NDFT_OK;
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, stream, R);
    return check_launch();
}

bool prec_ok(ndft_prec p) { return p == NDFT_FP32 || p == NDFT_BF16X2 || p == NDFT_FP8; }

// Table bytes for length n (coarse + fine two-level twiddle table).
int table_bytes_for(int64_t n)
{
    int tb = 0;
    while ((1LL << (2 * tb)) < n) ++tb;
    return (int)((cdiv(n, 1LL << tb) + (1LL << tb)) * sizeof(float2));
}

bool caf_args_ok(int64_t n, int64_t tau0, int64_t n_tau, int64_t n_dop)
{
    return n >= 1 && n <= NDFT_MAX_N && tau0 >= 0 && n_tau >= 1 && tau0 + n_tau <= n && n_dop >= 1 &&
           n_dop <= n;
}

ndft_status ws_ok(void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return NDFT_OK;
    if (!ws || ws_bytes < need || !aligned(ws, 256)) return NDFT_E_WORKSPACE;
    return NDFT_OK;
}

template <int SRC>
const void *dft12b_fn(int lb)
{
    static const void *fns[kDftMaxLog + 1] = {
        reinterpret_cast<const void *>(&dft12b_kernel<0, SRC>), reinterpret_cast<const void *>(&dft12b_kernel<1, SRC>),
        reinterpret_cast<const void *>(&dft12b_kernel<2, SRC>), reinterpret_cast<const void *>(&dft12b_kernel<3, SRC>),
        reinterpret_cast<const void *>(&dft12b_kernel<4, SRC>), reinterpret_cast<const void *>(&dft12b_kernel<5, SRC>),
        reinterpret_cast<const void *>(&dft12b_kernel<6, SRC>), reinterpret_cast<const void *>(&dft12b_kernel<7, SRC>),
        reinterpret_cast<const void *>(&dft12b_kernel<8, SRC>), reinterpret_cast<const void *>(&dft12b_kernel<9, SRC>)};
    static_assert(kDftMaxLog == 9, "one instance per transform length");
    return fns[lb];
}

template <int SRC>
const void *dft512_fn()
{
    return reinterpret_cast<const void *>(&dft512_kernel<SRC>);
}

std::once_flag g_dft_attr_once;
hipError_t g_dft_attr_err = hipSuccess;

// The decimated DFT of the lag products (src DFT_LAG: the Eq. (12b) surface) or of their
// exact signs (DFT_SIGNS / DFT_LIN_SIGNS: the twiddle half of the Eq. (12a) / Eq. (12c)
// sign-split forms, bin 0 left out), written to A or, with accumulate, added to it. ws
// holds the partial surfaces.
// The fast kernel on a sign half reads the packed sign codes at `codes` (code_wpc words per
// delay row, code_bytes in all) that the twiddle-sign kernel wrote earlier on the stream.
ndft_status launch_dft(const Dft12bLaunch &L, const float2 *surv, const float2 *ref, int64_t n, int64_t tau0,
                       int64_t n_tau, int64_t p0, int64_t n_dop, float2 *A, void *ws, int src, bool accumulate,
                       hipStream_t s, const uint32_t *codes = nullptr, int64_t code_wpc = 0, size_t code_bytes = 0,
                       const TsumParams *tsum = nullptr)
{
    std::call_once(g_dft_attr_once, [] {
        for (int lb = 0; lb <= kDftMaxLog; ++lb)
            for (const void *fn : {dft12b_fn<DFT_LAG>(lb), dft12b_fn<DFT_SIGNS>(lb), dft12b_fn<DFT_LIN_SIGNS>(lb)}) {
                hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
                if (e != hipSuccess && g_dft_attr_err == hipSuccess) g_dft_attr_err = e;
            }
        for (const void *fn : {dft512_fn<DFT_LAG>(), dft512_fn<DFT_CODES>()}) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
            if (e != hipSuccess && g_dft_attr_err == hipSuccess) g_dft_attr_err = e;
        }
    });
    if (g_dft_attr_err != hipSuccess) return NDFT_E_HIP;
    if (L.n_mg > 1 && cdiv((long long)n_tau * n_dop, 256) > (long long)UINT32_MAX) return NDFT_E_INVAL;
    Dft12bParams P;
    std::memset(&P, 0, sizeof(P));
    P.s = surv;
    P.r = ref;
    P.n = (int)n;
    P.tau0 = (int)tau0;
    P.n_tau = (int)n_tau;
    P.p0n = (int)mod_n(p0, n);
    P.n_dop = (int)n_dop;
    P.M = L.M;
    P.MB = L.MB;
    P.n_mg = L.n_mg;
    P.tb = L.tb;
    P.n_coarse = L.n_coarse;
    P.out = L.n_mg > 1 ? static_cast<float2 *>(ws) : A;
    P.accumulate = L.n_mg > 1 ? 0 : (accumulate ? 1 : 0);
    TsumParams T;
    std::memset(&T, 0, sizeof(T));
    void *args[] = {&P};
    void *args5[] = {&P, &T};
    if (L.fast) {
        // two work-groups per compute unit, each taking whole delay rows in turn
        if (src == DFT_LAG) {
            // the inputs with their exact signs (the reference after n zeros)
            float4 *s4 = static_cast<float4 *>(ws);
            float4 *r4 = reinterpret_cast<float4 *>(static_cast<char *>(ws) + align256((size_t)n * sizeof(float4)));
            ndft_status st = launch_prep_pair(surv, s4, n, ref, r4, 2 * n, n, n, 1.0f, s);
            if (st != NDFT_OK) return st;
            P.s4 = s4;
            P.r4 = r4;
        } else {
            // a sign half: the codes of the call's twiddle-sign kernel
            if (!L.codes || !codes || code_bytes >= (size_t(1) << 31) || code_wpc * 8 < n ||
                (size_t)(code_wpc * 4) * (size_t)n_tau > code_bytes)
                return NDFT_E_INVAL;
            P.codes = codes;
            P.code_wpc = (int)code_wpc;
            P.code_bytes = (unsigned)code_bytes;
            if (tsum) T = *tsum; // the other half's planes, added here instead of by a reduction
        }
        const dim3 grid((unsigned)std::min<int64_t>(n_tau, 2LL * device_cu_count()));
        const void *fn = src == DFT_LAG ? dft512_fn<DFT_LAG>() : dft512_fn<DFT_CODES>();
        ProfScope prof(s);
        hipError_t e = hipLaunchKernel(fn, grid, dim3(kD5Threads), args5, L.dyn_bytes, s);
        prof.stop();
        if (e != hipSuccess) return NDFT_E_HIP;
        return check_launch();
    }
    // about eight work-groups per compute unit, each looping over its delays (the table
    // is built once per work-group)
    const int64_t ydim = std::max<int64_t>(1, cdiv(8LL * device_cu_count(), L.n_mg));
    const dim3 grid((unsigned)L.n_mg, (unsigned)std::min<int64_t>(std::min<int64_t>(n_tau, ydim), 65535));
    const void *fn = src == DFT_SIGNS ? dft12b_fn<DFT_SIGNS>(L.lb)
                     : (src == DFT_LIN_SIGNS ? dft12b_fn<DFT_LIN_SIGNS>(L.lb) : dft12b_fn<DFT_LAG>(L.lb));
    ProfScope prof(s);
    hipError_t e = hipLaunchKernel(fn, grid, dim3(kDftThreads), args, L.dyn_bytes, s);
    prof.stop();
    if (e != hipSuccess) return NDFT_E_HIP;
    if (L.n_mg > 1) {
        const long long cells = (long long)n_tau * n_dop;
        hipLaunchKernelGGL(dft12b_reduce_kernel, dim3((unsigned)cdiv(cells, 256)), dim3(256), 0, s,
                           static_cast<const float2 *>(ws), L.n_mg, cells, A, accumulate ? 1 : 0);
    }
    return check_launch();
}

struct AdjLaunch {
    BaseMap bm;
    int n_bases, n_bases_pad;
    size_t eo_bytes, dz_bytes, ws_bytes;
};

AdjLaunch plan_adjoint(int64_t n, int64_t n_tau, int64_t p0, int64_t n_dop)
{
    AdjLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.bm = make_base_map(n, p0, n_dop, &L.n_bases);
    L.n_bases_pad = (int)(cdiv(L.n_bases, 8) * 8);
    L.eo_bytes = align256((size_t)L.n_bases_pad * n_tau * sizeof(float4));
    L.dz_bytes = align256((size_t)n_tau * n * sizeof(float2));
    L.ws_bytes = L.eo_bytes + L.dz_bytes;
    return L;
}

// ------------------------------------------------------------------------------------
// batched surfaces: geometry, tables and workspace layout
// ------------------------------------------------------------------------------------
struct BatchGeom {
    int plan = 0;
    int chunk = 0;
    int table_bytes = 0;
    int max_red_blocks = 1;
    int max_prep_blocks = 1;
    BatchRegions rg;
    size_t total = 0;
    std::vector<ContractParams> params;
    std::vector<ReduceParams> red;
    std::vector<long long> outoff;
    std::vector<PrepDesc> prep;
    std::vector<int4> items;
};

BatchPlanGeom batch_plan_geom(const Plan &P, int prec)
{
    BatchPlanGeom g;
    g.bt = P.bt;
    g.lt = P.lt;
    g.max_dynamic = plan_max_dynamic(P);
    g.sign_scale = P.sign_scale;
    g.fp8 = prec == NDFT_FP8 ? 1 : 0;
    return g;
}

// The plan of a batch: the override if it has a batched kernel, else the least summed
// cost over the CPIs (padded cells times samples, scaled per plan).
int batch_plan_choice(const ndft_cpi *cpis, int n_cpi, int prec)
{
    const std::vector<Plan> &ps = plans(prec);
    int pi;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        pi = g_plan_override[prec];
    }
    if (pi >= 0 && pi < (int)ps.size() && ps[pi].kfn_batched) return pi;
    double best = -1.0;
    pi = 0;
    for (int k = 0; k < (int)ps.size(); ++k) {
        if (!ps[k].kfn_batched) continue;
        double cost = 0.0;
        for (int c = 0; c < n_cpi; ++c) {
            int nb;
            make_base_map(cpis[c].n, cpis[c].p0, cpis[c].n_dop, &nb);
            double rows = (double)(cdiv(nb, ps[k].bt) * ps[k].bt);
            double cols = (double)(cdiv(cpis[c].n_tau, ps[k].lt) * ps[k].lt);
            cost += rows * cols * (double)cpis[c].n * ps[k].cost_scale;
        }
        if (best < 0 || cost < best * 0.999) {
            best = cost;
            pi = k;
        }
    }
    return pi;
}

// Pick the plan, lay out the workspace (ndft_batch.hpp) and build the tables; `base` is
// the workspace address (nullptr when only sizing).
ndft_status batch_geometry(const ndft_cpi *cpis, int n_cpi, int prec, int chunk, char *base, BatchGeom &G)
{
    if (!cpis || n_cpi < 1 || n_cpi > kMaxBatch || chunk < 0) return NDFT_E_INVAL;
    for (int c = 0; c < n_cpi; ++c)
        if (!cpi_valid(cpis[c])) return NDFT_E_INVAL;
    const int pi = batch_plan_choice(cpis, n_cpi, prec);
    const Plan &P = plans(prec)[pi];
    const BatchPlanGeom g = batch_plan_geom(P, prec);
    G.plan = pi;
    G.chunk = (int)(cdiv(chunk > 0 ? chunk : kDefaultChunk, P.kgran) * P.kgran);
    G.rg = batch_regions(n_cpi);
    G.params.resize(n_cpi);
    G.red.resize(n_cpi);
    G.outoff.resize(n_cpi);
    G.prep.resize(2 * n_cpi);
    G.items.clear();
    std::vector<CpiLayout> lay(n_cpi);
    int64_t total_items = 0;
    for (int c = 0; c < n_cpi; ++c) {
        if (!cpi_layout(cpis[c], g, G.chunk, lay[c])) return NDFT_E_UNSUPPORTED; // table beyond the LDS
        total_items += lay[c].items;
    }
    if (total_items >= (int64_t)1 << 30) return NDFT_E_INVAL;
    size_t off = balign(G.rg.items + sizeof(int4) * (size_t)total_items);
    std::vector<long long> cost;
    unsigned *absmax = base ? reinterpret_cast<unsigned *>(base + G.rg.absmax) : nullptr;
    for (int c = 0; c < n_cpi; ++c) {
        const ndft_cpi &d = cpis[c];
        CpiLayout &o = lay[c];
        G.table_bytes = std::max(G.table_bytes, o.table_bytes);
        const size_t s4_off = off, r4_off = off + o.s4_bytes, part_off = off + o.s4_bytes + o.r4_bytes;
        off = part_off + o.part_bytes;
        float4 *s4 = base ? reinterpret_cast<float4 *>(base + s4_off) : nullptr;
        float4 *r4 = base ? reinterpret_cast<float4 *>(base + r4_off) : nullptr;
        float4 *part = base ? reinterpret_cast<float4 *>(base + part_off) : nullptr;
        o.C.s4 = s4;
        o.C.r4 = r4;
        o.C.partial = part;
        o.C.absmax = g.fp8 && absmax ? absmax + 2 * c : nullptr;
        o.R.partial = part;
        G.params[c] = o.C;
        G.red[c] = o.R;
        G.outoff[c] = (long long)d.out_off;
        G.prep[2 * c] = PrepDesc{(long long)d.surv_off, s4, (int)d.n, 0, (long long)(d.n + kTailPad), P.sign_scale,
                                 g.fp8 && absmax ? absmax + 2 * c : nullptr};
        G.prep[2 * c + 1] = PrepDesc{(long long)d.ref_off, r4, (int)d.n, (int)d.n, (long long)(2 * d.n + kTailPad),
                                     P.sign_scale, g.fp8 && absmax ? absmax + 2 * c + 1 : nullptr};
        G.max_prep_blocks = std::max(G.max_prep_blocks, (int)std::min<int64_t>(cdiv(2 * d.n + kTailPad, 256), 1024));
        G.max_red_blocks =
            std::max(G.max_red_blocks, (int)std::min<int64_t>(cdiv((int64_t)o.C.n_cols * o.C.n_bases, 256), 4096));
        for (int tl = 0; tl < o.C.tiles_l; ++tl)
            for (int tbi = 0; tbi < o.C.tiles_b; ++tbi)
                for (int kc = 0; kc < o.C.ksplit; ++kc) {
                    G.items.push_back(make_int4(c, tbi, tl, kc));
                    cost.push_back(std::min<long long>(G.chunk, d.n - (long long)kc * G.chunk));
                }
    }
    // longest chunks first (stable, so equal items keep their surface order)
    std::vector<size_t> order(G.items.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<int4> sorted(G.items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = G.items[order[k]];
    G.items.swap(sorted);
    G.total = off;
    return NDFT_OK;
}

// The plan of a device-planned batch (descriptors unknown on the host): the override if it
// has a batched kernel, else the least cost on a representative CPI (N = 8192, 256
// delays, bins -512..511).
int dev_batch_plan(int prec)
{
    const ndft_cpi rep = {8192, 0, 0, 0, 0, 256, -512, 1024};
    return batch_plan_choice(&rep, 1, prec);
}

std::atomic<unsigned long long> g_batch_seq{0};

// ------------------------------------------------------------------------------------
// static scratch of the no-allocation surface entry point
// ------------------------------------------------------------------------------------
// Each device that loads the library holds one copy until the process ends. Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) char scratch[NDFT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the scratch address on device `dev` (nullptr on failure)
void *scratch_on(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
    return ptr;
}

// ------------------------------------------------------------------------------------
// tables of the fast exact transform, kept per device and length
// ------------------------------------------------------------------------------------
// The tables (group order, its inverse, the correlation spectra) depend on the length
// alone. Each device holds one slot per length 2^lg (lg = 3 .. 12) in a file-scope array,
// filled by the first call of that length outside stream capture, which waits for its
// stream so that the slot is complete before any stream reads it; slots are never written
// again. Under capture, a length not yet cached makes its tables in the call's workspace.
constexpr size_t align256c(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t fast_slot_bytes(int lg)
{
    return 2 * align256c(((size_t)1 << lg) / 2 * sizeof(int)) +
           align256c((size_t)std::max(1, fast_spec_entries(1 << lg)) * sizeof(float2));
}
constexpr size_t fast_slot_off(int lg)
{
    size_t o = 0;
    for (int l = 3; l < lg; ++l) o += fast_slot_bytes(l);
    return o;
}
constexpr size_t kFastCacheBytes = fast_slot_off(kFastLgMax + 1);
static_assert((1 << 3) == kFastMinN, "the first slot is the shortest length");
static __device__ __align__(256) char fast_cache[kFastCacheBytes];

std::mutex g_fast_mu;
void *g_fast_cache_ptr[kMaxDevices] = {};
std::atomic<unsigned> g_fast_valid[kMaxDevices];

void fast_tables_launch(char *base, int n, int lg, hipStream_t s)
{
    int *gtab = reinterpret_cast<int *>(base);
    int *dlog = reinterpret_cast<int *>(base + align256((size_t)(n / 2) * sizeof(int)));
    float2 *spec = reinterpret_cast<float2 *>(base + 2 * align256((size_t)(n / 2) * sizeof(int)));
    const int nspec = lg >= 6 ? 2 * (lg - 5) : 0;
    hipLaunchKernelGGL(fast_tables_kernel, dim3((unsigned)(nspec + 1)), dim3(kFastTabThreads), 0, s, n, lg, gtab,
                       dlog, spec);
}

// the device's cached tables of length 2^lg (nullptr: not available, the call makes its own)
char *fast_cached_tables(int lg, hipStream_t s)
{
    int dev = -1;
    if (s ? hipStreamGetDevice(s, &dev) != hipSuccess : hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices || lg < 3 || lg > kFastLgMax) return nullptr;
    const unsigned bit = 1u << lg;
    if ((g_fast_valid[dev].load(std::memory_order_acquire) & bit) && g_fast_cache_ptr[dev])
        return static_cast<char *>(g_fast_cache_ptr[dev]) + fast_slot_off(lg);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (cs != hipStreamCaptureStatusNone) return nullptr;
    std::lock_guard<std::mutex> lk(g_fast_mu);
    if (!g_fast_cache_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return nullptr;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(fast_cache));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_fast_cache_ptr[dev] = ptr;
    }
    char *base = static_cast<char *>(g_fast_cache_ptr[dev]) + fast_slot_off(lg);
    if (!(g_fast_valid[dev].load(std::memory_order_acquire) & bit)) {
        fast_tables_launch(base, 1 << lg, lg, s);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return nullptr;
        g_fast_valid[dev].fetch_or(bit, std::memory_order_release);
    }
    return base;
}

} // namespace

// ======================================================================================
// C ABI
// ======================================================================================
extern "C" {

const char *ndft_status_string(ndft_status st)
{
    switch (st) {
    case NDFT_OK: return "NDFT_OK";
    case NDFT_E_INVAL: return "NDFT_E_INVAL: invalid argument";
    case NDFT_E_UNSUPPORTED: return "NDFT_E_UNSUPPORTED: precision or shape not supported";
    case NDFT_E_WORKSPACE: return "NDFT_E_WORKSPACE: workspace missing, misaligned or too small";
    case NDFT_E_HIP: return "NDFT_E_HIP: HIP runtime error";
    }
    return "NDFT: unknown status";
}

const char *ndft_version(void) { return "ndft-mi355x 0.1 (gfx950)"; }

// The fast exact transform: the call's tables (group order, its inverse, the correlation
// spectra), then one work-group per row at a time, every bin of the row in LDS and the
// requested ones written out.
ndft_status launch_fast(const Launch &L, int mode, const float2 *x, const float2 *surv, const float2 *ref,
                        int64_t n, int64_t rows, int64_t tau0, int64_t p0, int64_t n_bins, float2 *out, void *ws,
                        hipStream_t s)
{
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    int lg = 0;
    while ((1LL << lg) < n) ++lg;
    char *base = fast_cached_tables(lg, s);
    if (!base) { // capture of a length not yet cached: the call's own tables in its workspace
        base = static_cast<char *>(ws);
        fast_tables_launch(base, (int)n, lg, s);
        const ndft_status st = check_launch();
        if (st != NDFT_OK) return st;
    }
    int *gtab = reinterpret_cast<int *>(base);
    int *dlog = reinterpret_cast<int *>(base + align256((size_t)(n / 2) * sizeof(int)));
    float2 *spec = reinterpret_cast<float2 *>(base + 2 * align256((size_t)(n / 2) * sizeof(int)));
    FastParams P;
    std::memset(&P, 0, sizeof(P));
    P.n = (int)n;
    P.lg = lg;
    P.rows = (int)rows;
    P.x = x;
    P.s = surv;
    P.r = ref;
    P.tau0 = (int)tau0;
    P.gtab = gtab;
    P.dlog = dlog;
    P.spec = spec;
    P.tb = L.tb;
    P.n_coarse = L.n_coarse;
    P.p0n = (int)mod_n(p0, n);
    P.n_dop = (int)n_bins;
    P.out = out;
    const int lds = fast_lds_bytes((int)n, L.n_coarse + (1 << L.tb));
    const int64_t per_cu = std::max(1, (160 * 1024) / lds);
    const unsigned grid = (unsigned)std::min<int64_t>(rows, per_cu * device_cu_count());
    ProfScope prof(s);
    if (mode == FAST_X)
        hipLaunchKernelGGL(fast_ndft_kernel<FAST_X>, dim3(grid), dim3(kFastThreads), (size_t)lds, s, P);
    else if (mode == FAST_LAG)
        hipLaunchKernelGGL(fast_ndft_kernel<FAST_LAG>, dim3(grid), dim3(kFastThreads), (size_t)lds, s, P);
    else
        hipLaunchKernelGGL(fast_ndft_kernel<FAST_LIN>, dim3(grid), dim3(kFastThreads), (size_t)lds, s, P);
    prof.stop();
    return check_launch();
}

size_t ndft_forward_workspace(int64_t batch, int64_t n, int64_t k0, int64_t k_count, ndft_prec prec)
{
    if (!prec_ok(prec) || n < 1 || n > NDFT_MAX_N || batch < 1 || k_count < 1 || k_count > n) return 0;
    const Launch L = plan_launch((int)prec, PROD_IDENTITY, n, batch, k0, k_count, batch * (n + kTailPad));
    return L.plan && L.fits ? L.ws_bytes : 0;
}

ndft_status ndft_forward(const ndft_c64 *x, ndft_c64 *X, int64_t batch, int64_t n, int64_t k0, int64_t k_count,
                         ndft_prec prec, void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || n > NDFT_MAX_N || batch < 0 || k_count < 1 || k_count > n) return NDFT_E_INVAL;
    if (batch > 0 && (!x || !X || !aligned(x, 8) || !aligned(X, 8))) return NDFT_E_INVAL;
    if (batch * n > ((int64_t)1 << 40)) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    if (batch == 0) return NDFT_OK;
    if (batch > INT32_MAX / 2) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, PROD_IDENTITY, n, batch, k0, k_count, batch * (n + kTailPad));
    if (!L.plan || !L.fits) return NDFT_E_UNSUPPORTED; // decided before anything is enqueued
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (L.plan->fastx)
        return launch_fast(L, FAST_X, reinterpret_cast<const float2 *>(x), nullptr, nullptr, n, batch, 0, k0, k_count,
                           reinterpret_cast<float2 *>(X), ws, s);
    float4 *part = reinterpret_cast<float4 *>(ws);
    float4 *x4 = reinterpret_cast<float4 *>(static_cast<char *>(ws) + L.part_bytes);
    st = launch_prep(reinterpret_cast<const float2 *>(x), x4, n, batch, n + kTailPad, 0, L.plan->sign_scale, s);
    if (st != NDFT_OK) return st;
    unsigned *amax = L.absmax_off ? reinterpret_cast<unsigned *>(static_cast<char *>(ws) + L.absmax_off) : nullptr;
    if (amax && (st = launch_absmax(amax, reinterpret_cast<const float2 *>(x), batch * n, nullptr, 0, s)) != NDFT_OK)
        return st;
    st = launch_contract(L, PROD_IDENTITY, x4, nullptr, n + kTailPad, n, batch, 0, part, s, nullptr, nullptr, nullptr,
                         amax);
    if (st != NDFT_OK) return st;
    return launch_reduce(L, part, n, batch, k0, k_count, reinterpret_cast<float2 *>(X), s);
}

// The FP32 sign-split plans after lsum_kernel: the twiddle half as an FFT of the exact lag
// signs (src DFT_SIGNS / DFT_LIN_SIGNS). The whole-row kernel reads the sign codes and adds
// the twiddle-sign half's planes to its bins, writing A once; otherwise the reduction writes
// that half into A and the FFT adds to it.
ndft_status launch_fft_half(const Launch &L, const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                            int64_t n_tau, int64_t p0, int64_t n_dop, ndft_c64 *A, void *ws, int src, hipStream_t s)
{
    const float4 *part = reinterpret_cast<const float4 *>(ws);
    const uint32_t *codes = reinterpret_cast<const uint32_t *>(static_cast<const char *>(ws) + L.code_off);
    TsumParams T;
    std::memset(&T, 0, sizeof(T));
    if (L.dft.fast) {
        T.part = part; // the fft_d plans have no matrix planes: lsum_kernel's come first
        T.ksplit = L.ksplit + L.ksT;
        T.cols_pad = L.n_cols_pad;
        T.bases_pad = L.n_bases_pad;
        T.bm = L.bm;
    } else {
        ndft_status st = launch_reduce(L, part, n, n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), s);
        if (st != NDFT_OK) return st;
    }
    return launch_dft(L.dft, reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), n, tau0,
                      n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), static_cast<char *>(ws) + L.dft_off, src, true,
                      s, codes, L.k_codes / 8, L.code_bytes, L.dft.fast ? &T : nullptr);
}

size_t ndft_caf_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop, ndft_prec prec)
{
    if (!prec_ok(prec) || !caf_args_ok(n, tau0, n_tau, n_dop)) return 0;
    const Launch L = plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad);
    return L.plan && L.fits ? L.ws_bytes : 0;
}

ndft_status ndft_caf(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                     int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec, void *ws, size_t ws_bytes,
                     void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !A || !aligned(surv, 8) || !aligned(ref, 8) || !aligned(A, 8)) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad);
    if (!L.plan || !L.fits) return NDFT_E_UNSUPPORTED; // decided before anything is enqueued
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (L.plan->fastx)
        return launch_fast(L, FAST_LAG, nullptr, reinterpret_cast<const float2 *>(surv),
                           reinterpret_cast<const float2 *>(ref), n, n_tau, tau0, p0, n_dop,
                           reinterpret_cast<float2 *>(A), ws, s);
    float4 *part = reinterpret_cast<float4 *>(ws);
    float4 *s4 = reinterpret_cast<float4 *>(static_cast<char *>(ws) + L.part_bytes);
    float4 *r4 = s4 + n + kTailPad; // n zeros, then the reference, then a zero tail
    if (!L.plan->raw_inputs) {
        const float g = L.plan->sign_scale;
        st = launch_prep_pair(reinterpret_cast<const float2 *>(surv), s4, n + kTailPad,
                              reinterpret_cast<const float2 *>(ref), r4, 2 * n + kTailPad, n, n, g, s);
        if (st != NDFT_OK) return st;
    }
    if (L.plan->lag_kfn) {
        st = launch_split(L, reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), n, n_tau,
                          tau0, part, ws, s);
        if (st == NDFT_OK && L.plan->fft_d) return launch_fft_half(L, surv, ref, n, tau0, n_tau, p0, n_dop, A, ws,
                                                                   DFT_SIGNS, s);
    } else {
        uint4 *planes =
            L.plan->planes_kfn ? reinterpret_cast<uint4 *>(static_cast<char *>(ws) + L.plane_off) : nullptr;
        unsigned *amax = L.absmax_off ? reinterpret_cast<unsigned *>(static_cast<char *>(ws) + L.absmax_off) : nullptr;
        if (amax && (st = launch_absmax(amax, reinterpret_cast<const float2 *>(surv), n,
                                        reinterpret_cast<const float2 *>(ref), n, s)) != NDFT_OK)
            return st;
        st = launch_contract(L, PROD_LAG, s4, r4, 0, n, n_tau, tau0, part, s, planes,
                             reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), amax);
    }
    if (st != NDFT_OK) return st;
    return launch_reduce(L, part, n, n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), s);
}

ndft_status ndft_caf_noalloc(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                             int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec, void *stream)
{
    // the checks of ndft_caf, then the workspace against the scratch size, all before
    // anything is enqueued
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !A || !aligned(surv, 8) || !aligned(ref, 8) || !aligned(A, 8)) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    const Launch L = plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad);
    if (!L.plan || !L.fits) return NDFT_E_UNSUPPORTED;
    if (L.ws_bytes > NDFT_NOALLOC_SCRATCH_BYTES) return NDFT_E_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = -1;
    if (s ? hipStreamGetDevice(s, &dev) != hipSuccess : hipGetDevice(&dev) != hipSuccess) return NDFT_E_HIP;
    void *ws = scratch_on(dev);
    if (!ws) return NDFT_E_HIP;
    t_no_prof = true;
    const ndft_status st = ndft_caf(surv, ref, n, tau0, n_tau, p0, n_dop, A, prec, ws, NDFT_NOALLOC_SCRATCH_BYTES, stream);
    t_no_prof = false;
    return st;
}

size_t ndft_caf12c_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop, ndft_prec prec)
{
    if (!prec_ok(prec) || !caf_args_ok(n, tau0, n_tau, n_dop)) return 0;
    Launch L = plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 0, true);
    return L.plan && L.fits ? L.ws_bytes : 0;
}

ndft_status ndft_caf12c(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                        int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec, void *ws, size_t ws_bytes,
                        void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !A || !aligned(surv, 8) || !aligned(ref, 8) || !aligned(A, 8)) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 0, true);
    if (!L.plan || !L.fits) return NDFT_E_UNSUPPORTED;
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (L.plan->fastx)
        return launch_fast(L, FAST_LIN, nullptr, reinterpret_cast<const float2 *>(surv),
                           reinterpret_cast<const float2 *>(ref), n, n_tau, tau0, p0, n_dop,
                           reinterpret_cast<float2 *>(A), ws, s);
    float4 *part = reinterpret_cast<float4 *>(ws);
    st = launch_split(L, reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), n, n_tau,
                      tau0, part, ws, s);
    if (st != NDFT_OK) return st;
    // FP32: the twiddle half by FFT of the exact signs of the ordinary lag products
    if (L.plan->fft_d) return launch_fft_half(L, surv, ref, n, tau0, n_tau, p0, n_dop, A, ws, DFT_LIN_SIGNS, s);
    return launch_reduce(L, part, n, n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), s);
}

size_t ndft_caf12b_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop, ndft_prec prec)
{
    if (prec != NDFT_FP32 || !caf_args_ok(n, tau0, n_tau, n_dop)) return 0;
    return plan_dft12b(n, n_tau, n_dop).ws_bytes;
}

ndft_status ndft_caf12b(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                        int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec, void *ws, size_t ws_bytes,
                        void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !A || !aligned(surv, 8) || !aligned(ref, 8) || !aligned(A, 8)) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    if (prec != NDFT_FP32) return NDFT_E_UNSUPPORTED;
    const Dft12bLaunch L = plan_dft12b(n, n_tau, n_dop);
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    return launch_dft(L, reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), n, tau0,
                      n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), ws, DFT_LAG, false,
                      reinterpret_cast<hipStream_t>(stream));
}

size_t ndft_nfft_workspace(int64_t batch, int64_t n)
{
    if (n < 1 || n > kNfftMaxLong || (n & (n - 1)) != 0 || batch < 0) return 0;
    if (n <= kNfftMaxN || batch == 0) return 0;
    // ping-pong rows for the top levels, then their twiddles, a table per level (n - 8192)
    return align256((size_t)batch * n * sizeof(float2)) + align256((size_t)(n - kNfftMaxN) * sizeof(float2));
}

ndft_status ndft_nfft(const ndft_c64 *x, ndft_c64 *X, int64_t batch, int64_t n, int32_t reading, void *ws,
                      size_t ws_bytes, void *stream)
{
    if (n < 1 || n > kNfftMaxLong || (n & (n - 1)) != 0 || batch < 0) return NDFT_E_INVAL;
    if (reading != NDFT_NFFT_EVERY_BUTTERFLY && reading != NDFT_NFFT_PRINTED) return NDFT_E_INVAL;
    if (batch == 0) return NDFT_OK;
    if (!x || !X || !aligned(x, 8) || !aligned(X, 8)) return NDFT_E_INVAL;
    if (batch * n > ((int64_t)1 << 40)) return NDFT_E_INVAL;
    const size_t need = ndft_nfft_workspace(batch, n);
    ndft_status st = ws_ok(ws, ws_bytes, need);
    if (st != NDFT_OK) return st;
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        for (const void *fn : {reinterpret_cast<const void *>(&nfft_kernel<false>),
                               reinterpret_cast<const void *>(&nfft_kernel<true>)}) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(kNfftMaxN + kNfftMaxN / 8 + kNfftMaxN) * (int)sizeof(float2));
            if (e != hipSuccess && attr == hipSuccess) attr = e;
        }
    });
    if (attr != hipSuccess) return NDFT_E_HIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool outer = reading == NDFT_NFFT_PRINTED;
    const float2 *xin = reinterpret_cast<const float2 *>(x);
    float2 *Xo = reinterpret_cast<float2 *>(X);
    // rows of up to 8192 samples: in LDS, 8192 / L rows per work-group at a time; longer
    // rows: their 2^lev decimated sequences of 8192 samples in LDS, then lev top levels
    int lev = 0;
    while ((kNfftMaxN << lev) < n) ++lev;
    const int L = (int)std::min<int64_t>(n, kNfftMaxN);
    const int sub = 1 << lev;
    const long long rows = (long long)batch * sub;
    float2 *buf = need ? static_cast<float2 *>(ws) : nullptr;
    float2 *tw = need ? reinterpret_cast<float2 *>(static_cast<char *>(ws) + align256((size_t)batch * n * sizeof(float2)))
                      : nullptr;
    // the top levels go two per pass over global memory (one more for an odd count); the
    // last pass writes X: the LDS stage writes X after an even number of passes
    const int passes = (lev + 1) / 2;
    float2 *first = (passes % 2 == 0) ? Xo : buf;
    const int rpb = kNfftMaxN / L;
    // padded rows (one entry per 8 more), then the per-level twiddle table (L - 1 entries)
    const size_t shmem = ((size_t)rpb * L + (size_t)rpb * L / 8 + L) * sizeof(float2);
    // as many work-groups as fit on the device at once (160 KB of LDS per compute unit),
    // each looping over row groups: the twiddle table is built once per work-group
    const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)shmem);
    const int64_t grid = std::min<int64_t>(cdiv(rows, rpb), per_cu * device_cu_count());
    ProfScope prof(s);
    if (outer)
        hipLaunchKernelGGL(nfft_kernel<true>, dim3((unsigned)grid), dim3(kNfftThreads), shmem, s, xin, first, rows, L,
                           rpb, sub, (long long)n);
    else
        hipLaunchKernelGGL(nfft_kernel<false>, dim3((unsigned)grid), dim3(kNfftThreads), shmem, s, xin, first, rows,
                           L, rpb, sub, (long long)n);
    if ((st = check_launch()) != NDFT_OK) return st;
    if (lev > 0) {
        hipLaunchKernelGGL(nfft_table_kernel, dim3((unsigned)cdiv(n - kNfftMaxN, 256)), dim3(256), 0, s, tw, (int)n);
        const unsigned cgrid = (unsigned)std::min<int64_t>(cdiv(batch * (n / 2), 256), 8LL * device_cu_count());
        const unsigned cgrid2 = (unsigned)std::min<int64_t>(cdiv(batch * (n / 4), 256), 8LL * device_cu_count());
        float2 *src = first;
        for (int S = sub / 2; S >= 1;) { // the level of stride S, inputs at stride 2 S
            float2 *dst = src == Xo ? buf : Xo;
            if (S >= 2) { // levels S and S / 2 in one pass
                if (outer)
                    hipLaunchKernelGGL(nfft_combine2_kernel<true>, dim3(cgrid2), dim3(256), 0, s, src, dst, tw,
                                       (long long)batch, (int)n, S / 2);
                else
                    hipLaunchKernelGGL(nfft_combine2_kernel<false>, dim3(cgrid2), dim3(256), 0, s, src, dst, tw,
                                       (long long)batch, (int)n, S / 2);
                S /= 4;
            } else {
                if (outer)
                    hipLaunchKernelGGL(nfft_combine_kernel<true>, dim3(cgrid), dim3(256), 0, s, src, dst, tw,
                                       (long long)batch, (int)n, S);
                else
                    hipLaunchKernelGGL(nfft_combine_kernel<false>, dim3(cgrid), dim3(256), 0, s, src, dst, tw,
                                       (long long)batch, (int)n, S);
                S /= 2;
            }
            src = dst;
        }
    }
    prof.stop();
    return check_launch();
}

ndft_status ndft_dbg_signs(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                           int64_t p0, int64_t n_dop, int8_t *tw_sign, int8_t *lag_sign, void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (lag_sign && (!surv || !ref || !aligned(surv, 8) || !aligned(ref, 8))) return NDFT_E_INVAL;
    int64_t ntw = tw_sign ? n_dop * n : 0;
    int64_t nlag = lag_sign ? n_tau * n : 0;
    if (ntw + nlag == 0) return NDFT_OK;
    if (ntw + nlag > ((int64_t)1 << 40)) return NDFT_E_INVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(dbg_signs_kernel, dim3((unsigned)cdiv(ntw + nlag, 256)), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), (int)n,
                       (int)tau0, (int)mod_n(p0, n), ntw, nlag, tw_sign, lag_sign);
    return check_launch();
}

int32_t ndft_dbg_fast_tables(int32_t reset)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return -1;
    }
    std::lock_guard<std::mutex> lk(g_fast_mu);
    const unsigned m = g_fast_valid[dev].load(std::memory_order_acquire);
    if (reset) g_fast_valid[dev].store(0, std::memory_order_release);
    return (int32_t)m;
}

ndft_status ndft_dbg_split(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                           int64_t p0, int64_t n_dop, ndft_prec prec, int32_t lin, int8_t *lag_sign, ndft_c64 *T,
                           void *ws, size_t ws_bytes, void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !aligned(surv, 8) || !aligned(ref, 8)) return NDFT_E_INVAL;
    if (T && !aligned(T, 8)) return NDFT_E_INVAL;
    if (!prec_ok(prec) || (lin != 0 && lin != 1)) return NDFT_E_INVAL;
    if (n_tau * n > ((int64_t)1 << 40)) return NDFT_E_INVAL;
    // the plan the surface entry point would take for these arguments
    Launch L = lin ? plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 0, true)
                   : plan_launch((int)prec, PROD_LAG, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad);
    if (!L.plan || !L.fits || !L.plan->lag_kfn) return NDFT_E_UNSUPPORTED;
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float4 *part = reinterpret_cast<float4 *>(ws);
    st = launch_split(L, reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), n, n_tau,
                      tau0, part, ws, s, true);
    if (st != NDFT_OK) return st;
    if (lag_sign) {
        const uint32_t *codes = reinterpret_cast<const uint32_t *>(static_cast<const char *>(ws) + L.code_off);
        const long long total = (long long)n_tau * n;
        hipLaunchKernelGGL(dbg_decode_codes_kernel, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, codes,
                           L.n_cols_pad, (int)n, total, lag_sign, L.plan->fft_d ? 1 : 0, L.k_codes / 8);
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    if (!T) return NDFT_OK;
    // the lag kernel's partial planes alone: the twiddle-sign half (and base 0 whole)
    Launch LT = L;
    LT.ksplit = 0;
    return launch_reduce(LT, part + (size_t)L.ksplit * L.n_cols_pad * L.n_bases_pad, n, n_tau, p0, n_dop,
                         reinterpret_cast<float2 *>(T), s);
}

size_t ndft_caf_backward_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop,
                                   ndft_prec prec)
{
    if (!prec_ok(prec) || !caf_args_ok(n, tau0, n_tau, n_dop)) return 0;
    return plan_adjoint(n, n_tau, p0, n_dop).ws_bytes;
}

ndft_status ndft_caf_backward(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                              int64_t p0, int64_t n_dop, const ndft_c64 *grad_A, ndft_c64 *grad_ref,
                              ndft_c64 *grad_surv, ndft_prec prec, void *ws, size_t ws_bytes, void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !grad_A || !grad_ref) return NDFT_E_INVAL;
    if (!aligned(surv, 8) || !aligned(ref, 8) || !aligned(grad_A, 8) || !aligned(grad_ref, 8)) return NDFT_E_INVAL;
    if (grad_surv && !aligned(grad_surv, 8)) return NDFT_E_INVAL;
    if (prec == NDFT_FP8) return NDFT_E_UNSUPPORTED;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    AdjLaunch L = plan_adjoint(n, n_tau, p0, n_dop);
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float4 *eo = reinterpret_cast<float4 *>(ws);
    float2 *dz = reinterpret_cast<float2 *>(static_cast<char *>(ws) + L.eo_bytes);
    int64_t neo = (int64_t)L.n_bases_pad * n_tau;
    hipLaunchKernelGGL(adj_prep_kernel, dim3((unsigned)cdiv(neo, 256)), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(grad_A), (int)n_tau, (int)n_dop, (int)n, (int)mod_n(p0, n),
                       L.bm, L.n_bases, L.n_bases_pad, eo);
    if ((st = check_launch()) != NDFT_OK) return st;
    AdjParams P;
    std::memset(&P, 0, sizeof(P));
    P.eo = eo;
    P.bm = L.bm;
    P.n = (int)n;
    P.n_tau = (int)n_tau;
    P.n_bases_pad = L.n_bases_pad;
    P.inv_n = 1.0 / (double)n;
    P.dz = dz;
    dim3 grid((unsigned)(cdiv(n_tau, 64) * cdiv(n, 64)));
    {
        ProfScope prof(s);
        if (prec == NDFT_BF16X2)
            hipLaunchKernelGGL(adj_contract_kernel<PREC_BF16X2>, grid, dim3(256), 0, s, P);
        else
            hipLaunchKernelGGL(adj_contract_kernel<PREC_FP32>, grid, dim3(256), 0, s, P);
        prof.stop();
    }
    if ((st = check_launch()) != NDFT_OK) return st;
    hipLaunchKernelGGL(adj_band_kernel, dim3((unsigned)cdiv(n, kAdjBandOut)), dim3(kAdjBandOut * kAdjBandGroups), 0, s, dz,
                       reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), (int)n,
                       (int)tau0, (int)n_tau, reinterpret_cast<float2 *>(grad_ref),
                       reinterpret_cast<float2 *>(grad_surv));
    return check_launch();
}

size_t ndft_caf_batched_workspace(const ndft_cpi *cpis, int32_t n_cpi, ndft_prec prec, int32_t chunk)
{
    if (!prec_ok(prec)) return 0;
    BatchGeom G;
    if (batch_geometry(cpis, n_cpi, (int)prec, chunk, nullptr, G) != NDFT_OK) return 0;
    return G.total;
}

ndft_status ndft_caf_batched_prepare(const ndft_cpi *cpis, int32_t n_cpi, ndft_prec prec, int32_t chunk, void *ws,
                                     size_t ws_bytes, ndft_batch *batch)
{
    if (!batch) return NDFT_E_INVAL;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    BatchGeom G;
    ndft_status st = batch_geometry(cpis, n_cpi, (int)prec, chunk, static_cast<char *>(ws), G);
    if (st != NDFT_OK) return st;
    if ((st = ws_ok(ws, ws_bytes, G.total)) != NDFT_OK) return st;
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    const Plan &P = plans((int)prec)[G.plan];
    if (G.table_bytes > plan_max_dynamic(P)) return NDFT_E_UNSUPPORTED;
    unsigned long long tag = (++g_batch_seq) ^
        ((unsigned long long)std::chrono::steady_clock::now().time_since_epoch().count() << 20);
    // host image of the tables (header .. items), copied in one blocking transfer
    std::vector<char> img(G.rg.items + sizeof(int4) * G.items.size(), 0);
    BatchHeader hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    hdr.counter = 0;
    hdr.n_items = (int)G.items.size();
    hdr.n_cpi = n_cpi;
    hdr.plan_id = (int)prec * 100 + G.plan;
    hdr.tag = tag;
    hdr.status = 0;
    std::memcpy(img.data(), &hdr, sizeof(hdr));
    std::memcpy(img.data() + G.rg.params, G.params.data(), sizeof(ContractParams) * n_cpi);
    std::memcpy(img.data() + G.rg.red, G.red.data(), sizeof(ReduceParams) * n_cpi);
    std::memcpy(img.data() + G.rg.outoff, G.outoff.data(), sizeof(long long) * n_cpi);
    std::memcpy(img.data() + G.rg.prep, G.prep.data(), sizeof(PrepDesc) * 2 * n_cpi);
    std::memcpy(img.data() + G.rg.items, G.items.data(), sizeof(int4) * G.items.size());
    if (hipMemcpy(ws, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) return NDFT_E_HIP;
    std::memset(batch, 0, sizeof(*batch));
    batch->prec = (int32_t)prec;
    batch->plan = G.plan;
    batch->n_cpi = n_cpi;
    batch->n_items = (int32_t)G.items.size();
    batch->grid = device_cu_count();
    batch->table_bytes = G.table_bytes;
    batch->max_red_blocks = G.max_red_blocks;
    batch->max_prep_blocks = G.max_prep_blocks;
    batch->tag = tag;
    batch->ws_bytes = G.total;
    (void)P;
    return NDFT_OK;
}

ndft_status ndft_caf_batched(const ndft_batch *batch, const ndft_c64 *surv_pool, const ndft_c64 *ref_pool,
                             ndft_c64 *out_pool, void *ws, size_t ws_bytes, void *stream)
{
    if (!batch || !surv_pool || !ref_pool || !out_pool) return NDFT_E_INVAL;
    if (!aligned(surv_pool, 8) || !aligned(ref_pool, 8) || !aligned(out_pool, 8)) return NDFT_E_INVAL;
    if (!prec_ok((ndft_prec)batch->prec)) return NDFT_E_INVAL;
    if (batch->plan < 0 || batch->plan >= (int)plans(batch->prec).size() ||
        !plans(batch->prec)[batch->plan].kfn_batched)
        return NDFT_E_INVAL;
    if (batch->n_cpi < 1 || batch->n_cpi > kMaxBatch || batch->grid < 1 || batch->table_bytes < 0 ||
        batch->table_bytes > plan_max_dynamic(plans(batch->prec)[batch->plan]) || batch->max_red_blocks < 1 ||
        batch->max_prep_blocks < 1)
        return NDFT_E_INVAL;
    ndft_status st = ws_ok(ws, ws_bytes, (size_t)batch->ws_bytes);
    if (st != NDFT_OK) return st;
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    char *base = static_cast<char *>(ws);
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(base);
    const BatchRegions rg = batch_regions(batch->n_cpi);
    const ContractParams *params = reinterpret_cast<const ContractParams *>(base + rg.params);
    const ReduceParams *red = reinterpret_cast<const ReduceParams *>(base + rg.red);
    const long long *outoff = reinterpret_cast<const long long *>(base + rg.outoff);
    const PrepDesc *prep = reinterpret_cast<const PrepDesc *>(base + rg.prep);
    unsigned *absmax = reinterpret_cast<unsigned *>(base + rg.absmax);
    const int4 *items = reinterpret_cast<const int4 *>(base + rg.items);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long tag = batch->tag;
    int plan_id = batch->prec * 100 + batch->plan;
    const Plan &P = plans(batch->prec)[batch->plan];
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, s, hdr,
                       batch->prec == NDFT_FP8 ? absmax : nullptr, 2 * batch->n_cpi);
    if ((st = check_launch()) != NDFT_OK) return st;
    const float2 *pool_s = reinterpret_cast<const float2 *>(surv_pool);
    const float2 *pool_r = reinterpret_cast<const float2 *>(ref_pool);
    if (!P.raw_inputs) {
        hipLaunchKernelGGL(prep_batched_kernel, dim3((unsigned)batch->max_prep_blocks, (unsigned)(2 * batch->n_cpi)),
                           dim3(256), 0, s, hdr, prep, pool_s, pool_r, tag);
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    {
        void *args[] = {&hdr, &params, &items, &tag, &plan_id, &pool_s, &pool_r};
        ProfScope prof(s);
        hipError_t e = hipLaunchKernel(P.kfn_batched, dim3((unsigned)batch->grid), dim3((unsigned)P.nt), args,
                                       (size_t)batch->table_bytes, s);
        prof.stop();
        if (e != hipSuccess) return NDFT_E_HIP;
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    hipLaunchKernelGGL(reduce_batched_kernel, dim3((unsigned)batch->max_red_blocks, (unsigned)batch->n_cpi), dim3(256),
                       0, s, hdr, red, outoff, reinterpret_cast<float2 *>(out_pool), tag);
    return check_launch();
}

size_t ndft_caf_batched_dev_workspace(int32_t n_cpi, int64_t max_n, int64_t max_tau, int64_t max_dop, ndft_prec prec)
{
    if (!prec_ok(prec) || n_cpi < 1 || n_cpi > kMaxDevBatch) return 0;
    // every CPI within the maxima takes at most what one CPI at the maxima takes, with
    // all its bins on one side (the most bases)
    const ndft_cpi worst = {max_n, 0, 0, 0, 0, max_tau, 0, std::min<int64_t>(max_dop, max_n / 2 + 1)};
    if (!cpi_valid(worst) || max_dop < 1 || max_dop > max_n) return 0;
    const int pi = dev_batch_plan((int)prec);
    const Plan &P = plans((int)prec)[pi];
    const int chunk = (int)(cdiv(kDefaultChunk, P.kgran) * P.kgran);
    CpiLayout o;
    if (!cpi_layout(worst, batch_plan_geom(P, (int)prec), chunk, o)) return 0;
    const BatchRegions rg = batch_regions(n_cpi);
    const unsigned long long items = (unsigned long long)n_cpi * (unsigned long long)o.items;
    if (items >= (1ULL << 30)) return 0;
    return balign(rg.items + sizeof(int4) * (size_t)items) +
           (size_t)n_cpi * (o.s4_bytes + o.r4_bytes + o.part_bytes);
}

ndft_status ndft_caf_batched_dev(const ndft_c64 *surv_pool, const ndft_c64 *ref_pool, ndft_c64 *out_pool,
                                 const ndft_cpi *cpis_dev, int32_t n_cpi, ndft_prec prec, void *ws, size_t ws_bytes,
                                 void *stream)
{
    if (!surv_pool || !ref_pool || !out_pool || !cpis_dev) return NDFT_E_INVAL;
    if (!aligned(surv_pool, 8) || !aligned(ref_pool, 8) || !aligned(out_pool, 8) || !aligned(cpis_dev, 8))
        return NDFT_E_INVAL;
    if (!prec_ok(prec) || n_cpi < 1 || n_cpi > kMaxDevBatch) return NDFT_E_INVAL;
    const BatchRegions rg = batch_regions(n_cpi);
    ndft_status st = ws_ok(ws, ws_bytes, rg.items);
    if (st != NDFT_OK) return st;
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    const int pi = dev_batch_plan((int)prec);
    const Plan &P = plans((int)prec)[pi];
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DevPlanArgs A;
    A.cpis = cpis_dev;
    A.n_cpi = n_cpi;
    A.g = batch_plan_geom(P, (int)prec);
    A.kgran = P.kgran;
    A.chunk = (int)(cdiv(kDefaultChunk, P.kgran) * P.kgran);
    A.ws = static_cast<char *>(ws);
    A.ws_bytes = ws_bytes;
    A.tag = ((++g_batch_seq) ^ ((unsigned long long)std::chrono::steady_clock::now().time_since_epoch().count() << 20)) |
            1ULL; // never 0 (the planner's "did not run" tag)
    A.plan_id = (int)prec * 100 + pi;
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, A);
    if ((st = check_launch()) != NDFT_OK) return st;
    char *base = static_cast<char *>(ws);
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(base);
    const ContractParams *params = reinterpret_cast<const ContractParams *>(base + rg.params);
    const ReduceParams *red = reinterpret_cast<const ReduceParams *>(base + rg.red);
    const long long *outoff = reinterpret_cast<const long long *>(base + rg.outoff);
    const PrepDesc *prep = reinterpret_cast<const PrepDesc *>(base + rg.prep);
    unsigned *absmax = reinterpret_cast<unsigned *>(base + rg.absmax);
    const int4 *items = reinterpret_cast<const int4 *>(base + rg.items);
    unsigned long long tag = A.tag;
    int plan_id = A.plan_id;
    // the queue counter is set by the planner; the maxima are cleared here (FP8)
    if (prec == NDFT_FP8) {
        hipLaunchKernelGGL(absmax_zero_kernel, dim3(1), dim3(256), 0, s, absmax, 2 * n_cpi);
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    const float2 *pool_s = reinterpret_cast<const float2 *>(surv_pool);
    const float2 *pool_r = reinterpret_cast<const float2 *>(ref_pool);
    if (!P.raw_inputs) {
        hipLaunchKernelGGL(prep_batched_kernel, dim3(64, (unsigned)(2 * n_cpi)), dim3(256), 0, s, hdr, prep, pool_s,
                           pool_r, tag);
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    {
        void *args[] = {&hdr, &params, &items, &tag, &plan_id, &pool_s, &pool_r};
        ProfScope prof(s);
        hipError_t e = hipLaunchKernel(P.kfn_batched, dim3((unsigned)device_cu_count()), dim3((unsigned)P.nt), args,
                                       (size_t)plan_max_dynamic(P), s);
        prof.stop();
        if (e != hipSuccess) return NDFT_E_HIP;
        if ((st = check_launch()) != NDFT_OK) return st;
    }
    hipLaunchKernelGGL(reduce_batched_kernel, dim3(64, (unsigned)n_cpi), dim3(256), 0, s, hdr, red, outoff,
                       reinterpret_cast<float2 *>(out_pool), tag);
    return check_launch();
}

ndft_status ndft_caf_batched_dev_status(const void *ws, int32_t *status, void *stream)
{
    if (!ws || !status || !aligned(ws, 256) || !aligned(status, 4)) return NDFT_E_INVAL;
    hipLaunchKernelGGL(batch_status_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream),
                       static_cast<const BatchHeader *>(ws), reinterpret_cast<int *>(status));
    return check_launch();
}

int32_t ndft_plan_count(ndft_prec prec)
{
    if (!prec_ok(prec)) return 0;
    return (int32_t)plans((int)prec).size();
}

const char *ndft_plan_name(ndft_prec prec, int32_t plan)
{
    if (!prec_ok(prec) || plan < 0 || plan >= ndft_plan_count(prec)) return nullptr;
    return plans((int)prec)[plan].name;
}

ndft_status ndft_set_plan(ndft_prec prec, int32_t plan, int32_t ksplit)
{
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    if (plan >= ndft_plan_count(prec) || plan < -1 || ksplit < 0) return NDFT_E_INVAL;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plan_override[prec] = plan;
    g_ksplit_override[prec] = ksplit;
    return NDFT_OK;
}

ndft_status ndft_get_plan(ndft_prec prec, int64_t n, int64_t n_cols, int64_t p0, int64_t n_bins, int32_t *plan,
                          int32_t *ksplit)
{
    if (!prec_ok(prec) || n < 1 || n > NDFT_MAX_N || n_cols < 1 || n_bins < 1 || n_bins > n) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, PROD_LAG, n, n_cols, p0, n_bins, 0);
    if (plan) *plan = (int32_t)(L.plan - plans((int)prec).data());
    if (ksplit) *ksplit = L.ksplit;
    return NDFT_OK;
}

ndft_status ndft_prof_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return NDFT_OK;
}

ndft_status ndft_prof_read(double *contract_ms, int64_t *launches)
{
    return ndft_prof_read_slot(0, contract_ms, launches);
}

ndft_status ndft_prof_read_slot(int32_t slot, double *ms_sum, int64_t *launches)
{
    if (slot < 0 || slot >= kProfSlots) return NDFT_E_INVAL;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending[slot]);
    }
    double total = 0.0;
    ndft_status st = NDFT_OK;
    for (auto &ev : pend) {
        if (hipEventSynchronize(ev.second) != hipSuccess) st = NDFT_E_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess) st = NDFT_E_HIP;
        total += ms;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto &ev : pend) {
            g_event_pool.push_back(ev.first);
            g_event_pool.push_back(ev.second);
        }
    }
    if (ms_sum) *ms_sum = total;
    if (launches) *launches = (int64_t)pend.size();
    return st;
}

} // extern "C"
