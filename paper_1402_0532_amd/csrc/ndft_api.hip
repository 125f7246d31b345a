// libndft.so: C ABI of the NDFT hot path (declarations and conventions in include/ndft.h).
// Host side: argument validation, base-bin segments, tile plans, workspace layout,
// kernel launches on the caller's stream and optional hipEvent timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "ndft.h"
#include "ndft_backward.hpp"
#include "ndft_contract.hpp"
#include "ndft_debug.hpp"

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
    int static_lds;
    const void *kfn[2]; // [PROD_LAG, PROD_IDENTITY]
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
    p.static_lds = 2 * (Cfg::STAGE_A_F4 + Cfg::STAGE_B_F4) * 16;
    p.kfn[0] = reinterpret_cast<const void *>(&contract_kernel<PREC, PROD_LAG, WAVES_B, WAVES_L, WB, WL, KS>);
    p.kfn[1] = reinterpret_cast<const void *>(&contract_kernel<PREC, PROD_IDENTITY, WAVES_B, WAVES_L, WB, WL, KS>);
    return p;
}

const std::vector<Plan> &plans(int prec)
{
    // name: bases x delays per work-group, waves, samples per stage
    static const std::vector<Plan> f32 = {
        make_plan<PREC_FP32, 2, 4, 2, 1, 8>("fp32_b128_l128_w8_ks8"),
        make_plan<PREC_FP32, 1, 8, 2, 1, 8>("fp32_b64_l256_w8_ks8"),
        make_plan<PREC_FP32, 4, 2, 2, 1, 8>("fp32_b256_l64_w8_ks8"),
        make_plan<PREC_FP32, 3, 4, 1, 1, 8>("fp32_b96_l128_w12_ks8"),
    };
    static const std::vector<Plan> bf16 = {
        make_plan<PREC_BF16X2, 2, 4, 2, 1, 8>("bf16x2_b128_l128_w8_ks8"),
        make_plan<PREC_BF16X2, 1, 8, 2, 1, 8>("bf16x2_b64_l256_w8_ks8"),
        make_plan<PREC_BF16X2, 4, 2, 2, 1, 8>("bf16x2_b256_l64_w8_ks8"),
        make_plan<PREC_BF16X2, 3, 4, 1, 1, 8>("bf16x2_b96_l128_w12_ks8"),
    };
    return prec == NDFT_BF16X2 ? bf16 : f32;
}

std::mutex g_plan_mu;
int g_plan_override[2] = {-1, -1};
int g_ksplit_override[2] = {0, 0};

// Largest twiddle-table size (N = 2^24: 4096 coarse + 4096 fine entries).
constexpr int kMaxTableBytes = 8192 * 8;

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

void set_kernel_attributes()
{
    for (int prec = 0; prec < 2; ++prec)
        for (const Plan &p : plans(prec))
            for (int k = 0; k < 2; ++k) {
                hipError_t e = hipFuncSetAttribute(p.kfn[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   kMaxTableBytes);
                if (e != hipSuccess && g_attr_err == hipSuccess) g_attr_err = e;
            }
}

struct Launch {
    const Plan *plan;
    int prec;
    int ksplit, kchunk;
    int tiles_b, tiles_l;
    int n_bases, n_bases_pad, n_cols_pad;
    int tb, n_coarse;
    BaseMap bm;
    size_t part_bytes; // split-K partials
    size_t ws_bytes;   // partials + signed copies of the inputs
};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int pick_ksplit(int tiles, int64_t n, int ks, int cus)
{
    int max_k = (int)std::max<int64_t>(1, cdiv(n, 8LL * ks)); // at least ~8 stages per chunk
    int best = 1;
    double best_eff = -1.0;
    for (int k = 1; k <= max_k; ++k) {
        int64_t w = (int64_t)tiles * k;
        int64_t waves = cdiv(w, cus);
        double eff = (double)w / (double)(waves * cus);
        if (eff > best_eff + 0.05) {
            best_eff = eff;
            best = k;
        }
        if (best_eff >= 0.9) break;
    }
    return best;
}

Launch plan_launch(int prec, int64_t n, int64_t n_cols, int64_t p0, int64_t n_bins, int64_t signed_elems)
{
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.prec = prec;
    L.bm = make_base_map(n, p0, n_bins, &L.n_bases);
    int pi, ko;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        pi = g_plan_override[prec];
        ko = g_ksplit_override[prec];
    }
    const std::vector<Plan> &ps = plans(prec);
    if (pi < 0 || pi >= (int)ps.size()) {
        // built-in choice: padded matrix-core work plus operand generation (a tile
        // generates one twiddle row per base and one lag column per delay, shared by
        // the other dimension), then the earlier plan
        double best = -1.0;
        pi = 0;
        for (int k = 0; k < (int)ps.size(); ++k) {
            double rows = (double)(cdiv(L.n_bases, ps[k].bt) * ps[k].bt);
            double cols = (double)(cdiv(n_cols, ps[k].lt) * ps[k].lt);
            double cost = rows * cols * (1.0 + 64.0 / ps[k].bt + 64.0 / ps[k].lt);
            if (best < 0 || cost < best * 0.999) {
                best = cost;
                pi = k;
            }
        }
    }
    L.plan = &ps[pi];
    L.tiles_b = (int)cdiv(L.n_bases, L.plan->bt);
    L.tiles_l = (int)cdiv(n_cols, L.plan->lt);
    L.n_bases_pad = L.tiles_b * L.plan->bt;
    L.n_cols_pad = L.tiles_l * L.plan->lt;
    int max_split = (int)std::max<int64_t>(1, cdiv(n, L.plan->ks));
    L.ksplit = ko > 0 ? std::min(ko, max_split) : pick_ksplit(L.tiles_b * L.tiles_l, n, L.plan->ks, device_cu_count());
    L.kchunk = (int)(cdiv(cdiv(n, L.ksplit), L.plan->ks) * L.plan->ks);
    L.ksplit = (int)cdiv(n, L.kchunk); // no empty chunks
    int tb = 0;
    while ((1LL << (2 * tb)) < n) ++tb; // 2^tb >= sqrt(n)
    L.tb = tb;
    L.n_coarse = (int)cdiv(n, 1LL << tb);
    L.part_bytes = align256((size_t)L.ksplit * L.n_cols_pad * L.n_bases_pad * sizeof(float4));
    L.ws_bytes = L.part_bytes + align256((size_t)signed_elems * sizeof(float4));
    return L;
}

// ------------------------------------------------------------------------------------
// profiling events
// ------------------------------------------------------------------------------------
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pending;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit ProfScope(hipStream_t st) : s(st)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on) return;
        a = take_event();
        b = take_event();
        if (a && b) (void)hipEventRecord(a, s);
    }
    void stop()
    {
        if (!(a && b)) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending.push_back({a, b});
        a = b = nullptr;
    }
};

ndft_status check_launch()
{
    return hipGetLastError() == hipSuccess ? NDFT_OK : NDFT_E_HIP;
}

ndft_status launch_prep(const float2 *x, float4 *out, int64_t n, int64_t rows, int64_t ostride, int64_t lead,
                        hipStream_t stream)
{
    int64_t count = rows * ostride;
    if (count == 0) return NDFT_OK;
    hipLaunchKernelGGL(sign_prep_kernel, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, stream, x, out, (int)n,
                       (long long)rows, (long long)ostride, (int)lead);
    return check_launch();
}

ndft_status launch_contract(const Launch &L, int prod, const float4 *s4, const float4 *r4, long long col_stride,
                            int64_t n, int64_t n_cols, int64_t tau0, float4 *partial, hipStream_t stream)
{
    std::call_once(g_attr_once, set_kernel_attributes);
    if (g_attr_err != hipSuccess) return NDFT_E_HIP;
    ContractParams P;
    std::memset(&P, 0, sizeof(P));
    P.s4 = s4;
    P.r4 = r4;
    P.col_stride = col_stride;
    P.n = (int)n;
    P.n_cols = (int)n_cols;
    P.tau0 = (int)tau0;
    P.n_bases = L.n_bases;
    P.bm = L.bm;
    P.tb = L.tb;
    P.n_coarse = L.n_coarse;
    P.kchunk = L.kchunk;
    P.ksplit = L.ksplit;
    P.tiles_b = L.tiles_b;
    P.tiles_l = L.tiles_l;
    P.n_bases_pad = L.n_bases_pad;
    P.n_cols_pad = L.n_cols_pad;
    P.partial = partial;
    void *args[] = {&P};
    size_t shmem = (size_t)(L.n_coarse + (1 << L.tb)) * sizeof(float2);
    dim3 grid((unsigned)((int64_t)L.tiles_b * L.tiles_l * L.ksplit));
    dim3 block((unsigned)L.plan->nt);
    ProfScope prof(stream);
    hipError_t e = hipLaunchKernel(L.plan->kfn[prod], grid, block, args, shmem, stream);
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
    R.ksplit = L.ksplit;
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

bool prec_ok(ndft_prec p) { return p == NDFT_FP32 || p == NDFT_BF16X2; }

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

size_t ndft_forward_workspace(int64_t batch, int64_t n, int64_t k0, int64_t k_count, ndft_prec prec)
{
    if (!prec_ok(prec) || n < 1 || n > NDFT_MAX_N || batch < 1 || k_count < 1 || k_count > n) return 0;
    return plan_launch((int)prec, n, batch, k0, k_count, batch * (n + kTailPad)).ws_bytes;
}

ndft_status ndft_forward(const ndft_c64 *x, ndft_c64 *X, int64_t batch, int64_t n, int64_t k0, int64_t k_count,
                         ndft_prec prec, void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || n > NDFT_MAX_N || batch < 0 || k_count < 1 || k_count > n) return NDFT_E_INVAL;
    if (batch > 0 && (!x || !X || !aligned(x, 8) || !aligned(X, 8))) return NDFT_E_INVAL;
    if (batch * n > ((int64_t)1 << 40)) return NDFT_E_INVAL;
    if (prec == NDFT_FP8) return NDFT_E_UNSUPPORTED;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    if (batch == 0) return NDFT_OK;
    if (batch > INT32_MAX / 2) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, n, batch, k0, k_count, batch * (n + kTailPad));
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float4 *part = reinterpret_cast<float4 *>(ws);
    float4 *x4 = reinterpret_cast<float4 *>(static_cast<char *>(ws) + L.part_bytes);
    st = launch_prep(reinterpret_cast<const float2 *>(x), x4, n, batch, n + kTailPad, 0, s);
    if (st != NDFT_OK) return st;
    st = launch_contract(L, PROD_IDENTITY, x4, nullptr, n + kTailPad, n, batch, 0, part, s);
    if (st != NDFT_OK) return st;
    return launch_reduce(L, part, n, batch, k0, k_count, reinterpret_cast<float2 *>(X), s);
}

size_t ndft_caf_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop, ndft_prec prec)
{
    if (!prec_ok(prec) || !caf_args_ok(n, tau0, n_tau, n_dop)) return 0;
    return plan_launch((int)prec, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad).ws_bytes;
}

ndft_status ndft_caf(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0, int64_t n_tau,
                     int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec, void *ws, size_t ws_bytes,
                     void *stream)
{
    if (!caf_args_ok(n, tau0, n_tau, n_dop)) return NDFT_E_INVAL;
    if (!surv || !ref || !A || !aligned(surv, 8) || !aligned(ref, 8) || !aligned(A, 8)) return NDFT_E_INVAL;
    if (prec == NDFT_FP8) return NDFT_E_UNSUPPORTED;
    if (!prec_ok(prec)) return NDFT_E_INVAL;
    Launch L = plan_launch((int)prec, n, n_tau, p0, n_dop, 3 * n + 2 * kTailPad);
    ndft_status st = ws_ok(ws, ws_bytes, L.ws_bytes);
    if (st != NDFT_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float4 *part = reinterpret_cast<float4 *>(ws);
    float4 *s4 = reinterpret_cast<float4 *>(static_cast<char *>(ws) + L.part_bytes);
    float4 *r4 = s4 + n + kTailPad; // n zeros, then the reference, then a zero tail
    st = launch_prep(reinterpret_cast<const float2 *>(surv), s4, n, 1, n + kTailPad, 0, s);
    if (st == NDFT_OK) st = launch_prep(reinterpret_cast<const float2 *>(ref), r4, n, 1, 2 * n + kTailPad, n, s);
    if (st != NDFT_OK) return st;
    st = launch_contract(L, PROD_LAG, s4, r4, 0, n, n_tau, tau0, part, s);
    if (st != NDFT_OK) return st;
    return launch_reduce(L, part, n, n_tau, p0, n_dop, reinterpret_cast<float2 *>(A), s);
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
    P.dz = dz;
    dim3 grid((unsigned)(cdiv(n_tau, 64) * cdiv(n, 128)));
    {
        ProfScope prof(s);
        if (prec == NDFT_BF16X2)
            hipLaunchKernelGGL(adj_contract_kernel<PREC_BF16X2>, grid, dim3(256), 0, s, P);
        else
            hipLaunchKernelGGL(adj_contract_kernel<PREC_FP32>, grid, dim3(256), 0, s, P);
        prof.stop();
    }
    if ((st = check_launch()) != NDFT_OK) return st;
    hipLaunchKernelGGL(adj_band_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, dz,
                       reinterpret_cast<const float2 *>(surv), reinterpret_cast<const float2 *>(ref), (int)n,
                       (int)tau0, (int)n_tau, reinterpret_cast<float2 *>(grad_ref),
                       reinterpret_cast<float2 *>(grad_surv));
    return check_launch();
}

size_t ndft_caf_batched_workspace(const ndft_cpi *, int32_t, ndft_prec) { return 0; }

ndft_status ndft_caf_batched_prepare(const ndft_cpi *, int32_t, ndft_prec, void *, size_t)
{
    return NDFT_E_UNSUPPORTED;
}

ndft_status ndft_caf_batched(const ndft_c64 *, const ndft_c64 *, ndft_c64 *, ndft_prec, void *, size_t, void *)
{
    return NDFT_E_UNSUPPORTED;
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
    Launch L = plan_launch((int)prec, n, n_cols, p0, n_bins, 0);
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
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending);
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
    if (contract_ms) *contract_ms = total;
    if (launches) *launches = (int64_t)pend.size();
    return st;
}

} // extern "C"
