/*
 * ndft.h -- C ABI of libndft.so: the multiplication-free nonlinear DFT (NDFT) and the
 * NDFT cross-ambiguity surface on AMD Instinct MI355X (gfx950).
 *
 * Method: Bozkurt, Arslan, Sevimli, Akbas, Cetin, "Approximate Computation of DFT
 * without Performing Any Multiplications: Applications to Radar Signal Processing"
 * (arXiv 1402.0532).
 *
 *   a (x) b = sign(a*b)(|a| + |b|), 0 when either operand is 0        -- Eq. (1)-(2)
 *   complex:  a (x) b = a_r(x)b_r - a_i(x)b_i + j(a_i(x)b_r + b_i(x)a_r) -- Eq. (6)
 *   NDFT:     X[k] = sum_n W^{kn mod N} (x) x[n],  W = e^{-j 2 pi / N}  -- Eq. (7)
 *   surface:  A[l][p] = sum_i (s[i] (x) conj(r[i-d])) (x) W^{ip}        -- Eq. (12a)
 *
 * Conventions shared by every entry point:
 *   - Complex data is complex64: interleaved {re, im} float pairs (ndft_c64), the
 *     layout of torch.complex64 and std::complex<float>.
 *   - All data pointers are DEVICE pointers owned by the caller. The library allocates
 *     no device memory: scratch space comes from the caller as `ws` (size from the
 *     matching *_workspace query; a NULL ws is allowed when the query returns 0).
 *     Pointers must be 8-byte aligned; `ws` must be 256-byte aligned.
 *   - Outputs must not alias inputs or the workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls
 *     only enqueue work on it and never synchronize; results are visible after the
 *     stream is synchronized. All calls are asynchronous and thread-safe.
 *   - Arguments are validated on the host before anything is enqueued; a rejected
 *     call returns NDFT_E_INVAL, NDFT_E_UNSUPPORTED or NDFT_E_WORKSPACE and touches no
 *     memory. A workspace query returns 0 for a call that would be rejected.
 *   - Inputs must be finite, with magnitudes below 1e30.
 *   - Doppler / frequency bins are taken mod N, so negative starts are allowed.
 *   - Results are deterministic for a fixed plan: no floating-point atomics.
 *   - No exception crosses this boundary.
 */
#ifndef NDFT_H
#define NDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float re, im;
} ndft_c64;

typedef enum {
    NDFT_OK = 0,
    NDFT_E_INVAL = 1,       /* invalid argument (checked before any launch)        */
    NDFT_E_UNSUPPORTED = 2, /* precision or shape not available                   */
    NDFT_E_WORKSPACE = 3,   /* ws NULL, misaligned or smaller than the query      */
    NDFT_E_HIP = 4          /* a HIP runtime call or kernel launch failed         */
} ndft_status;

/* Arithmetic of the dense contraction (sign operands are exact in every form):
 *   NDFT_FP32   FP32 operands on FP32 matrix cores, FP32 accumulation. For n a power of
 *               two from 8 to 4096 and wide bin windows the built-in choice is the fast
 *               exact transform (plan "fp32x_fast_exact": every bin of a row from FFTs
 *               and cyclic correlations over the odd residues mod n, the same terms as
 *               Eq. (7) regrouped, FP32 arithmetic). Its tables depend on n alone and
 *               are kept per device and length in a library-held array (98 KB, no
 *               allocation): the first call of a length outside stream capture fills
 *               them and waits for its stream once; under capture an uncached length
 *               makes them in the call's workspace.
 *   NDFT_BF16X2 data split into BF16 hi + lo (|v - hi - lo| <= 2^-18 |v|), exact BF16
 *               signs, FP32 accumulation.
 *   NDFT_FP8    data split into four e4m3 terms (v = t0 + t1/16 + t2/256 + t3/4096 up to
 *               ~2^-16 |v|), exact e4m3 signs, block-scaled FP8 matrix cores, FP32
 *               accumulation. The data are carried scaled by a power of two taken from
 *               the inputs' largest |re| + |im| (one extra pass); at or above
 *               M = max(|s_r|+|s_i|) + max(|r_r|+|r_i|) = 2^29 (the forward NDFT:
 *               max(|x_r|+|x_i|)) the combined kernel returns NaN outputs, the FP8
 *               sign-split plans have no input limit. n is limited by LDS
 *               (NDFT_E_UNSUPPORTED above 2^20 for some plans). The adjoint has no FP8
 *               form (NDFT_E_UNSUPPORTED).                                            */
typedef enum { NDFT_FP32 = 0, NDFT_BF16X2 = 1, NDFT_FP8 = 2 } ndft_prec;

/* Maximum transform length. */
#define NDFT_MAX_N (1 << 24)

/* ---------------------------------------------------------------------------------
 * NDFT, Eq. (7) (no 1/N normalisation):
 *   X[b][q] = sum_{n=0}^{N-1} W^{(k0+q) n mod N} (x) x[b][n],  q in [0, k_count).
 * x: [batch][n] complex64 (row-major), X: [batch][k_count] complex64.
 * Limits: 1 <= n <= NDFT_MAX_N, batch >= 0, 1 <= k_count <= n, k0 any integer.
 * ------------------------------------------------------------------------------- */
size_t ndft_forward_workspace(int64_t batch, int64_t n, int64_t k0, int64_t k_count,
                              ndft_prec prec);
ndft_status ndft_forward(const ndft_c64 *x, ndft_c64 *X, int64_t batch, int64_t n, int64_t k0,
                         int64_t k_count, ndft_prec prec, void *ws, size_t ws_bytes,
                         void *stream);

/* ---------------------------------------------------------------------------------
 * Cross-ambiguity surface, Eq. (12a) of Section 4, read as
 *   A[l][q] = sum_{i=0}^{N-1} ( s[i] (x) conj(r[i - d]) ) (x) W^{i p mod N},
 *   d = tau0 + l (l in [0, n_tau)),  p = p0 + q mod N (q in [0, n_dop)),
 *   r[m] = 0 for m < 0 (the record is not circular).
 * The conjugate on the reference is the one of Eq. (11); the two operators associate
 * left to right, i.e. each range row is the NDFT of its lag-product sequence.
 * surv, ref: [n] complex64. A: [n_tau][n_dop] complex64, row-major (delay-major).
 * Limits: 1 <= n <= NDFT_MAX_N, 0 <= tau0, n_tau >= 1, tau0 + n_tau <= n,
 *         1 <= n_dop <= n, p0 any integer.
 * ------------------------------------------------------------------------------- */
size_t ndft_caf_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop,
                          ndft_prec prec);
ndft_status ndft_caf(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                     int64_t n_tau, int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec,
                     void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * ndft_caf without a caller workspace and without any allocation, for callers that
 * cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same surface, arguments, limits and kernels as
 * ndft_caf (bit-identical results for the same plan); the call's scratch is a static
 * device array of NDFT_NOALLOC_SCRATCH_BYTES that each GPU using the library holds
 * until the process ends. A call whose ndft_caf workspace exceeds that size returns
 * NDFT_E_WORKSPACE before anything is enqueued (at N = 65536 with 1024 delays x 512
 * bins: FP32 and BF16X2 fit, FP8 does not). The call allocates nothing (no hipMalloc,
 * no event records even with ndft_prof_enable on). All calls on one GPU share its
 * scratch and its contents are left as the last call wrote them: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be serialized by the
 * caller, e.g. by issuing them on one stream.
 * ------------------------------------------------------------------------------- */
#define NDFT_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)
ndft_status ndft_caf_noalloc(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                             int64_t n_tau, int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec,
                             void *stream);

/* ---------------------------------------------------------------------------------
 * NFFT of Section 3 (Eq. (10)): the radix-2 decimation-in-time FFT whose butterflies carry
 * the operator of Eq. (6), E / O the transforms of the even / odd samples, recursively
 * down to single samples. Two readings of the printed equation (`reading`):
 *   NDFT_NFFT_EVERY_BUTTERFLY: every butterfly's twiddle product is the operator,
 *     X[k] = E[k] + O[k] (x) W_n^k,  X[k + n/2] = E[k] - O[k] (x) W_n^k (W_n^0 = 1
 *     included): the multiplication-free transform the text describes;
 *   NDFT_NFFT_PRINTED: the twiddle in front of the odd half is an ordinary complex
 *     product, X[k] = E[k] + W_n^k O[k], and the operator sits in the sums, whose
 *     length-1 terms at the bottom are x (x) 1 (so the result is the DFT of x + csgn(x)).
 * Either way the values differ from the NDFT of Eq. (7) for n > 4 (the operator is not
 * linear). FP32, evaluated butterfly by butterfly in the recursion's operations (products
 * and sums rounded one by one); twiddles are e^{-j 2 pi m / n} rounded once to FP32, exact
 * at the quadrant points. x, X: [batch][n] complex64 device pointers (X may not alias x);
 * n a power of two, 1 <= n <= 2^24; batch >= 0. Rows longer than 8192 need the workspace
 * of ndft_nfft_workspace (ping-pong rows and a twiddle table; 0 otherwise, and for invalid
 * arguments). Returns NDFT_E_INVAL for invalid arguments, NDFT_E_WORKSPACE for a missing
 * or small workspace.
 * ------------------------------------------------------------------------------- */
#define NDFT_NFFT_EVERY_BUTTERFLY 0
#define NDFT_NFFT_PRINTED 1
size_t ndft_nfft_workspace(int64_t batch, int64_t n);
ndft_status ndft_nfft(const ndft_c64 *x, ndft_c64 *X, int64_t batch, int64_t n, int32_t reading, void *ws,
                      size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * The Eq. (12b) surface of Section 4: the lag product of Eq. (6), then the ordinary DFT,
 *   A[l][q] = sum_{i=0}^{N-1} ( s[i] (x) conj(r[i - d]) ) W^{i p mod N},
 * with d, p, the zero reference before the record, the layout and the limits of
 * ndft_caf. The outer transform is linear and is computed as a decimated DFT (length-L
 * FFTs, L the largest power of two dividing n up to 512, then n / L terms per requested
 * bin), in FP32: prec must be NDFT_FP32 (NDFT_BF16X2 / NDFT_FP8 return
 * NDFT_E_UNSUPPORTED). ndft_caf12b_workspace returns the bytes of the transform's scratch
 * (the inputs with their signs, or partial surfaces; 0 for invalid arguments).
 * Errors and stream as for ndft_caf.
 * ------------------------------------------------------------------------------- */
size_t ndft_caf12b_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop,
                             ndft_prec prec);
ndft_status ndft_caf12b(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                        int64_t n_tau, int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec,
                        void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * The Eq. (12c) surface of Section 4: the ordinary lag product of Eq. (11), then the
 * operator of Eq. (6) with the twiddle,
 *   A[l][q] = sum_{i=0}^{N-1} ( s[i] conj(r[i - d]) ) (x) W^{i p mod N},
 * with d, p, the zero reference before the record, the layout and the limits of
 * ndft_caf. The lag product's component signs are exact (FP64 from the complex64
 * inputs); its value enters in FP32.
 * The sign-split plans compute it (for any Doppler window): NDFT_BF16X2 / NDFT_FP8 with
 * the twiddle half on the matrix cores, NDFT_FP32 with it as an FFT of the exact lag
 * signs; in NDFT_FP32 the fast exact transform ("fp32x_fast_exact") too, the built-in
 * choice for n a power of two up to 4096 where the sign-split walk would be long (the
 * largest base b with 64 b > n). ndft_set_plan overrides apply when they name one of
 * these plans. Errors, workspace and stream as for ndft_caf.
 * ------------------------------------------------------------------------------- */
size_t ndft_caf12c_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0, int64_t n_dop,
                             ndft_prec prec);
ndft_status ndft_caf12c(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                        int64_t n_tau, int64_t p0, int64_t n_dop, ndft_c64 *A, ndft_prec prec,
                        void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * Batched surfaces: many CPIs of uneven length in one persistent launch.
 * CPI c computes the ndft_caf surface of
 *   surv_pool[surv_off .. surv_off + n), ref_pool[ref_off .. ref_off + n)
 * into out_pool[out_off .. out_off + n_tau * n_dop) with its own (n, tau0, n_tau, p0,
 * n_dop); offsets are in complex elements. Each CPI obeys the ndft_caf limits.
 *
 * ndft_caf_batched_prepare() validates the CPIs, picks one tile plan for the batch,
 * splits every surface into (tile, sample chunk) work items of about `chunk` samples
 * (0 = 4096; rounded to the plan's stage size), writes the CPI tables and the item list
 * (longest chunks first) into `ws` with a blocking host-to-device copy, and fills the
 * host struct `batch`. Call it outside stream capture. The `cpis` array is host memory
 * and may be freed afterwards.
 *
 * ndft_caf_batched() then only launches kernels on `stream` (no copies, allocations or
 * memsets), so it may be captured into a hipGraph and replayed; each run recomputes
 * every surface from the current pool contents. `batch` and `ws` must come from the
 * same prepare call (the kernels check a tag stored in `ws` and do nothing otherwise).
 * Calls that share a workspace must not overlap in time.
 * ------------------------------------------------------------------------------- */
typedef struct {
    int64_t n, surv_off, ref_off, out_off, tau0, n_tau, p0, n_dop;
} ndft_cpi;

typedef struct {
    int32_t prec, plan, n_cpi, n_items, grid, table_bytes, max_red_blocks, max_prep_blocks;
    uint64_t tag;
    uint64_t ws_bytes;
} ndft_batch;

size_t ndft_caf_batched_workspace(const ndft_cpi *cpis, int32_t n_cpi, ndft_prec prec, int32_t chunk);
ndft_status ndft_caf_batched_prepare(const ndft_cpi *cpis, int32_t n_cpi, ndft_prec prec, int32_t chunk,
                                     void *ws, size_t ws_bytes, ndft_batch *batch);
ndft_status ndft_caf_batched(const ndft_batch *batch, const ndft_c64 *surv_pool, const ndft_c64 *ref_pool,
                             ndft_c64 *out_pool, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * Device-described batches: the same surfaces, with the CPI descriptors in DEVICE memory
 * (cpis_dev[n_cpi], 8-byte aligned; 1 <= n_cpi <= 4096) and no host-side preparation.
 * A planning kernel reads the descriptors, lays out `ws` as ndft_caf_batched_prepare
 * would for the same descriptors, plan and default chunk, doubling the sample chunk while
 * the partial sums do not fit ws_bytes (fewer chunks: the same surfaces up to rounding
 * order), and the batched kernels follow on `stream`. The call enqueues kernels only (no copies, no allocation, no synchronization),
 * so descriptors and pools may change between replays of a captured graph. The tile plan
 * is the ndft_set_plan override when it has a batched form, else a fixed choice per
 * precision.
 * Errors found on the host (pointers, alignment, n_cpi, workspace smaller than the
 * tables) return before anything is enqueued. Errors only the device can see (an invalid
 * descriptor: the ndft_caf limits or a negative offset; a workspace too small even with
 * one chunk per surface) leave every output untouched and are reported by
 * ndft_caf_batched_dev_status, which copies the batch's status (0 = ran, else an
 * ndft_status value) to the caller's device int32 on `stream`. Pool bounds are the
 * caller's: offsets must keep every surface inside its pool.
 * ndft_caf_batched_dev_workspace: a size that fits any n_cpi CPIs with n <= max_n,
 * n_tau <= max_tau and n_dop <= max_dop at the default chunk (0 for invalid maxima).
 * ------------------------------------------------------------------------------- */
size_t ndft_caf_batched_dev_workspace(int32_t n_cpi, int64_t max_n, int64_t max_tau, int64_t max_dop,
                                      ndft_prec prec);
ndft_status ndft_caf_batched_dev(const ndft_c64 *surv_pool, const ndft_c64 *ref_pool, ndft_c64 *out_pool,
                                 const ndft_cpi *cpis_dev, int32_t n_cpi, ndft_prec prec, void *ws,
                                 size_t ws_bytes, void *stream);
ndft_status ndft_caf_batched_dev_status(const void *ws, int32_t *status, void *stream);

/* ---------------------------------------------------------------------------------
 * Adjoint of the surface with respect to the reference (and optionally the
 * surveillance) input, for a real loss L. grad_A[l][q] = dL/dRe A + j dL/dIm A; the
 * outputs use the same convention (grad_ref[m] = dL/dRe r[m] + j dL/dIm r[m]).
 * Derivative rule at every operator node: d(x (x) y)/dx = sign(y) (almost everywhere;
 * the jump of the sign is ignored), so no lag-product value enters the adjoint:
 *   gz[l][i]     = sum_q conj(grad_A[l][q]) csgn(W^{i p_q})
 *   grad_ref[m]  = sum_l csgn(s[m + d_l]) gz[l][m + d_l]
 *   grad_surv[i] = sum_l csgn(r[i - d_l]) conj(gz[l][i])
 * grad_ref, grad_surv: [n] complex64, fully overwritten; grad_surv may be NULL.
 * Same limits as ndft_caf. prec selects the contraction arithmetic of gz.
 * ------------------------------------------------------------------------------- */
size_t ndft_caf_backward_workspace(int64_t n, int64_t tau0, int64_t n_tau, int64_t p0,
                                   int64_t n_dop, ndft_prec prec);
ndft_status ndft_caf_backward(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                              int64_t n_tau, int64_t p0, int64_t n_dop, const ndft_c64 *grad_A,
                              ndft_c64 *grad_ref, ndft_c64 *grad_surv, ndft_prec prec, void *ws,
                              size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * Test hook: the exact ternary sign operands the kernels use, as int8 in {-1, 0, 1}.
 *   tw_sign[q][i][2]  = (sign Re, sign Im) of W^{i (p0+q) mod N}   (Eq. (7) twiddles)
 *   lag_sign[l][i][2] = (sign Re, sign Im) of s[i] (x) conj(r[i - tau0 - l])
 * Either output may be NULL. Same limits as ndft_caf. Device pointers.
 * ------------------------------------------------------------------------------- */
ndft_status ndft_dbg_signs(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                           int64_t n_tau, int64_t p0, int64_t n_dop, int8_t *tw_sign,
                           int8_t *lag_sign, void *stream);

/* ---------------------------------------------------------------------------------
 * Test hook: the sign operands of the sign-split plans, taken from the hot path itself.
 * With a (x) b = csgn(a) b + a csgn(b) (Eq. (1)-(2) applied to the four real operators of
 * Eq. (6)), each surface cell splits into T = sum_i csgn(W^{ip}) z_l[i] (twiddle signs
 * against lag values) and D = sum_i W^{ip} csgn(z_l[i]) (twiddles against lag signs).
 * This call picks the plan that ndft_caf (lin = 0, z the Eq. (6) lag product) or
 * ndft_caf12c (lin = 1, z = s conj(r), Eq. (11)) would pick for the same arguments, and
 * runs that plan's lag kernel exactly as the surface call does, without the rest:
 *   lag_sign[l][i][2] (int8, may be NULL): the exact lag signs (sign Re, sign Im) of
 *       z_l[i] as the lag kernel encodes them for the matrix-core half (2-bit code words),
 *       decoded; values in {-1, 0, 1} (2 would mark an invalid code);
 *   T[l][q] (complex64, may be NULL): the lag kernel's own partial sums reduced alone,
 *       i.e. T at every requested bin, except bins p = 0 mod n, which that kernel sums
 *       whole (T + D, the twiddle there being 1).
 * ws: the workspace of ndft_caf_workspace (lin = 0) or ndft_caf12c_workspace (lin = 1)
 * for the same arguments. Returns NDFT_E_UNSUPPORTED when the chosen plan is not a
 * sign-split plan (ndft_set_plan can force one). Limits and errors as ndft_caf.
 * ------------------------------------------------------------------------------- */
ndft_status ndft_dbg_split(const ndft_c64 *surv, const ndft_c64 *ref, int64_t n, int64_t tau0,
                           int64_t n_tau, int64_t p0, int64_t n_dop, ndft_prec prec, int32_t lin,
                           int8_t *lag_sign, ndft_c64 *T, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * Test hook: the lengths whose fast-exact-transform tables (group order of the odd
 * residues, its inverse, the correlation spectra) the current device holds, as a bit mask
 * (bit lg set: N = 2^lg cached). The library fills a length's slot on the first call of
 * that length outside stream capture (that call waits for its stream once); under capture
 * an uncached length makes its tables in the call's workspace. reset != 0 clears the
 * mask after reading it, so the next call of each length fills its slot again (with the
 * same values). Returns -1 when no device is current.
 * ------------------------------------------------------------------------------- */
int32_t ndft_dbg_fast_tables(int32_t reset);

/* ---------------------------------------------------------------------------------
 * Tile plans (used by the autotuner). A plan is a tile shape of the contraction
 * kernel; ksplit is the number of sample chunks reduced in a fixed order (0 = pick
 * from the shape). Setting plan -1 restores the built-in choice. The setting is
 * process-wide per precision (mutex-guarded); calls already enqueued are unaffected.
 * ------------------------------------------------------------------------------- */
int32_t ndft_plan_count(ndft_prec prec);
const char *ndft_plan_name(ndft_prec prec, int32_t plan);
ndft_status ndft_set_plan(ndft_prec prec, int32_t plan, int32_t ksplit);
/* The plan and ksplit ndft_caf / ndft_forward would use for (n, n_cols = delays or
 * rows, bins p0 .. p0 + n_bins - 1). ksplit counts the matrix-core sample chunks: 0 for
 * a plan with no matrix part (the FP32 sign-split plan, whose twiddle half is an FFT). */
ndft_status ndft_get_plan(ndft_prec prec, int64_t n, int64_t n_cols, int64_t p0, int64_t n_bins,
                          int32_t *plan, int32_t *ksplit);

/* ---------------------------------------------------------------------------------
 * Timing of the contraction kernel: when enabled, every call records a pair of
 * hipEvents around its contraction launch on the call's stream (the matrix-core kernel,
 * or the FFT of the twiddle half for the FP32 sign-split plan), and the sign-split
 * surfaces another pair around the twiddle-sign kernel. ndft_prof_read() waits for the
 * contraction events, returns the summed milliseconds and the number of launches since
 * the last read, and resets both; ndft_prof_read_slot(0, ...) is the same and slot 1 reads
 * the twiddle-sign kernel's events (other slots: NDFT_E_INVAL). Process-wide,
 * mutex-guarded.
 * ------------------------------------------------------------------------------- */
ndft_status ndft_prof_enable(int32_t on);
ndft_status ndft_prof_read(double *contract_ms, int64_t *launches);
ndft_status ndft_prof_read_slot(int32_t slot, double *ms_sum, int64_t *launches);

const char *ndft_status_string(ndft_status st);
const char *ndft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NDFT_H */
