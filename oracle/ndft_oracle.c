/*
 * Plain FP64 CPU oracle for the multiplication-free nonlinear DFT (NDFT) and the
 * NDFT-based cross-ambiguity surface.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code, header, table or
 * helper with the GPU path: it evaluates the paper's definitions literally, term by
 * term, in double precision, with no blocking, fusion or reordering.
 *
 * Paper: Bozkurt, Arslan, Sevimli, Akbas, Cetin, "Approximate Computation of DFT
 * without Performing Any Multiplications: Applications to Radar Signal Processing"
 * (arXiv 1402.0532).
 *
 *   rop(a,b)   real additive operator, Eq. (1) with the sign table of Eq. (2):
 *              sign(a*b)(|a|+|b|), and 0 when either operand is zero.
 *   cop(a,b)   complex additive operator, Eq. (6):
 *              a_r(x)b_r - a_i(x)b_i + j(a_i(x)b_r + b_i(x)a_r).
 *   NDFT       Eq. (7): X[k] = sum_n W^{kn mod N} (x) x[n], W = e^{-j2pi/N}, no 1/N.
 *   CAF        Eq. (12a), Section 4, read as ((s[i] (x) conj(r[i-d])) (x) W^{ip}):
 *              the lag product of the surveillance sample and the conjugated reference
 *              sample (the conjugate is the one written in Eq. (11)), then one NDFT per
 *              range bin. Reference samples before the start of the record are zero.
 *   NFFT       Section 3, Eq. (10): radix-2 decimation in time with every butterfly's
 *              twiddle product replaced by the operator of Eq. (6) (FP64, and FP32).
 *   CAF (12b)  Eq. (12b): the lag product of Eq. (6), then the ordinary DFT (complex
 *              products with W^{ip}).
 *   CAF (12c)  Eq. (12c): the ordinary lag product s[i] conj(r[i-d]) (Eq. (11)), then
 *              the operator of Eq. (6) with W^{ip}; signs of the lag product exact.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   - sign(0) = 0 and -0.0 counts as zero (Eq. (2) "otherwise").
 *   - Twiddles at quadrant multiples (4m divisible by N) are exactly 1, -j, -1, +j.
 *   - Doppler bin p = p0 + q is taken mod N; delays d = tau0 + l; r[m < 0] = 0.
 *   - The sign of every lag-product component is the exact sign of the real number
 *     defined by the (float32-valued) inputs, obtained with an exact fixed-point sum.
 *   - Gradients use the almost-everywhere derivative d(x(x)y)/dx = sign(y) at every
 *     operator node (the jump of the sign function is ignored).
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp (no -ffast-math, so no FTZ/DAZ).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------ */
/* Eq. (2): sign of a product, by case analysis.                                   */
/* ------------------------------------------------------------------------------ */
static int sign_of_product(double a, double b)
{
    if ((a > 0 && b > 0) || (a < 0 && b < 0)) return 1;
    if ((a < 0 && b > 0) || (a > 0 && b < 0)) return -1;
    return 0; /* "otherwise": at least one operand is +0 or -0 */
}

static int sgn(double a) { return a > 0 ? 1 : (a < 0 ? -1 : 0); }

/* Eq. (1): a (x) b = sign(a*b)(|a| + |b|). */
double oracle_rop(double a, double b)
{
    int s = sign_of_product(a, b);
    if (s == 0) return 0.0;
    return s * (fabs(a) + fabs(b));
}

/* Eq. (6): complex operator on interleaved {re, im} pairs. */
void oracle_cop(const double *a, const double *b, double *out)
{
    double ar = a[0], ai = a[1], br = b[0], bi = b[1];
    double re = oracle_rop(ar, br) - oracle_rop(ai, bi);
    double im = oracle_rop(ai, br) + oracle_rop(bi, ar);
    out[0] = re;
    out[1] = im;
}

/* ------------------------------------------------------------------------------ */
/* Exact sign of a signed sum of finite doubles.                                   */
/* Every finite double is an integer multiple of 2^-1074. Each |v_k| is written    */
/* as that integer in base-2^32 digits and the signed terms are added digit by     */
/* digit in 64-bit integers, so the result is exact.                               */
/* ------------------------------------------------------------------------------ */
#define EXACT_DIGITS 72 /* 72 * 32 = 2304 bits > 1074 + 1024 + 53 */

static int exact_sign_of_sum(const double *v, const int *c, int n)
{
    int64_t dig[EXACT_DIGITS];
    memset(dig, 0, sizeof(dig));
    for (int k = 0; k < n; ++k) {
        if (c[k] == 0 || v[k] == 0.0) continue;
        int e;
        double m = frexp(fabs(v[k]), &e);       /* |v| = m * 2^e, m in [0.5, 1) */
        uint64_t M = (uint64_t)ldexp(m, 53);    /* exact: |v| = M * 2^(e-53)    */
        int sh = e - 53 + 1074;                 /* |v| = M * 2^(sh) * 2^-1074   */
        while (sh < 0) {                        /* only trailing zero bits drop */
            M >>= 1;
            sh += 1;
        }
        int d = sh / 32, o = sh % 32;
        unsigned __int128 w = ((unsigned __int128)M) << o; /* < 2^85 */
        for (int t = 0; t < 3 && d + t < EXACT_DIGITS; ++t) {
            int64_t chunk = (int64_t)(uint32_t)(w >> (32 * t));
            dig[d + t] += c[k] > 0 ? chunk : -chunk;
        }
    }
    /* carry-normalise: digits 0..D-2 into [0, 2^32), the top digit keeps the sign */
    for (int i = 0; i < EXACT_DIGITS - 1; ++i) {
        int64_t carry = dig[i] >> 32; /* arithmetic shift: floor division */
        dig[i] -= carry * ((int64_t)1 << 32);
        dig[i + 1] += carry;
    }
    if (dig[EXACT_DIGITS - 1] != 0) return dig[EXACT_DIGITS - 1] > 0 ? 1 : -1;
    for (int i = EXACT_DIGITS - 2; i >= 0; --i)
        if (dig[i] != 0) return 1;
    return 0;
}

int oracle_exact_sign_of_sum(const double *v, const int *c, int n)
{
    return exact_sign_of_sum(v, c, n);
}

/* ------------------------------------------------------------------------------ */
/* A real number carried as its FP64 value and its exact sign.                     */
/* ------------------------------------------------------------------------------ */
typedef struct {
    double v; /* value (rounded to FP64 at most once per operation)          */
    int s;    /* exact sign of the real number that v stands for             */
} xreal;

/* rop where the first operand's sign is known exactly (Eq. (1)-(2)). */
static double rop_x(xreal a, double b)
{
    int s = a.s * sgn(b);
    if (s == 0) return 0.0;
    return s * (fabs(a.v) + fabs(b));
}

/* ------------------------------------------------------------------------------ */
/* Twiddle W^m = e^{-j 2 pi m / N}, exponent reduced mod N (Eq. (7)).              */
/* Exactly 1, -j, -1, +j at the quadrant multiples.                                */
/* ------------------------------------------------------------------------------ */
static int64_t mod_n(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

void oracle_twiddle(int64_t m, int64_t n, double *out)
{
    m = mod_n(m, n);
    if ((4 * m) % n == 0) {
        static const double q[4][2] = {{1, 0}, {0, -1}, {-1, 0}, {0, 1}};
        int k = (int)((4 * m) / n);
        out[0] = q[k][0];
        out[1] = q[k][1];
        return;
    }
    double th = 2.0 * M_PI * (double)m / (double)n;
    out[0] = cos(th);
    out[1] = -sin(th);
}

/* ------------------------------------------------------------------------------ */
/* Lag product z = s (x) conj(r) (Eq. (6) applied to the Eq. (11) product), with   */
/* the exact sign of each component.                                               */
/* ------------------------------------------------------------------------------ */
static void lag_product(double sr, double si, double rr, double ri, xreal *zr, xreal *zi)
{
    double br = rr, bi = -ri; /* conj(r) */
    /* z_r = s_r (x) b_r - s_i (x) b_i */
    double t1 = oracle_rop(sr, br), t2 = oracle_rop(si, bi);
    zr->v = t1 - t2;
    {
        int e1 = sign_of_product(sr, br), e2 = sign_of_product(si, bi);
        double v[4] = {sr, br, si, bi};
        int c[4] = {e1, e1, -e2, -e2};
        zr->s = exact_sign_of_sum(v, c, 4);
    }
    /* z_i = s_i (x) b_r + b_i (x) s_r */
    double t3 = oracle_rop(si, br), t4 = oracle_rop(bi, sr);
    zi->v = t3 + t4;
    {
        int e3 = sign_of_product(si, br), e4 = sign_of_product(bi, sr);
        double v[4] = {si, br, bi, sr};
        int c[4] = {e3, e3, e4, e4};
        zi->s = exact_sign_of_sum(v, c, 4);
    }
}

/* ------------------------------------------------------------------------------ */
/* Linear lag product z = s conj(r) (the ordinary product of Eq. (11), used by the */
/* Eq. (12c) surface), with the exact sign of each component: each real product is */
/* split exactly into value + error (fma), and the sign of their sum is exact.     */
/* ------------------------------------------------------------------------------ */
static void two_product(double a, double b, double *p, double *e)
{
    *p = a * b;
    *e = fma(a, b, -*p);
}

static void linear_lag_product(double sr, double si, double rr, double ri, xreal *zr, xreal *zi)
{
    double br = rr, bi = -ri; /* conj(r) */
    double p[4], e[4];
    /* z_r = s_r b_r - s_i b_i */
    two_product(sr, br, &p[0], &e[0]);
    two_product(si, bi, &p[1], &e[1]);
    zr->v = p[0] - p[1];
    {   /* exact_sign_of_sum weighs |v[k]| by c[k]: the signs of the terms go into c */
        double v[4] = {p[0], e[0], p[1], e[1]};
        int c[4] = {sgn(p[0]), sgn(e[0]), -sgn(p[1]), -sgn(e[1])};
        zr->s = exact_sign_of_sum(v, c, 4);
    }
    /* z_i = s_i b_r + s_r b_i */
    two_product(si, br, &p[2], &e[2]);
    two_product(sr, bi, &p[3], &e[3]);
    zi->v = p[2] + p[3];
    {
        double v[4] = {p[2], e[2], p[3], e[3]};
        int c[4] = {sgn(p[2]), sgn(e[2]), sgn(p[3]), sgn(e[3])};
        zi->s = exact_sign_of_sum(v, c, 4);
    }
}

/* One lag-product row: z[i] = s[i] (x) conj(r[i-d]), i in [0, n); r[m<0] = 0.
 * z is interleaved complex FP64 [n][2]; zsign (optional) is int8 [n][2]. */
static void lag_row_impl(const double *s, const double *r, int64_t n, int64_t d, double *z, int8_t *zsign,
                         int linear)
{
    for (int64_t i = 0; i < n; ++i) {
        double rr = 0.0, ri = 0.0;
        if (i - d >= 0 && i - d < n) {
            rr = r[2 * (i - d)];
            ri = r[2 * (i - d) + 1];
        }
        xreal zr, zi;
        if (linear)
            linear_lag_product(s[2 * i], s[2 * i + 1], rr, ri, &zr, &zi);
        else
            lag_product(s[2 * i], s[2 * i + 1], rr, ri, &zr, &zi);
        z[2 * i] = zr.v;
        z[2 * i + 1] = zi.v;
        if (zsign) {
            zsign[2 * i] = (int8_t)zr.s;
            zsign[2 * i + 1] = (int8_t)zi.s;
        }
    }
}

void oracle_lag_row(const double *s, const double *r, int64_t n, int64_t d, double *z,
                    int8_t *zsign)
{
    lag_row_impl(s, r, n, d, z, zsign, 0);
}

/* The linear lag-product row of Eq. (12c): z[i] = s[i] conj(r[i-d]). */
void oracle_lag_row_lin(const double *s, const double *r, int64_t n, int64_t d, double *z,
                        int8_t *zsign)
{
    lag_row_impl(s, r, n, d, z, zsign, 1);
}

/* Signs of the twiddle operand, csgn(W^{(p0+q) i mod N}) as int8 [n_dop][n][2]. */
void oracle_twiddle_signs(int64_t n, int64_t p0, int64_t n_dop, int8_t *out)
{
    for (int64_t q = 0; q < n_dop; ++q) {
        int64_t p = mod_n(p0 + q, n);
        for (int64_t i = 0; i < n; ++i) {
            double w[2];
            oracle_twiddle(mod_n(p * i, n), n, w);
            out[2 * (q * n + i)] = (int8_t)sgn(w[0]);
            out[2 * (q * n + i) + 1] = (int8_t)sgn(w[1]);
        }
    }
}

/* ------------------------------------------------------------------------------ */
/* NDFT, Eq. (7). X[b][q] = sum_n cop(W^{(k0+q) n mod N}, x[b][n]).                */
/* scale[b][q] = sum over n of the magnitudes of the four real operator terms.    */
/* ------------------------------------------------------------------------------ */
int oracle_ndft(const double *x, int64_t batch, int64_t n, int64_t k0, int64_t k_count,
                double *X, double *scale)
{
    if (n < 1 || batch < 0 || k_count < 0) return 1;
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int64_t b = 0; b < batch; ++b) {
        for (int64_t q = 0; q < k_count; ++q) {
            const double *xb = x + 2 * b * n;
            int64_t k = mod_n(k0 + q, n);
            double re = 0.0, im = 0.0, sc = 0.0;
            for (int64_t t = 0; t < n; ++t) {
                double w[2];
                oracle_twiddle(mod_n(k * t, n), n, w);
                /* cop(W, x): W_r(x)x_r - W_i(x)x_i + j(W_i(x)x_r + x_i(x)W_r) */
                double a = oracle_rop(w[0], xb[2 * t]);
                double bb = oracle_rop(w[1], xb[2 * t + 1]);
                double c = oracle_rop(w[1], xb[2 * t]);
                double d = oracle_rop(xb[2 * t + 1], w[0]);
                re += a - bb;
                im += c + d;
                sc += fabs(a) + fabs(bb) + fabs(c) + fabs(d);
            }
            X[2 * (b * k_count + q)] = re;
            X[2 * (b * k_count + q) + 1] = im;
            if (scale) scale[b * k_count + q] = sc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* Cross-ambiguity surface, Eq. (12a):                                             */
/*   A[l][q] = sum_i cop( cop(s[i], conj(r[i-d])), W^{i p mod N} ),                 */
/*   d = tau0 + rows[l] (or tau0 + l when rows == NULL), p = p0 + q mod N.          */
/* Output A[n_rows][n_dop] interleaved complex; scale[n_rows][n_dop] (optional).    */
/* ------------------------------------------------------------------------------ */
static int caf_impl(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                    int64_t p0, int64_t n_dop, const int64_t *rows, int64_t n_rows, double *A,
                    double *scale, int linear, int linear_outer)
{
    if (n < 1 || tau0 < 0 || n_tau < 0 || tau0 + n_tau > n || n_dop < 0) return 1;
    if (!rows) n_rows = n_tau;
#pragma omp parallel
    {
        double *zrow = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        int8_t *zsg = (int8_t *)malloc((size_t)(2 * n));
#pragma omp for schedule(dynamic)
        for (int64_t li = 0; li < n_rows; ++li) {
            int64_t l = rows ? rows[li] : li;
            int64_t d = tau0 + l;
            lag_row_impl(s, r, n, d, zrow, zsg, linear);
            if (linear_outer) { /* Eq. (12b): the ordinary DFT of the lag-product row */
                for (int64_t q = 0; q < n_dop; ++q) {
                    int64_t p = mod_n(p0 + q, n);
                    double re = 0.0, im = 0.0, sc = 0.0;
                    for (int64_t i = 0; i < n; ++i) {
                        double w[2];
                        oracle_twiddle(mod_n(i * p, n), n, w);
                        const double a = zrow[2 * i] * w[0], b = zrow[2 * i + 1] * w[1];
                        const double c = zrow[2 * i + 1] * w[0], e = zrow[2 * i] * w[1];
                        re += a - b;
                        im += c + e;
                        sc += fabs(a) + fabs(b) + fabs(c) + fabs(e);
                    }
                    A[2 * (li * n_dop + q)] = re;
                    A[2 * (li * n_dop + q) + 1] = im;
                    if (scale) scale[li * n_dop + q] = sc;
                }
                continue;
            }
            for (int64_t q = 0; q < n_dop; ++q) {
                int64_t p = mod_n(p0 + q, n);
                double re = 0.0, im = 0.0, sc = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    double w[2];
                    oracle_twiddle(mod_n(i * p, n), n, w);
                    xreal zr = {zrow[2 * i], zsg[2 * i]};
                    xreal zi = {zrow[2 * i + 1], zsg[2 * i + 1]};
                    /* cop(z, W) = z_r(x)c - z_i(x)t + j(z_i(x)c + t(x)z_r) */
                    double a = rop_x(zr, w[0]);
                    double b = rop_x(zi, w[1]);
                    double c = rop_x(zi, w[0]);
                    double e = rop_x(zr, w[1]);
                    re += a - b;
                    im += c + e;
                    sc += fabs(a) + fabs(b) + fabs(c) + fabs(e);
                }
                A[2 * (li * n_dop + q)] = re;
                A[2 * (li * n_dop + q) + 1] = im;
                if (scale) scale[li * n_dop + q] = sc;
            }
        }
        free(zrow);
        free(zsg);
    }
    return 0;
}

/* Eq. (12a): A[l][q] = sum_i cop(cop(s[i], conj(r[i-l])), W^{i p}) (see above). */
int oracle_caf(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
               int64_t p0, int64_t n_dop, const int64_t *rows, int64_t n_rows, double *A,
               double *scale)
{
    return caf_impl(s, r, n, tau0, n_tau, p0, n_dop, rows, n_rows, A, scale, 0, 0);
}

/* Eq. (12c): the linear lag product s[i] conj(r[i-l]), then the operator of Eq. (6)
 * with the twiddle: A[l][q] = sum_i cop(s[i] conj(r[i-l]), W^{i p}); scale as above. */
int oracle_caf_lin(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                   int64_t p0, int64_t n_dop, const int64_t *rows, int64_t n_rows, double *A,
                   double *scale)
{
    return caf_impl(s, r, n, tau0, n_tau, p0, n_dop, rows, n_rows, A, scale, 1, 0);
}

/* Eq. (12b): the lag product of Eq. (6), s[i] (x) conj(r[i-l]), then the ordinary DFT:
 * A[l][q] = sum_i z_i W^{i p} (complex products), scale = sum_i of the four |real
 * products| of z_i W^{i p}. */
int oracle_caf_dft(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                   int64_t p0, int64_t n_dop, const int64_t *rows, int64_t n_rows, double *A,
                   double *scale)
{
    return caf_impl(s, r, n, tau0, n_tau, p0, n_dop, rows, n_rows, A, scale, 0, 1);
}

/* ------------------------------------------------------------------------------ */
/* Loss and gradient of L = sum_{l,q} w[l][q] |A[l][q]|^2 (or any upstream G).     */
/* ------------------------------------------------------------------------------ */

/* Reverse-mode through the literal expression of Eq. (12a) with the a.e. rule
 * d rop(a,b)/da = sign(b), d rop(a,b)/db = sign(a). G[l][q] = dL/dRe A + j dL/dIm A.
 * Outputs grad_r, grad_s (either may be NULL) in the same convention, [n][2].
 * Each thread accumulates its own partial gradient; the partials are added in thread
 * order at the end. */
int oracle_caf_grad(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                    int64_t p0, int64_t n_dop, const double *G, double *grad_r, double *grad_s)
{
    if (n < 1 || tau0 < 0 || n_tau < 0 || tau0 + n_tau > n || n_dop < 0) return 1;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nthr * 4 * (size_t)n, sizeof(double));
    if (!part) return 2;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gr = part + (size_t)tid * 4 * (size_t)n; /* grad_r partial [n][2] */
        double *gs = gr + 2 * n;                          /* grad_s partial [n][2] */
        double *zrow = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        int8_t *zsg = (int8_t *)malloc((size_t)(2 * n));
        double *dz = (double *)malloc(sizeof(double) * 2 * (size_t)n);
#pragma omp for schedule(dynamic)
        for (int64_t l = 0; l < n_tau; ++l) {
            int64_t d = tau0 + l;
            oracle_lag_row(s, r, n, d, zrow, zsg);
            /* dL/dz for the outer operator, summed over Doppler bins */
            for (int64_t i = 0; i < n; ++i) {
                dz[2 * i] = 0.0;
                dz[2 * i + 1] = 0.0;
            }
            for (int64_t q = 0; q < n_dop; ++q) {
                int64_t p = mod_n(p0 + q, n);
                double gre = G[2 * (l * n_dop + q)], gim = G[2 * (l * n_dop + q) + 1];
                for (int64_t i = 0; i < n; ++i) {
                    double w[2];
                    oracle_twiddle(mod_n(i * p, n), n, w);
                    int sc = sgn(w[0]), st = sgn(w[1]);
                    /* re = z_r(x)c - z_i(x)t ; im = z_i(x)c + t(x)z_r */
                    dz[2 * i] += gre * sc + gim * st;
                    dz[2 * i + 1] += -gre * st + gim * sc;
                }
            }
            /* through the lag product a = s[i], b = conj(r[i-d]) */
            for (int64_t i = d; i < n; ++i) {
                double ar = s[2 * i], ai = s[2 * i + 1];
                double br = r[2 * (i - d)], bi = -r[2 * (i - d) + 1];
                double dzr = dz[2 * i], dzi = dz[2 * i + 1];
                /* z_r = a_r(x)b_r - a_i(x)b_i ; z_i = a_i(x)b_r + b_i(x)a_r */
                double dar = dzr * sgn(br) + dzi * sgn(bi);
                double dai = -dzr * sgn(bi) + dzi * sgn(br);
                double dbr = dzr * sgn(ar) + dzi * sgn(ai);
                double dbi = -dzr * sgn(ai) + dzi * sgn(ar);
                gs[2 * i] += dar;
                gs[2 * i + 1] += dai;
                gr[2 * (i - d)] += dbr;
                gr[2 * (i - d) + 1] -= dbi; /* b_i = -r_i */
            }
        }
        free(zrow);
        free(zsg);
        free(dz);
    }
    for (int64_t k = 0; k < 2 * n; ++k) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < nthr; ++t) {
            a += part[(size_t)t * 4 * (size_t)n + (size_t)k];
            b += part[(size_t)t * 4 * (size_t)n + 2 * (size_t)n + (size_t)k];
        }
        if (grad_r) grad_r[k] = a;
        if (grad_s) grad_s[k] = b;
    }
    free(part);
    return 0;
}

/* L = sum w |A|^2 of the literal surface. */
double oracle_caf_loss(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                       int64_t p0, int64_t n_dop, const double *w)
{
    double *A = (double *)malloc(sizeof(double) * 2 * (size_t)(n_tau * n_dop));
    if (!A) return NAN;
    oracle_caf(s, r, n, tau0, n_tau, p0, n_dop, NULL, 0, A, NULL);
    double L = 0.0;
    for (int64_t k = 0; k < n_tau * n_dop; ++k)
        L += w[k] * (A[2 * k] * A[2 * k] + A[2 * k + 1] * A[2 * k + 1]);
    free(A);
    return L;
}

/* Central finite differences of L = sum w |A|^2 with respect to selected real
 * coordinates of the reference: coord c means Re r[c/2] (c even) or Im r[c/2] (c odd).
 * A perturbation of r[m] only changes the lag products z_l[m + d], so each side is
 * evaluated by replacing those terms in the stored surface (no reordering of what
 * each term is). out[k] = (L(r + h e_c) - L(r - h e_c)) / (2h). */
int oracle_caf_loss_fd(const double *s, const double *r, int64_t n, int64_t tau0, int64_t n_tau,
                       int64_t p0, int64_t n_dop, const double *w, const int64_t *coords,
                       int64_t n_coords, double h, double *out)
{
    if (n < 1 || tau0 < 0 || n_tau < 0 || tau0 + n_tau > n || n_dop < 0) return 1;
    double *A = (double *)malloc(sizeof(double) * 2 * (size_t)(n_tau * n_dop));
    double *tw = (double *)malloc(sizeof(double) * 2 * (size_t)n); /* W^v, v < n, as oracle_twiddle gives it */
    if (!A || !tw) {
        free(A);
        free(tw);
        return 2;
    }
    oracle_caf(s, r, n, tau0, n_tau, p0, n_dop, NULL, 0, A, NULL);
    for (int64_t v = 0; v < n; ++v) oracle_twiddle(v, n, tw + 2 * v);
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < n_coords; ++k) {
        int64_t m = coords[k] / 2;
        int part = (int)(coords[k] % 2);
        double Lside[2];
        for (int side = 0; side < 2; ++side) {
            double delta = side == 0 ? h : -h;
            double L = 0.0;
            for (int64_t l = 0; l < n_tau; ++l) {
                int64_t d = tau0 + l;
                int64_t i = m + d; /* the only sample whose lag product moves */
                int touched = (i < n);
                xreal zo_r, zo_i, zn_r, zn_i;
                if (touched) {
                    double rr = r[2 * m], ri = r[2 * m + 1];
                    lag_product(s[2 * i], s[2 * i + 1], rr, ri, &zo_r, &zo_i);
                    if (part == 0) rr += delta; else ri += delta;
                    lag_product(s[2 * i], s[2 * i + 1], rr, ri, &zn_r, &zn_i);
                }
                for (int64_t q = 0; q < n_dop; ++q) {
                    double re = A[2 * (l * n_dop + q)], im = A[2 * (l * n_dop + q) + 1];
                    if (touched) {
                        int64_t p = mod_n(p0 + q, n);
                        const double *wv = tw + 2 * mod_n(i * p, n);
                        re += (rop_x(zn_r, wv[0]) - rop_x(zn_i, wv[1])) -
                              (rop_x(zo_r, wv[0]) - rop_x(zo_i, wv[1]));
                        im += (rop_x(zn_i, wv[0]) + rop_x(zn_r, wv[1])) -
                              (rop_x(zo_i, wv[0]) + rop_x(zo_r, wv[1]));
                    }
                    L += w[l * n_dop + q] * (re * re + im * im);
                }
            }
            Lside[side] = L;
        }
        out[k] = (Lside[0] - Lside[1]) / (2.0 * h);
    }
    free(A);
    free(tw);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------ */
/* NFFT, Section 3 (Eq. (10)): radix-2 decimation in time, recursively down to     */
/* single samples, with every twiddle product of a butterfly replaced by the       */
/* operator of Eq. (6): X[k] = E[k] + cop(O[k], W_n^k), X[k + n/2] = E[k] -        */
/* cop(O[k], W_n^k), E / O the NFFTs of the even / odd samples (W_n^0 = 1 included: */
/* no ordinary multiplication is left). The sign of every intermediate decides a    */
/* jump of the result, so besides FP64 the same recursion is given in FP32 (the     */
/* GPU's precision) with twiddles rounded once from FP64.                           */
/* ------------------------------------------------------------------------------ */
static void nfft64_rec(const double *x, int64_t n, int64_t stride, int64_t N, double *X, double *tmp)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    const int64_t h = n / 2;
    double *E = tmp, *O = tmp + 2 * h, *sub = tmp + 4 * h;
    nfft64_rec(x, h, 2 * stride, N, E, sub);
    nfft64_rec(x + 2 * stride, h, 2 * stride, N, O, sub);
    for (int64_t k = 0; k < h; ++k) {
        double w[2], t[2];
        oracle_twiddle(k * (N / n), N, w);
        oracle_cop(O + 2 * k, w, t);
        X[2 * k] = E[2 * k] + t[0];
        X[2 * k + 1] = E[2 * k + 1] + t[1];
        X[2 * (k + h)] = E[2 * k] - t[0];
        X[2 * (k + h) + 1] = E[2 * k + 1] - t[1];
    }
}

static float rop32(float a, float b)
{
    const int s = sign_of_product((double)a, (double)b);
    if (s == 0) return 0.0f;
    const float m = fabsf(a) + fabsf(b);
    return s > 0 ? m : -m;
}

static void nfft32_rec(const float *x, int64_t n, int64_t stride, int64_t N, const float *tw, float *X, float *tmp)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    const int64_t h = n / 2;
    float *E = tmp, *O = tmp + 2 * h, *sub = tmp + 4 * h;
    nfft32_rec(x, h, 2 * stride, N, tw, E, sub);
    nfft32_rec(x + 2 * stride, h, 2 * stride, N, tw, O, sub);
    for (int64_t k = 0; k < h; ++k) {
        const float *w = tw + 2 * (k * (N / n));
        const float orr = O[2 * k], oi = O[2 * k + 1];
        const float tr = rop32(orr, w[0]) - rop32(oi, w[1]);
        const float ti = rop32(oi, w[0]) + rop32(w[1], orr);
        X[2 * k] = E[2 * k] + tr;
        X[2 * k + 1] = E[2 * k + 1] + ti;
        X[2 * (k + h)] = E[2 * k] - tr;
        X[2 * (k + h) + 1] = E[2 * k + 1] - ti;
    }
}

/* ------------------------------------------------------------------------------ */
/* The printed reading of Eq. (10): the twiddle W_n^k in front of the odd half is an  */
/* ordinary complex product at every level, X[k] = E[k] + W_n^k O[k], X[k + n/2] =   */
/* E[k] - W_n^k O[k], and the operator of Eq. (6) sits in the sums themselves, whose  */
/* terms at the bottom of the recursion are single samples against W^0 = 1: the       */
/* length-1 transform of a sample x is x (x) 1.                                       */
/* ------------------------------------------------------------------------------ */
static void nfft64o_rec(const double *x, int64_t n, int64_t stride, int64_t N, double *X, double *tmp)
{
    if (n == 1) {
        const double one[2] = {1.0, 0.0};
        oracle_cop(x, one, X);
        return;
    }
    const int64_t h = n / 2;
    double *E = tmp, *O = tmp + 2 * h, *sub = tmp + 4 * h;
    nfft64o_rec(x, h, 2 * stride, N, E, sub);
    nfft64o_rec(x + 2 * stride, h, 2 * stride, N, O, sub);
    for (int64_t k = 0; k < h; ++k) {
        double w[2];
        oracle_twiddle(k * (N / n), N, w);
        const double tr = O[2 * k] * w[0] - O[2 * k + 1] * w[1];
        const double ti = O[2 * k] * w[1] + O[2 * k + 1] * w[0];
        X[2 * k] = E[2 * k] + tr;
        X[2 * k + 1] = E[2 * k + 1] + ti;
        X[2 * (k + h)] = E[2 * k] - tr;
        X[2 * (k + h) + 1] = E[2 * k + 1] - ti;
    }
}

/* The same in FP32, every product and sum rounded on its own (no fused multiply-add). */
static void nfft32o_rec(const float *x, int64_t n, int64_t stride, int64_t N, const float *tw, float *X, float *tmp)
{
    if (n == 1) {
        X[0] = rop32(x[0], 1.0f) - rop32(x[1], 0.0f);
        X[1] = rop32(x[1], 1.0f) + rop32(0.0f, x[0]);
        return;
    }
    const int64_t h = n / 2;
    float *E = tmp, *O = tmp + 2 * h, *sub = tmp + 4 * h;
    nfft32o_rec(x, h, 2 * stride, N, tw, E, sub);
    nfft32o_rec(x + 2 * stride, h, 2 * stride, N, tw, O, sub);
    for (int64_t k = 0; k < h; ++k) {
        const float *w = tw + 2 * (k * (N / n));
        const float orr = O[2 * k], oi = O[2 * k + 1];
        const float p1 = orr * w[0], p2 = oi * w[1], p3 = orr * w[1], p4 = oi * w[0];
        const float tr = p1 - p2, ti = p3 + p4;
        X[2 * k] = E[2 * k] + tr;
        X[2 * k + 1] = E[2 * k + 1] + ti;
        X[2 * (k + h)] = E[2 * k] - tr;
        X[2 * (k + h) + 1] = E[2 * k + 1] - ti;
    }
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* x, X: [batch][n][2] FP64; n a power of two. */
int oracle_nfft(const double *x, int64_t batch, int64_t n, double *X)
{
    if (!is_pow2(n) || batch < 0) return 1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < batch; ++b) {
        double *tmp = (double *)malloc(sizeof(double) * 8 * (size_t)n + 16);
        nfft64_rec(x + 2 * b * n, n, 1, n, X + 2 * b * n, tmp);
        free(tmp);
    }
    return 0;
}

/* The same in FP32: x, X [batch][n][2] float; twiddle W_n^m = e^{-j 2 pi m / n} rounded
 * to FP32 from the FP64 values of oracle_twiddle (exact at the quadrant points). */
int oracle_nfft32(const float *x, int64_t batch, int64_t n, float *X)
{
    if (!is_pow2(n) || batch < 0) return 1;
    float *tw = (float *)malloc(sizeof(float) * 2 * (size_t)n);
    for (int64_t m = 0; m < n; ++m) {
        double w[2];
        oracle_twiddle(m, n, w);
        tw[2 * m] = (float)w[0];
        tw[2 * m + 1] = (float)w[1];
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < batch; ++b) {
        float *tmp = (float *)malloc(sizeof(float) * 8 * (size_t)n + 16);
        nfft32_rec(x + 2 * b * n, n, 1, n, tw, X + 2 * b * n, tmp);
        free(tmp);
    }
    free(tw);
    return 0;
}


/* Printed reading of Eq. (10) (see nfft64o_rec): FP64 and FP32. */
int oracle_nfft_outer(const double *x, int64_t batch, int64_t n, double *X)
{
    if (!is_pow2(n) || batch < 0) return 1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < batch; ++b) {
        double *tmp = (double *)malloc(sizeof(double) * 8 * (size_t)n + 16);
        nfft64o_rec(x + 2 * b * n, n, 1, n, X + 2 * b * n, tmp);
        free(tmp);
    }
    return 0;
}

int oracle_nfft32_outer(const float *x, int64_t batch, int64_t n, float *X)
{
    if (!is_pow2(n) || batch < 0) return 1;
    float *tw = (float *)malloc(sizeof(float) * 2 * (size_t)n);
    for (int64_t m = 0; m < n; ++m) {
        double w[2];
        oracle_twiddle(m, n, w);
        tw[2 * m] = (float)w[0];
        tw[2 * m + 1] = (float)w[1];
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < batch; ++b) {
        float *tmp = (float *)malloc(sizeof(float) * 8 * (size_t)n + 16);
        nfft32o_rec(x + 2 * b * n, n, 1, n, tw, X + 2 * b * n, tmp);
        free(tmp);
    }
    free(tw);
    return 0;
}
