/*
 * FP64 CPU oracle for the Bayesian logistic-regression log-posterior and its
 * gradient.  TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against a plain, slow, obviously correct computation.  Nothing in the
 * product links or calls it, and it shares no code with the GPU library.
 *
 * What it computes (plain definition, written out):
 *   u_n   = sum_k x_nk beta_k                                  (linear predictor)
 *   L     = sum_n [ y_n u_n - softplus(u_n) ]
 *           which is the paper's logistic log-likelihood (Sec. 3.1.1,
 *           eq-loglike-binlogit): -( (1-y) u + log(1+exp(-u)) ) = y u - softplus(u)
 *   g_L   = sum_n (y_n - sigmoid(u_n)) x_n = X^t g_f          (Sec. 4.2,
 *           eq-grad-expanded / eq-grad-compact, with f_n'(u) = y_n - 1/(1+e^-u))
 *   prior : Gaussian N(m, prec^-1 I) on beta (Sec. 3.1.1 names a Gaussian prior
 *           without fixing it); its log density up to the normalising constant
 *           is -prec/2 |beta - m|^2 with gradient -prec (beta - m).
 *   f     = L - prec/2 |beta - m|^2,   g = g_L - prec (beta - m).
 *
 * Poisson regression (log link; the paper notes that only the per-row map
 * changes for other GLMs, Sec. 3.4) replaces the per-row terms by
 *   t_n = y_n u_n - exp(u_n),  r_n = y_n - exp(u_n)   (y_n a count 0..255),
 * leaving out the constant -log(y_n!).
 *
 * For the logistic model the response y_n must be 0 or 1.  softplus and sigmoid are evaluated in the
 * overflow-free forms softplus(u) = max(u,0) + log1p(exp(-|u|)) and
 * sigmoid(u) = 1/(1+exp(-u)) (u >= 0) or exp(u)/(1+exp(u)) (u < 0); in exact
 * arithmetic these equal log(1+exp(u)) and 1/(1+exp(-u)).
 *
 * Precision: all arithmetic in IEEE double.  The sums over rows n are taken
 * in ascending n with Neumaier's compensated summation (A. Neumaier, ZAMM 54,
 * 1974), one running sum for f and one for each g_k.  The stored X is
 * converted to double element by element (exact for FP32 and BF16; for FP8
 * the decoded code times its FP32 column scale, also exact in double).
 *
 * Storage formats (decoders / encoders follow the bit-level definitions):
 *   BF16: the upper 16 bits of an IEEE binary32; encoding rounds to nearest,
 *         ties to even.
 *   FP8 E4M3 (OCP "E4M3FN"): 1 sign, 4 exponent (bias 7), 3 mantissa bits,
 *         no infinities, S.1111.111 is NaN, largest finite 448; encoding of
 *         x / s_k rounds to nearest even and saturates at +-448.  The column
 *         scale is s_k = max_n |x_nk| / 448 in FP32 (s_k = 1 for an all-zero
 *         column).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_F64 = 0, ORC_F32 = 1, ORC_BF16 = 2, ORC_FP8 = 3 };
enum { ORC_LOGISTIC = 0, ORC_POISSON = 1 };

/* ---------------------------------------------------------------- decoding */

double orc_bf16_to_double(uint16_t h) {
    uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

double orc_fp8_to_double(uint8_t q) {
    int sign = (q >> 7) & 1;
    int e = (q >> 3) & 0xF;
    int m = q & 7;
    double v;
    if (e == 0xF && m == 7) return NAN;
    if (e == 0)
        v = ldexp((double)m, -9);               /* subnormal: m * 2^-6 / 8 */
    else
        v = ldexp(1.0 + m / 8.0, e - 7);
    return sign ? -v : v;
}

static double elem(const void* X, int dtype, int64_t idx, const float* scale, int k) {
    switch (dtype) {
    case ORC_F64: return ((const double*)X)[idx];
    case ORC_F32: return (double)((const float*)X)[idx];
    case ORC_BF16: return orc_bf16_to_double(((const uint16_t*)X)[idx]);
    case ORC_FP8: return orc_fp8_to_double(((const uint8_t*)X)[idx]) * (double)scale[k];
    }
    return NAN;
}

/* ------------------------------------------------------- compensated sums */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------- scalar functions */

double orc_softplus(double u) {
    return (u > 0.0 ? u : 0.0) + log1p(exp(-fabs(u)));
}

double orc_sigmoid(double u) {
    if (u >= 0.0) return 1.0 / (1.0 + exp(-u));
    double e = exp(u);
    return e / (1.0 + e);
}

/* ---------------------------------------------------------------- the oracle

 * X: row-major, element (n, k) at X[n * ldx + k] in the storage dtype.
 * scale: K FP32 column scales (FP8 only; ignored otherwise).
 * y: N bytes, each 0 or 1.  beta: K doubles.  mean: K doubles or NULL (zero).
 * out: 1 + K doubles, out[0] = f, out[1 + k] = g_k.
 * Returns 0, or -1 on invalid arguments (K < 1, N < 0, ldx < K, y not 0/1,
 * NULL pointers where data is needed, unknown dtype).
 */
int orc_logpost_grad(const void* X, int dtype, int64_t ldx, const float* scale,
                     const uint8_t* y, int64_t N, int K, const double* beta,
                     double prec, const double* mean, int family, double* out) {
    if (K < 1 || N < 0 || ldx < K || !beta || !out) return -1;
    if (family != ORC_LOGISTIC && family != ORC_POISSON) return -1;
    if (dtype < ORC_F64 || dtype > ORC_FP8) return -1;
    if (N > 0 && (!X || !y)) return -1;
    if (dtype == ORC_FP8 && N > 0 && !scale) return -1;

    nsum f = {0.0, 0.0};
    nsum* g = (nsum*)calloc((size_t)K, sizeof(nsum));
    double* x = (double*)malloc((size_t)K * sizeof(double));
    if (!g || !x) { free(g); free(x); return -1; }

    for (int64_t n = 0; n < N; ++n) {
        if (family == ORC_LOGISTIC && y[n] > 1) { free(g); free(x); return -1; }
        double yn = (double)y[n];
        double u = 0.0;
        for (int k = 0; k < K; ++k) {
            x[k] = elem(X, dtype, n * ldx + k, scale, k);
            u += x[k] * beta[k];
        }
        double t, r;
        if (family == ORC_LOGISTIC) {
            t = yn * u - orc_softplus(u);
            r = yn - orc_sigmoid(u);
        } else {
            /* Poisson with log link: log p(y | u) = y u - exp(u) - log(y!),
             * the last term constant in beta and left out */
            t = yn * u - exp(u);
            r = yn - exp(u);
        }
        nsum_add(&f, t);
        for (int k = 0; k < K; ++k) nsum_add(&g[k], r * x[k]);
    }

    double pf = 0.0;
    for (int k = 0; k < K; ++k) {
        double d = beta[k] - (mean ? mean[k] : 0.0);
        pf += d * d;
        out[1 + k] = nsum_get(&g[k]) - prec * d;
    }
    out[0] = nsum_get(&f) - 0.5 * prec * pf;
    free(g);
    free(x);
    return 0;
}

/* Linear predictor u_n = sum_k x_nk beta_k (FP64, k order), the quantity the
 * differential update (Sec. 3.4.4) keeps resident between steps. */
int orc_linpred(const void* X, int dtype, int64_t ldx, const float* scale, int64_t N, int K,
                const double* beta, double* u) {
    if (K < 1 || N < 0 || ldx < K || !beta) return -1;
    if (dtype < ORC_F64 || dtype > ORC_FP8) return -1;
    if (N > 0 && (!X || !u)) return -1;
    if (dtype == ORC_FP8 && N > 0 && !scale) return -1;
    for (int64_t n = 0; n < N; ++n) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += elem(X, dtype, n * ldx + k, scale, k) * beta[k];
        u[n] = acc;
    }
    return 0;
}

/* Hessian of f: H = -sum_n w_n x_n x_n^t - prec I, with the per-row weight
 * w_n = -d^2 t_n / du^2 = sigmoid(u)(1 - sigmoid(u)) (logistic) or exp(u)
 * (Poisson).  Every entry is a Neumaier-compensated sum over n in ascending
 * order; H is K x K row-major (both triangles written). */
int orc_hessian(const void* X, int dtype, int64_t ldx, const float* scale, int64_t N, int K,
                const double* beta, double prec, int family, double* H) {
    if (K < 1 || N < 0 || ldx < K || !beta || !H) return -1;
    if (family != ORC_LOGISTIC && family != ORC_POISSON) return -1;
    if (N > 0 && !X) return -1;
    nsum* acc = (nsum*)calloc((size_t)K * K, sizeof(nsum));
    double* x = (double*)malloc((size_t)K * sizeof(double));
    if (!acc || !x) { free(acc); free(x); return -1; }
    for (int64_t n = 0; n < N; ++n) {
        double u = 0.0;
        for (int k = 0; k < K; ++k) {
            x[k] = elem(X, dtype, n * ldx + k, scale, k);
            u += x[k] * beta[k];
        }
        double w;
        if (family == ORC_LOGISTIC) {
            double s = orc_sigmoid(u);
            w = s * (1.0 - s);
        } else {
            w = exp(u);
        }
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) nsum_add(&acc[(size_t)i * K + j], w * x[i] * x[j]);
    }
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            H[(size_t)i * K + j] = -nsum_get(&acc[(size_t)i * K + j]) - (i == j ? prec : 0.0);
    free(acc);
    free(x);
    return 0;
}

/* Several evaluation points on one data set: betas and out are b x K and
 * b x (1 + K), row-major; means is b x K or NULL. */
int orc_logpost_grad_multi(const void* X, int dtype, int64_t ldx, const float* scale,
                           const uint8_t* y, int64_t N, int K, const double* betas,
                           int b, double prec, const double* means, int family, double* out) {
    for (int i = 0; i < b; ++i) {
        int rc = orc_logpost_grad(X, dtype, ldx, scale, y, N, K, betas + (int64_t)i * K,
                                  prec, means ? means + (int64_t)i * K : NULL, family,
                                  out + (int64_t)i * (1 + K));
        if (rc) return rc;
    }
    return 0;
}

/* Hierarchical model (Sec. 4.1): group g owns rows offsets[g] .. offsets[g+1]-1
 * of the stacked X and y and its own coefficient vector betas[g*K ..].  The
 * prior mean is shared (K doubles) when mean_per_group == 0, else G x K. */
int orc_logpost_grad_groups(const void* X, int dtype, int64_t ldx, const float* scale,
                            const uint8_t* y, const int64_t* offsets, int G, int K,
                            const double* betas, double prec, const double* mean,
                            int mean_per_group, int family, double* out) {
    size_t es = dtype == ORC_F64 ? 8 : dtype == ORC_F32 ? 4 : dtype == ORC_BF16 ? 2 : 1;
    for (int g = 0; g < G; ++g) {
        int64_t a = offsets[g], b = offsets[g + 1];
        if (b < a) return -1;
        const char* Xg = (const char*)X + (size_t)(a * ldx) * es;
        const double* mg = mean ? (mean_per_group ? mean + (int64_t)g * K : mean) : NULL;
        int rc = orc_logpost_grad(Xg, dtype, ldx, scale, y + a, b - a, K,
                                  betas + (int64_t)g * K, prec, mg, family,
                                  out + (int64_t)g * (1 + K));
        if (rc) return rc;
    }
    return 0;
}

/* ----------------------------------------------------------------- encoders */

uint16_t orc_bf16_from_float(float v) {
    uint32_t bits;
    memcpy(&bits, &v, 4);
    if ((bits & 0x7F800000u) == 0x7F800000u && (bits & 0x007FFFFFu))
        return (uint16_t)((bits >> 16) | 0x0040u);        /* quiet NaN */
    uint32_t keep = bits >> 16, rest = bits & 0xFFFFu;
    if (rest > 0x8000u || (rest == 0x8000u && (keep & 1u))) keep += 1u;
    return (uint16_t)keep;
}

/* Nearest FP8 E4M3FN code to v (ties to even), saturating at +-448. */
uint8_t orc_fp8_from_float(float v) {
    if (isnan(v)) return 0x7F;
    uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs((double)v);
    if (a >= 448.0) return sign | 0x7E;
    if (a < ldexp(1.0, -6)) {                  /* subnormal range: steps of 2^-9 */
        double m = nearbyint(ldexp(a, 9));     /* 0 .. 8; 8 is the smallest normal */
        return sign | (uint8_t)m;
    }
    int e2;
    double fr = frexp(a, &e2);                 /* a = fr * 2^e2, fr in [0.5, 1) */
    int e = e2 - 1;                            /* a = (2 fr) * 2^e, 2 fr in [1, 2) */
    double m = nearbyint((2.0 * fr - 1.0) * 8.0);
    if (m == 8.0) { m = 0.0; e += 1; }
    if (e + 7 > 15 || (e + 7 == 15 && m == 7.0)) return sign | 0x7E;
    return sign | (uint8_t)(((e + 7) << 3) | (int)m);
}

int orc_quantize_bf16(const float* X, int64_t N, int K, int64_t ldx,
                      uint16_t* Q, int64_t ldq) {
    if (K < 1 || N < 0 || ldx < K || ldq < K) return -1;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) Q[n * ldq + k] = orc_bf16_from_float(X[n * ldx + k]);
    return 0;
}

int orc_fp8_col_scales(const float* X, int64_t N, int K, int64_t ldx, float* scale) {
    if (K < 1 || N < 0 || ldx < K) return -1;
    /* scale[] first holds the running column maxima (rows in storage order) */
    for (int k = 0; k < K; ++k) scale[k] = 0.0f;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            float a = fabsf(X[n * ldx + k]);
            if (a > scale[k]) scale[k] = a;
        }
    for (int k = 0; k < K; ++k) scale[k] = scale[k] > 0.0f ? scale[k] / 448.0f : 1.0f;
    return 0;
}

int orc_quantize_fp8(const float* X, int64_t N, int K, int64_t ldx,
                     const float* scale, uint8_t* Q, int64_t ldq) {
    if (K < 1 || N < 0 || ldx < K || ldq < K) return -1;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            float v = X[n * ldx + k] / scale[k];
            Q[n * ldq + k] = orc_fp8_from_float(v);
        }
    return 0;
}

/* ------------------------------------------------------------ random numbers
 *
 * Philox4x64-10, the counter-based generator of J. K. Salmon, M. A. Moraes,
 * R. O. Dror and D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11), written from its published definition: the output block is a keyed
 * bijection of a four-word counter.  Each of the ten rounds forms the 128-bit
 * products of counter words 0 and 2 with two fixed odd multipliers and
 * recombines them as (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
 * lo(M0 x0)); between rounds the two key words are advanced by Weyl constants
 * (the golden ratio and sqrt(3) - 1 in 64-bit fixed point). */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL, PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL, PHILOX_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        const unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        const uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform in (0, 1) from a 64-bit word: its top 52 bits plus one half, times
 * 2^-52; every step is exact in double, and the result lies in
 * [2^-53, 1 - 2^-53]. */
double orc_u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1.0p-52; }

/* Standard normals by Marsaglia's polar method (G. Marsaglia and T. A. Bray,
 * "A convenient method for generating normal variables", SIAM Review 6,
 * 1964): a point (u, v) uniform in the square (-1, 1)^2 is accepted when
 * 0 < s = u^2 + v^2 < 1, and then u c and v c with c = sqrt(-2 log(s) / s)
 * are two independent standard normals.  Pair p of a stream takes its
 * attempts a = 0, 1, ... from the blocks at counter (p, a / 2, purpose,
 * stream), words 2 (a mod 2) and 2 (a mod 2) + 1; s is formed as
 * fma(u, u, v v) so that the acceptance test is a fixed function of the
 * bits.  Writes z[0..1]; returns the attempts used. */
int orc_polar_pair(uint64_t seed, uint64_t chain, uint64_t purpose, uint64_t stream, uint64_t p,
                   double z[2]) {
    const uint64_t key[2] = {seed, chain};
    z[0] = z[1] = 0.0;
    /* at most 256 attempts: all miss the disc with probability below 10^-170,
       and such a pair is (0, 0) */
    for (int a = 0; a < 256; ++a) {
        const uint64_t ctr[4] = {p, (uint64_t)(a >> 1), purpose, stream};
        uint64_t w[4];
        orc_philox4x64_10(ctr, key, w);
        const double u = 2.0 * orc_u01(w[2 * (a & 1)]) - 1.0;
        const double v = 2.0 * orc_u01(w[2 * (a & 1) + 1]) - 1.0;
        const double s = fma(u, u, v * v);
        if (s > 0.0 && s < 1.0) {
            const double c = sqrt(-2.0 * log(s) / s);
            z[0] = u * c;
            z[1] = v * c;
            return a + 1;
        }
    }
    return 256;
}
