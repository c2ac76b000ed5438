/*
 * zmc_oracle.c -- serial FP64 CPU oracle for multi-function direct Monte Carlo.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant
 * generator with the GPU library: it defines its own copy of the function-table
 * layout (the input format is the only thing the two sides have in common) and
 * its own random-number generator, written from the published definitions.
 *
 * What it computes (paper, "Solution method"): each integrand is integrated by
 * direct Monte Carlo over its own box, independently of the others
 * ("Multi-function Integrations", Eq. (1) and Eq. (2): integrands that differ
 * in form, dimension and domain).  For N uniform samples x_i in the box,
 *
 *     F_hat = V * (1/N) * sum_i f(x_i),      V = prod_j (hi_j - lo_j),
 *     s^2   = (sum f^2 - (sum f)^2 / N) / (N - 1),
 *     SE    = V * sqrt(s^2 / N).
 *
 * The paper gives a value with an error bar for every integral (Fig. 1
 * caption); it is silent on the random-number generator, the uniform
 * construction and the variance denominator.  Readings taken here:
 *
 *   RNG      Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 *            numbers: as easy as 1, 2, 3", SC'11).  Key = (seed mod 2^32,
 *            seed >> 32).  Samples are taken four at a time: sample i is
 *            member s = i mod 4 of quad q = i / 4, and its coordinate j is
 *            output word s of the Philox block with counter
 *            (b mod 2^32, b >> 32, 0, 0), b = q*d + j.  A quad uses exactly
 *            d blocks and no output word is wasted; equivalently coordinate j
 *            of sample i is word g = 4*(q*d + j) + s of the function's stream.
 *   Uniform  u = (2*(r mod 2^23) + 1) * 2^-24 from a 32-bit word r: the
 *            midpoints of a 2^23 grid, strictly inside (0, 1), exact in FP32
 *            and FP64.
 *   Mapping  x_j = fma(hi_j - lo_j, u_j, lo_j).
 *   Variance unbiased (N - 1), clamped at zero.
 *
 * Integrand formulas, evaluated in this fixed order with explicit fma:
 *   HARMONIC      (Eq. 1)   theta = sum_j k_j x_j;  f = a cos(theta) + b sin(theta)
 *   ABS_LINEAR    (Eq. 2)   s = c0 + sum_j c_j x_j; f = a |s|
 *   GAUSSIAN                q = sum_j (x_j - mu_j)^2; f = A exp(-q / (2 sigma^2))
 *   POLY_PRODUCT            f = prod_j (1 + p_j x_j^{d_j}), integer d_j >= 0
 *
 * Sums use Neumaier's compensated summation so that the oracle is the more
 * accurate side of every comparison.  Threads only ever split the work
 * *across* functions; each function's sum is serial and deterministic.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DIM 12
#define ORC_N_PARAMS 32
#define ORC_V0 2
#define ORC_W0 (2 + ORC_MAX_DIM)

enum { ORC_HARMONIC = 0, ORC_ABS_LINEAR = 1, ORC_GAUSSIAN = 2, ORC_POLY_PRODUCT = 3 };

/* One integrand, 472 bytes: the input table format. */
typedef struct {
    uint32_t family;
    uint32_t dim;
    uint64_t n_samples;
    uint64_t seed;
    double lo[ORC_MAX_DIM];
    double hi[ORC_MAX_DIM];
    double params[ORC_N_PARAMS];
} orc_function;

/* Per-function result. */
typedef struct {
    double mean;     /* F_hat */
    double stderr_;  /* SE */
    double sum_f;    /* S1 = sum f (compensated) */
    double sum_f2;   /* S2 = sum f^2 (compensated) */
    double sum_abs;  /* A = sum |f| (compensated), the scale of S1's rounding */
    double volume;   /* V */
    uint64_t n;
    int32_t status;  /* 0 ok, <0 invalid input */
    int32_t pad;
} orc_result;

/* ---------------- Philox4x32-10 (SC'11 definition) ---------------- */

static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

/* One Philox4x32 round: two 32x32->64 products, the high halves are xored with
 * the other two counter words and the round key, and the words are permuted. */
static void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k0, k1);
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ---------------- uniform, sample point ---------------- */

double orc_uniform(uint32_t r)
{
    /* (2m + 1) * 2^-24 with m = r mod 2^23: exact in double. */
    uint32_t m = r & 0x7FFFFFu;
    return ldexp((double)(2u * m + 1u), -24);
}

/* The 32-bit word that coordinate j of sample i draws. */
uint32_t orc_word(uint64_t seed, uint32_t dim, uint64_t i, uint32_t j)
{
    uint64_t q = i / 4u;                       /* quad */
    uint32_t s = (uint32_t)(i % 4u);           /* member of the quad */
    uint64_t b = q * (uint64_t)dim + (uint64_t)j;
    uint32_t ctr[4] = {(uint32_t)b, (uint32_t)(b >> 32), 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[s];
}

void orc_sample_point(const orc_function* fn, uint64_t i, double* x)
{
    for (uint32_t j = 0; j < fn->dim; ++j) {
        double u = orc_uniform(orc_word(fn->seed, fn->dim, i, j));
        double w = fn->hi[j] - fn->lo[j];
        x[j] = fma(w, u, fn->lo[j]);
    }
}

/* Points of samples [i0, i0 + count) of one function, row-major (count x dim):
 * the same samples as above, for integrands evaluated outside this file (the
 * run-time compiled families, whose formula the caller supplies). */
void orc_sample_points(const orc_function* fn, uint64_t i0, uint64_t count, double* out)
{
    for (uint64_t k = 0; k < count; ++k) orc_sample_point(fn, i0 + k, out + k * fn->dim);
}

/* ---------------- integrands ---------------- */

double orc_eval(const orc_function* fn, const double* x)
{
    const double* p = fn->params;
    const uint32_t d = fn->dim;
    switch (fn->family) {
    case ORC_HARMONIC: { /* Eq. (1) */
        double theta = 0.0;
        for (uint32_t j = 0; j < d; ++j) theta = fma(p[ORC_V0 + j], x[j], theta);
        return fma(p[0], cos(theta), p[1] * sin(theta));
    }
    case ORC_ABS_LINEAR: { /* Eq. (2) */
        double s = p[1];
        for (uint32_t j = 0; j < d; ++j) s = fma(p[ORC_V0 + j], x[j], s);
        return p[0] * fabs(s);
    }
    case ORC_GAUSSIAN: {
        double q = 0.0;
        for (uint32_t j = 0; j < d; ++j) {
            double t = x[j] - p[ORC_V0 + j];
            q = fma(t, t, q);
        }
        double h = 0.5 / (p[1] * p[1]);
        return p[0] * exp(-q * h);
    }
    case ORC_POLY_PRODUCT: {
        double prod = 1.0;
        for (uint32_t j = 0; j < d; ++j) {
            int deg = (int)p[ORC_W0 + j];
            double xp = 1.0;
            for (int e = 0; e < deg; ++e) xp *= x[j];
            prod *= fma(p[ORC_V0 + j], xp, 1.0);
        }
        return prod;
    }
    default:
        return NAN;
    }
}

/* ---------------- validation ---------------- */

int orc_validate(const orc_function* fn)
{
    if (fn->family > ORC_POLY_PRODUCT) return -2;
    if (fn->dim < 1 || fn->dim > ORC_MAX_DIM) return -3;
    if (fn->n_samples < 2) return -1;
    for (uint32_t j = 0; j < fn->dim; ++j) {
        if (!isfinite(fn->lo[j]) || !isfinite(fn->hi[j]) || !(fn->lo[j] < fn->hi[j])) return -4;
    }
    for (uint32_t j = 0; j < ORC_N_PARAMS; ++j)
        if (!isfinite(fn->params[j])) return -5;
    if (fn->family == ORC_GAUSSIAN && !(fn->params[1] > 0.0)) return -5;
    if (fn->family == ORC_POLY_PRODUCT) {
        for (uint32_t j = 0; j < fn->dim; ++j) {
            double dg = fn->params[ORC_W0 + j];
            if (!(dg >= 0.0 && dg <= 8.0 && dg == floor(dg))) return -5;
        }
    }
    return 0;
}

/* ---------------- Neumaier compensated sum ---------------- */

typedef struct { double s, c; } orc_sum;

static void nsum_add(orc_sum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const orc_sum* a) { return a->s + a->c; }

/* ---------------- one function ---------------- */

/* Direct MC over samples [i0, i1) of one function; raw compensated sums. */
void orc_partial_sums(const orc_function* fn, uint64_t i0, uint64_t i1,
                      double* s1, double* s2, double* sabs)
{
    orc_sum a1 = {0, 0}, a2 = {0, 0}, aa = {0, 0};
    double x[ORC_MAX_DIM];
    for (uint64_t i = i0; i < i1; ++i) {
        orc_sample_point(fn, i, x);
        double f = orc_eval(fn, x);
        nsum_add(&a1, f);
        nsum_add(&a2, f * f);
        nsum_add(&aa, fabs(f));
    }
    *s1 = nsum_value(&a1);
    *s2 = nsum_value(&a2);
    *sabs = nsum_value(&aa);
}

double orc_volume(const orc_function* fn)
{
    double v = 1.0;
    for (uint32_t j = 0; j < fn->dim; ++j) v *= (fn->hi[j] - fn->lo[j]);
    return v;
}

/* Mean and standard error from the sums (direct MC estimator). */
void orc_finalize(double volume, uint64_t n, double s1, double s2, double* mean, double* se)
{
    double dn = (double)n;
    double var = (s2 - s1 * s1 / dn) / (dn - 1.0);
    if (!(var > 0.0)) var = 0.0;
    *mean = volume * (s1 / dn);
    *se = volume * sqrt(var / dn);
}

int orc_integrate(const orc_function* fn, orc_result* out)
{
    memset(out, 0, sizeof(*out));
    int st = orc_validate(fn);
    out->status = st;
    if (st != 0) return st;
    double s1, s2, sa;
    orc_partial_sums(fn, 0, fn->n_samples, &s1, &s2, &sa);
    out->sum_f = s1;
    out->sum_f2 = s2;
    out->sum_abs = sa;
    out->n = fn->n_samples;
    out->volume = orc_volume(fn);
    orc_finalize(out->volume, out->n, s1, s2, &out->mean, &out->stderr_);
    return 0;
}

/* ---------------- many functions, threads across functions only ---------------- */

typedef struct {
    const orc_function* fns;
    orc_result* out;
    size_t n;
    size_t next;
    pthread_mutex_t lock;
} orc_pool;

static void* orc_worker(void* arg)
{
    orc_pool* pool = (orc_pool*)arg;
    for (;;) {
        pthread_mutex_lock(&pool->lock);
        size_t i = pool->next++;
        pthread_mutex_unlock(&pool->lock);
        if (i >= pool->n) break;
        orc_integrate(&pool->fns[i], &pool->out[i]);
    }
    return NULL;
}

/* Integrate n functions with up to n_threads threads; returns the thread count used. */
int orc_integrate_batch(const orc_function* fns, size_t n, orc_result* out, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if ((size_t)n_threads > n) n_threads = (int)(n > 0 ? n : 1);
    orc_pool pool;
    pool.fns = fns;
    pool.out = out;
    pool.n = n;
    pool.next = 0;
    pthread_mutex_init(&pool.lock, NULL);
    if (n_threads == 1) {
        orc_worker(&pool);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
        int started = 0;
        for (int t = 0; t < n_threads; ++t)
            if (pthread_create(&th[t], NULL, orc_worker, &pool) == 0) ++started;
        if (started == 0) orc_worker(&pool);
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
        n_threads = started > 0 ? started : 1;
    }
    pthread_mutex_destroy(&pool.lock);
    return n_threads;
}

size_t orc_sizeof_function(void) { return sizeof(orc_function); }
size_t orc_sizeof_result(void) { return sizeof(orc_result); }
