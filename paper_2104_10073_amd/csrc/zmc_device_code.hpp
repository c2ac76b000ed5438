// zmc_device_code.hpp -- device code of the multi-function direct Monte Carlo path.
//
// Shared by the built-in kernels (zmc_kernels.hip) and by the kernels compiled at
// run time for caller-supplied integrands (hipRTC, zmc_host.hip), so both run
// the same sampling, accumulation and reduction code.
//
// Per sample (paper, "Solution method": direct Monte Carlo per integrand):
//   1. counter-based uniforms: Philox4x32-10 (SC'11) in registers;
//   2. mapping into the function's box;
//   3. the integrand (Eq. (1) harmonic, Eq. (2) |linear|, Gaussian, product
//      polynomial, or a caller's function);
//   4. compensated per-lane sums of f and f^2;
// then per segment a fixed 64-lane butterfly in FP64, per tile an LDS tree over
// its segments, and per function an atomic-free FP64 finalize pass giving the
// mean and standard error.  No MFMA: nothing here is a dense contraction; the
// bound is VALU issue (integer multiplies of Philox, FP32 FMAs, transcendentals).
//
// Sample layout.  Samples are handled four at a time (a quad): quad q of a
// d-dimensional function uses Philox blocks q*d .. q*d + d - 1, and block
// q*d + j holds coordinate j of the quad's four samples, one per output word.
#pragma once

#include "zmc_device.hpp"

namespace zmc {

// ---------------------------------------------------------------- Philox4x32-10

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // a ^ b ^ c in one VALU op
}

// Block at counter (b_lo, b_hi, 0, 0).  The two zero counter words make the first
// round a single product and the second round's first xor two-input; from the
// third round on every round is two 32x32->64 products and two 3-input xors.
// Round keys are wave-uniform and stay in scalar registers.
__device__ __forceinline__ void philox_block(uint32_t b_lo, uint32_t b_hi, uint32_t k0, uint32_t k1,
                                             uint32_t out[4])
{
    uint32_t c0, c1, c2, c3;
    {   // first Philox round: c2 = c3 = 0
        const uint64_t p0 = (uint64_t)kPhiloxM0 * b_lo;
        c0 = b_hi ^ k0;
        c1 = 0u;
        c2 = (uint32_t)(p0 >> 32) ^ k1;
        c3 = (uint32_t)p0;
    }
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    {   // second Philox round: c1 = 0
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ k0;
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// The same block at counter (b, 0, 0, 0), for functions whose block indices fit
// in 32 bits.  With the counter's second word zero, the first round leaves
// c0 = k0 and c1 = 0, so the second round's first product M0 * k0 and the xor
// terms it feeds are wave-uniform: they are formed on the scalar unit, and
// every VALU xor takes at most one scalar operand (gfx950 reads one scalar
// operand per vector instruction; a second would cost a copy).
__device__ __forceinline__ void philox_block_narrow(uint32_t b, uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0, c1, c2, c3;
    // first round: counter (b, 0, 0, 0)
    const uint64_t p = (uint64_t)kPhiloxM0 * b;
    c2 = (uint32_t)(p >> 32) ^ k1;
    c3 = (uint32_t)p;
    // second round: counter (k0, 0, c2, c3); M0 * k0 is wave-uniform
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    const uint64_t u = (uint64_t)kPhiloxM0 * (k0 - kPhiloxW0);
    const uint32_t u_hi_k1 = (uint32_t)(u >> 32) ^ k1;
    const uint32_t u_lo = (uint32_t)u;
    {
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        c0 = (uint32_t)(p1 >> 32) ^ k0;
        c1 = (uint32_t)p1;
        c2 = c3 ^ u_hi_k1;
    }
    // third round: c3 = u_lo is wave-uniform
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    {
        const uint32_t lo_k1 = u_lo ^ k1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ lo_k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// ---------------------------------------------------------------- function records

// Function records are read-only while kernels run.  Reading them through the
// constant address space turns every wave-uniform field access into a scalar
// load (scalar cache, scalar registers) instead of 64 identical vector loads.
typedef const __attribute__((address_space(4))) DevFn CDevFn;

__device__ __forceinline__ CDevFn* scalar_view(const DevFn* p)
{
    return (CDevFn*)(uintptr_t)p;
}

// ---------------------------------------------------------------- uniforms

// t = 1 + m 2^-23 in [1, 2) from the low 23 bits m of a word: one VALU op.
// The uniform of the definition is u = t - (1 - 2^-24) exactly.
__device__ __forceinline__ float word_to_t(uint32_t r)
{
    return __uint_as_float((r & 0x007FFFFFu) | 0x3F800000u);
}

constexpr float kTShift = 0x1.fffffep-1f;  // 1 - 2^-24

// u = (2 m + 1) 2^-24 in FP64, exact.
__device__ __forceinline__ double word_to_u64(uint32_t r)
{
    return (double)(((r & 0x007FFFFFu) << 1) | 1u) * 0x1p-24;
}

// One quad of samples whose first Philox block is b0 = q*d: blocks b0 .. b0 + d - 1,
// block b0 + j giving coordinate j of the four samples, folded into the samples'
// states as soon as it is produced (the built-in families need no more than one
// state per sample).  B is uint32_t when every block index of the function fits
// in 32 bits: the counter's second word is then the constant 0, which makes part
// of the first two Philox rounds wave-uniform (scalar) work; otherwise uint64_t.
template <class B>
__device__ __forceinline__ void philox_at(B b, uint32_t k0, uint32_t k1, uint32_t w[4])
{
    if constexpr (sizeof(B) == 4) philox_block_narrow(b, k0, k1, w);
    else philox_block((uint32_t)b, (uint32_t)(b >> 32), k0, k1, w);
}

template <class Ev, class T, class B>
__device__ __forceinline__ void stream_quad(const Ev& ev, uint32_t d, uint32_t k0, uint32_t k1, B b0, T g[4])
{
    T st[4];
    uint32_t w[4];
    philox_at<B>(b0, k0, k1, w);
    ev.first(st, w);  // d >= 1
    for (uint32_t j = 1; j < d; ++j) {
        philox_at<B>(b0 + j, k0, k1, w);
        ev.add(st, j, w);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) g[s] = ev.finish(st[s]);
}

// ---------------------------------------------------------------- FP32 integrands

// An evaluator holds a function (wave-uniform pointer) and works on the four
// samples of a quad: first(st, w) sets their states from coordinate 0 (the
// state an empty sum would start from, folded into the first operation), add(st,
// j, w) folds coordinate j from the block's four words, finish() returns g with
// f = scale1 * g (scale1
// and scale2 = scale1^2 are applied in FP64 at finalize).  Coefficients were
// derived on the host in FP64 and rounded once; they are read with scalar loads.

template <int FAM> struct Eval32;

// Eq. (1): a cos(theta) + b sin(theta) = R cos(theta - phi).  The phase in
// revolutions is f0 + sum_j kappa_j t_j; v_fract + v_cos_f32 (which computes
// cos(2 pi x)) give the cosine: one transcendental per sample.
template <> struct Eval32<HARMONIC> {
    CDevFn* fn;
    typedef float Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t d, uint32_t k0, uint32_t k1, B b0, float g[4]) const
    {
        stream_quad(*this, d, k0, k1, b0, g);
    }
    __device__ __forceinline__ void first(float st[4], const uint32_t w[4]) const
    {
        const float c = fn->fc[0], f0 = fn->f0;
#pragma unroll
        for (int s = 0; s < 4; ++s) st[s] = fmaf(c, word_to_t(w[s]), f0);
    }
    __device__ __forceinline__ void add(float st[4], uint32_t j, const uint32_t w[4]) const
    {
        const float c = fn->fc[j];
#pragma unroll
        for (int s = 0; s < 4; ++s) st[s] = fmaf(c, word_to_t(w[s]), st[s]);
    }
    __device__ __forceinline__ float finish(float th) const
    {
        return __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(th));
    }
};

// Eq. (2): a |c0 + c.x|; the offset is carried as a two-float sum so the
// hyperplane is placed to FP64 accuracy.
template <> struct Eval32<ABS_LINEAR> {
    CDevFn* fn;
    typedef float Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t d, uint32_t k0, uint32_t k1, B b0, float g[4]) const
    {
        stream_quad(*this, d, k0, k1, b0, g);
    }
    __device__ __forceinline__ void first(float st[4], const uint32_t w[4]) const
    {
        const float c = fn->fc[0], f0 = fn->f0;
#pragma unroll
        for (int s = 0; s < 4; ++s) st[s] = fmaf(c, word_to_t(w[s]), f0);
    }
    __device__ __forceinline__ void add(float st[4], uint32_t j, const uint32_t w[4]) const
    {
        const float c = fn->fc[j];
#pragma unroll
        for (int s = 0; s < 4; ++s) st[s] = fmaf(c, word_to_t(w[s]), st[s]);
    }
    __device__ __forceinline__ float finish(float st) const { return fabsf(st + fn->f0lo); }
};

// A exp(-|x - mu|^2 / (2 sigma^2)) = A 2^(-sum_j (c_j (t_j - m_j))^2); t - m is
// exact (both in [1, 2] for a centre inside the box), v_exp_f32 computes 2^x.
template <> struct Eval32<GAUSSIAN> {
    CDevFn* fn;
    typedef float Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t d, uint32_t k0, uint32_t k1, B b0, float g[4]) const
    {
        stream_quad(*this, d, k0, k1, b0, g);
    }
    __device__ __forceinline__ void first(float st[4], const uint32_t w[4]) const
    {
        const float c = fn->fc[0], m = fn->fo[0];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float y = c * (word_to_t(w[s]) - m);
            st[s] = fmaf(y, y, 0.0f);
        }
    }
    __device__ __forceinline__ void add(float st[4], uint32_t j, const uint32_t w[4]) const
    {
        const float c = fn->fc[j], m = fn->fo[j];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float y = c * (word_to_t(w[s]) - m);
            st[s] = fmaf(y, y, st[s]);
        }
    }
    __device__ __forceinline__ float finish(float q) const { return __builtin_amdgcn_exp2f(-q); }
};

// prod_j (1 + p_j x_j^{n_j}), x_j = lo_j + w_j u_j with u_j = t_j - (1 - 2^-24)
// exact; the power is a wave-uniform loop shared by the quad's four samples.
template <> struct Eval32<POLY_PRODUCT> {
    CDevFn* fn;
    typedef float Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t d, uint32_t k0, uint32_t k1, B b0, float g[4]) const
    {
        stream_quad(*this, d, k0, k1, b0, g);
    }
    __device__ __forceinline__ void factors(uint32_t j, const uint32_t w[4], float fac[4]) const
    {
        const float c = fn->fc[j], o = fn->fo[j], p = fn->fp[j];
        const int e = fn->deg[j] < kMaxPolyDegree ? fn->deg[j] : kMaxPolyDegree;  // bounded whatever the record holds
        float x[4], xp[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            x[s] = fmaf(c, word_to_t(w[s]) - kTShift, o);
            xp[s] = 1.0f;
        }
        for (int k = 0; k < e; ++k) {
#pragma unroll
            for (int s = 0; s < 4; ++s) xp[s] *= x[s];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) fac[s] = fmaf(p, xp[s], 1.0f);
    }
    __device__ __forceinline__ void first(float st[4], const uint32_t w[4]) const { factors(0, w, st); }
    __device__ __forceinline__ void add(float st[4], uint32_t j, const uint32_t w[4]) const
    {
        float fac[4];
        factors(j, w, fac);
#pragma unroll
        for (int s = 0; s < 4; ++s) st[s] *= fac[s];
    }
    __device__ __forceinline__ float finish(float g) const { return g; }
};

// ---------------------------------------------------------------- FP64 integrands

// The definition in its reference operation order (explicit fma), FP64 libm.
template <int FAM> struct Eval64 {
    CDevFn* fn;
    typedef double Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t d, uint32_t k0, uint32_t k1, B b0, double g[4]) const
    {
        stream_quad(*this, d, k0, k1, b0, g);
    }
    __device__ __forceinline__ void first(double st[4], const uint32_t w[4]) const
    {
        double v = 0.0;
        if constexpr (FAM == ABS_LINEAR) v = fn->s1;
        if constexpr (FAM == POLY_PRODUCT) v = 1.0;
        for (int s = 0; s < 4; ++s) st[s] = v;
        add(st, 0, w);
    }
    __device__ __forceinline__ void add(double st[4], uint32_t j, const uint32_t w[4]) const
    {
        const double lo = fn->lo[j], wd = fn->w[j], v = fn->v[j];
        double x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) x[s] = fma(wd, word_to_u64(w[s]), lo);
        if constexpr (FAM == HARMONIC || FAM == ABS_LINEAR) {
#pragma unroll
            for (int s = 0; s < 4; ++s) st[s] = fma(v, x[s], st[s]);
        } else if constexpr (FAM == GAUSSIAN) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double t = x[s] - v;
                st[s] = fma(t, t, st[s]);
            }
        } else {
            const int e = fn->deg[j] < kMaxPolyDegree ? fn->deg[j] : kMaxPolyDegree;  // bounded whatever the record holds
            double xp[4] = {1.0, 1.0, 1.0, 1.0};
            for (int k = 0; k < e; ++k) {
#pragma unroll
                for (int s = 0; s < 4; ++s) xp[s] *= x[s];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) st[s] *= fma(v, xp[s], 1.0);
        }
    }
    __device__ __forceinline__ double finish(double st) const
    {
        if constexpr (FAM == HARMONIC) {
            double sn, cs;
            sincos(st, &sn, &cs);
            return fma(fn->s0, cs, fn->s1 * sn);
        } else if constexpr (FAM == ABS_LINEAR) {
            return fn->s0 * fabs(st);
        } else if constexpr (FAM == GAUSSIAN) {
            return fn->s0 * exp(-st * fn->h);
        } else {
            return st;
        }
    }
};

// ---------------------------------------------------------------- reductions

// Fixed xor butterfly: level m pairs lanes l and l^m, so the result is the
// pairwise tree over lane order and every lane holds the same bits.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// ---------------------------------------------------------------- one segment

// Lane sums over the lane's 16 quads of one segment, quads quad0 + 64 k; b0 is
// the first Philox block of the lane's current quad, advanced by 64 d per quad.
// TAIL marks a segment that can hold quads or samples past N (the function's
// last one, or any segment of a function whose block indices need 64 bits).
template <bool TAIL, class B, class Ev>
__device__ __forceinline__ void segment_fp32(const Ev& ev, uint32_t d, uint32_t k0, uint32_t k1,
                                             uint64_t quad0, uint64_t n_quads, uint64_t n_samples,
                                             double& out1, double& out2)
{
    float s1 = 0.0f, c1 = 0.0f, s2 = 0.0f, c2 = 0.0f;
    B b0 = (B)(quad0 * d);
    const B step = (B)kWave * (B)d;
#pragma unroll 1
    for (int k = 0; k < kQuadsPerLane; ++k, b0 += step) {
        const uint64_t q = quad0 + (uint64_t)(k * kWave);
        if (TAIL && q >= n_quads) break;
        float g[4];
        ev.quad(d, k0, k1, b0, g);
        if (TAIL) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (4 * q + (uint64_t)s >= n_samples) g[s] = 0.0f;
        }
        const float a1 = (g[0] + g[1]) + (g[2] + g[3]);
        const float a2 = fmaf(g[1], g[1], g[0] * g[0]) + fmaf(g[3], g[3], g[2] * g[2]);
        kahan_add(s1, c1, a1);
        kahan_add(s2, c2, a2);
    }
    out1 = (double)s1 - (double)c1;
    out2 = (double)s2 - (double)c2;
}

template <bool TAIL, class B, class Ev>
__device__ __forceinline__ void segment_fp64(const Ev& ev, uint32_t d, uint32_t k0, uint32_t k1,
                                             uint64_t quad0, uint64_t n_quads, uint64_t n_samples,
                                             double& out1, double& out2)
{
    double s1 = 0.0, s2 = 0.0;
    B b0 = (B)(quad0 * d);
    const B step = (B)kWave * (B)d;
#pragma unroll 1
    for (int k = 0; k < kQuadsPerLane; ++k, b0 += step) {
        const uint64_t q = quad0 + (uint64_t)(k * kWave);
        if (TAIL && q >= n_quads) break;
        double f[4];
        ev.quad(d, k0, k1, b0, f);
        if (TAIL) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (4 * q + (uint64_t)s >= n_samples) f[s] = 0.0;
        }
        s1 += (f[0] + f[1]) + (f[2] + f[3]);
        s2 += (f[0] * f[0] + f[1] * f[1]) + (f[2] * f[2] + f[3] * f[3]);
    }
    out1 = s1;
    out2 = s2;
}

template <bool TAIL, class B, class Ev>
__device__ __forceinline__ void segment_sums(const Ev& ev, uint32_t d, uint32_t k0, uint32_t k1, uint64_t quad0,
                                             uint64_t n_quads, uint64_t n_samples, double& out1, double& out2)
{
    if constexpr (sizeof(typename Ev::Value) == 8)
        segment_fp64<TAIL, B>(ev, d, k0, k1, quad0, n_quads, n_samples, out1, out2);
    else
        segment_fp32<TAIL, B>(ev, d, k0, k1, quad0, n_quads, n_samples, out1, out2);
}

// ---------------------------------------------------------------- one tile

// Wave `wave` of the workgroup evaluates segments seg0 + wave*2^L + i, i < 2^L,
// and leaves each segment's (S1, S2) in LDS slot wave*2^L + i (zero past the
// function's last segment).  All arguments are wave-uniform.
template <class Ev>
__device__ __forceinline__ void tile_segments(CDevFn* fn, uint32_t seg0, uint32_t seg_log2, uint32_t wave,
                                              uint32_t lane, Partial* s_seg)
{
    const uint32_t per_wave = 1u << seg_log2;
    const uint32_t n_seg = fn->n_segments;
    const uint64_t n_quads = fn->n_quads;
    const uint64_t n_samples = fn->n_samples;
    const uint32_t d = fn->dim;
    const uint32_t k0 = fn->key0, k1 = fn->key1;
    const uint32_t first = seg0 + wave * per_wave;
    // every block index q*d + j of the function below 2^32: 32-bit counters
    const bool narrow = n_quads * (uint64_t)d <= 0x100000000ull;
    const Ev ev{fn};
    for (uint32_t i = 0; i < per_wave; ++i) {
        const uint32_t seg = first + i;
        double a = 0.0, b = 0.0;
        if (seg < n_seg) {
            const uint64_t quad0 = (uint64_t)seg * kSegQuads + lane;
            const bool tail = (uint64_t)(seg + 1) * kSegSamples > n_samples;
            if (!narrow)
                segment_sums<true, uint64_t>(ev, d, k0, k1, quad0, n_quads, n_samples, a, b);
            else if (tail)
                segment_sums<true, uint32_t>(ev, d, k0, k1, quad0, n_quads, n_samples, a, b);
            else
                segment_sums<false, uint32_t>(ev, d, k0, k1, quad0, n_quads, n_samples, a, b);
            a = wave_sum(a);
            b = wave_sum(b);
        }
        if (lane == 0) s_seg[wave * per_wave + i] = Partial{a, b};
    }
}

// How tile partials are read and written.  The launch path's kernels use
// ordinary loads and stores (a kernel boundary separates the writers from the
// readers).  The resident kernel, whose workgroups hand partials to each other
// within one launch, writes them through to memory and reads them past every
// cache (system-scope atomics), so no line of them is ever dirty or stale in
// any XCD's L2 and no cache maintenance is needed per tile.
struct PlainMem {
    __device__ static __forceinline__ Partial load(const Partial* p) { return *p; }
    __device__ static __forceinline__ void store(Partial* p, const Partial& v) { *p = v; }
    __device__ static __forceinline__ void sync() {}
};

struct CoherentMem {
    __device__ static __forceinline__ Partial load(const Partial* p)
    {
        const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
        const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return Partial{__longlong_as_double((long long)a), __longlong_as_double((long long)b)};
    }
    __device__ static __forceinline__ void store(Partial* p, const Partial& v)
    {
        uint64_t* q = reinterpret_cast<uint64_t*>(p);
        __hip_atomic_store(q, (uint64_t)__double_as_longlong(v.s1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(q + 1, (uint64_t)__double_as_longlong(v.s2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // the wave's stores have completed (every lane's later loads see them)
    __device__ static __forceinline__ void sync()
    {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
};

// Pairwise tree over the tile's 4 * 2^L segment sums (L <= 6, so at most 4 per lane),
// then the lane butterfly: the same tree as over the whole function.
template <class Mem = PlainMem>
__device__ __forceinline__ void tile_tree(const Partial* s_seg, uint32_t count, uint32_t lane, Partial* out)
{
    const uint32_t per = count > kWave ? count / kWave : 1u;
    double a = 0.0, b = 0.0;
    if (lane * per < count) {
        const Partial* p = s_seg + lane * per;
        if (per == 1) {
            a = p[0].s1;
            b = p[0].s2;
        } else if (per == 2) {
            a = p[0].s1 + p[1].s1;
            b = p[0].s2 + p[1].s2;
        } else {
            a = (p[0].s1 + p[1].s1) + (p[2].s1 + p[3].s1);
            b = (p[0].s2 + p[1].s2) + (p[2].s2 + p[3].s2);
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) Mem::store(out, Partial{a, b});
}

// ---------------------------------------------------------------- one function's result

// The per-function second pass, run by one wave: the tile partials P[0 .. n)
// are summed by repeated 64-wide butterflies over aligned chunks (compacted in
// place), which is the pairwise tree over tile index; then mean and standard
// error in FP64.  Every lane returns the result.
template <class Mem = PlainMem>
__device__ __forceinline__ DevResult finalize_function(CDevFn* fn, Partial* P, uint32_t n, uint32_t lane,
                                                       int32_t status)
{
    while (n > 1) {
        const uint32_t chunks = (n + kWave - 1) / kWave;
        for (uint32_t c = 0; c < chunks; ++c) {
            const uint32_t i = c * kWave + lane;
            double a = 0.0, b = 0.0;
            if (i < n) {
                const Partial q = Mem::load(P + i);
                a = q.s1;
                b = q.s2;
            }
            a = wave_sum(a);
            b = wave_sum(b);
            if (lane == 0) Mem::store(P + c, Partial{a, b});
            Mem::sync();
            __threadfence_block();
        }
        n = chunks;
    }
    const Partial top = Mem::load(P);
    const double g1 = top.s1, g2 = top.s2;
    const double S1 = fn->scale1 * g1;
    const double S2 = fn->scale2 * g2;
    const uint64_t N = fn->n_samples;
    const double dn = (double)N;
    double var = (S2 - S1 * S1 / dn) / (dn - 1.0);
    if (!(var > 0.0)) var = 0.0;
    DevResult r;
    r.mean = fn->volume * (S1 / dn);
    r.std_error = fn->volume * sqrt(var / dn);
    r.sum_f = S1;
    r.sum_f2 = S2;
    r.n = N;
    r.status = status;
    r.precision = fn->precision;
    return r;
}

// ---------------------------------------------------------------- caller-supplied integrands

// A run-time compiled family calls F::f(x, p, d) once per sample, with x the
// sample's d coordinates in the box and p the function's 32 parameters.  The
// dimension is a template constant (one instantiation per dimension), so the
// caller's loops over coordinates unroll and the point stays in registers.
template <class F, uint32_t D>
struct EvalUser32 {
    CDevFn* fn;
    typedef float Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t, uint32_t k0, uint32_t k1, B b0, float g[4]) const
    {
        float x[4][D];
#pragma unroll
        for (uint32_t j = 0; j < D; ++j) {
            uint32_t w[4];
            philox_at<B>(b0 + j, k0, k1, w);
            const float c = fn->fc[j], o = fn->fo[j];
#pragma unroll
            for (int s = 0; s < 4; ++s) x[s][j] = fmaf(c, word_to_t(w[s]) - kTShift, o);
        }
        float p[kUserParams];
#pragma unroll
        for (int k = 0; k < kUserParams; ++k) p[k] = fn->up32[k];
#pragma unroll
        for (int s = 0; s < 4; ++s) g[s] = F::template f<float>(x[s], p, D);
    }
};

template <class F, uint32_t D>
struct EvalUser64 {
    CDevFn* fn;
    typedef double Value;
    template <class B>
    __device__ __forceinline__ void quad(uint32_t, uint32_t k0, uint32_t k1, B b0, double g[4]) const
    {
        double x[4][D];
#pragma unroll
        for (uint32_t j = 0; j < D; ++j) {
            uint32_t w[4];
            philox_at<B>(b0 + j, k0, k1, w);
            const double lo = fn->lo[j], wd = fn->w[j];
#pragma unroll
            for (int s = 0; s < 4; ++s) x[s][j] = fma(wd, word_to_u64(w[s]), lo);
        }
        double p[kUserParams];
#pragma unroll
        for (int k = 0; k < kUserParams; ++k) p[k] = fn->up[k];
#pragma unroll
        for (int s = 0; s < 4; ++s) g[s] = F::template f<double>(x[s], p, D);
    }
};

template <class F, bool F64, uint32_t D>
__device__ __forceinline__ void user_tile(CDevFn* fn, uint32_t seg0, uint32_t seg_log2, uint32_t wave,
                                          uint32_t lane, Partial* s_seg)
{
    if constexpr (F64) tile_segments<EvalUser64<F, D>>(fn, seg0, seg_log2, wave, lane, s_seg);
    else tile_segments<EvalUser32<F, D>>(fn, seg0, seg_log2, wave, lane, s_seg);
}

// Dispatch of a run-time compiled kernel: only its own family, by dimension.
template <class F, uint32_t FAMILY, bool F64>
struct UserDispatch {
    __device__ static __forceinline__ bool run(CDevFn* fn, uint32_t fam, uint32_t seg0, uint32_t seg_log2,
                                               uint32_t wave, uint32_t lane, Partial* s_seg)
    {
        if (fam != FAMILY) return false;
        switch (fn->dim) {
        case 1: user_tile<F, F64, 1>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 2: user_tile<F, F64, 2>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 3: user_tile<F, F64, 3>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 4: user_tile<F, F64, 4>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 5: user_tile<F, F64, 5>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 6: user_tile<F, F64, 6>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 7: user_tile<F, F64, 7>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 8: user_tile<F, F64, 8>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 9: user_tile<F, F64, 9>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 10: user_tile<F, F64, 10>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 11: user_tile<F, F64, 11>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        case 12: user_tile<F, F64, 12>(fn, seg0, seg_log2, wave, lane, s_seg); break;
        default: return false;
        }
        return true;
    }
};

// ---------------------------------------------------------------- persistent kernel body

// Persistent batched kernel: every workgroup fetches tiles from its kernel's
// part of the launch's tile list through one counter until that part is
// exhausted (or the abort word in device memory is set), evaluates them, and
// writes one partial per tile.  `Dispatch::run` evaluates a tile's segments for
// the function's family (false: not a family this kernel knows).  Indices read
// from the lists are checked against the launch's bounds; a bad record is
// skipped and counted instead of being dereferenced.
template <class Dispatch>
__device__ __forceinline__ void batched_body(const LaunchDesc* __restrict__ Ld, uint32_t kidx)
{
    __shared__ Partial s_seg[kBlockWaves << kMaxSegLog2];
    __shared__ uint32_t s_tile;
    const DevFn* fns = Ld->fns;
    const bool kidx_ok = kidx < (uint32_t)kMaxKernels;
    const Tile* tiles = Ld->tiles + (kidx_ok ? Ld->tile_begin[kidx] : 0u);
    const uint32_t n_tiles = kidx_ok ? Ld->tile_count[kidx] : 0u;
    if (n_tiles == 0) return;  // (uniform over the grid) no tiles for this kernel in this launch
    const uint32_t n_fns = Ld->n_fns;
    const uint64_t n_partials = Ld->n_partials;
    uint32_t* counters = Ld->counters;
    const uint32_t* abort_word = Ld->abort_word;
    Partial* partials = Ld->partials;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (uint32_t iter = 0;; ++iter) {
        if (threadIdx.x == 0) {
            uint32_t ti = n_tiles;
            if (kidx_ok) ti = atomicAdd(&counters[kCounterTiles + kidx], 1u);
            if ((iter & 7u) == 0u &&
                __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                atomicOr(&counters[kCounterAborted], 1u);
                ti = n_tiles;
            }
            s_tile = ti;
        }
        __syncthreads();
        const uint32_t ti = __builtin_amdgcn_readfirstlane(s_tile);
        if (ti >= n_tiles) break;
        const Tile t = tiles[ti];
        const uint32_t fi = __builtin_amdgcn_readfirstlane(t.fn);
        const uint32_t seg0 = __builtin_amdgcn_readfirstlane(t.seg0);
        const uint32_t seg_log2 = __builtin_amdgcn_readfirstlane(t.seg_log2);
        const uint32_t out = __builtin_amdgcn_readfirstlane(t.out);
        bool ok = fi < n_fns && seg_log2 <= (uint32_t)kMaxSegLog2 && out < n_partials;
        CDevFn* fn = scalar_view(fns + (ok ? fi : 0u));
        const uint32_t dim = fn->dim;
        ok = ok && dim >= 1 && dim <= (uint32_t)kMaxDim;
        if (ok) ok = Dispatch::run(fn, fn->kfam, seg0, seg_log2, wave, lane, s_seg);
        if (!ok && threadIdx.x == 0) atomicAdd(&counters[kCounterBadRecords], 1u);
        __syncthreads();
        if (ok && wave == 0) tile_tree(s_seg, (uint32_t)kBlockWaves << seg_log2, lane, &partials[out]);
    }
}

// ---------------------------------------------------------------- built-in family dispatch

template <bool B, class T, class F>
struct pick_type {
    typedef T type;
};
template <class T, class F>
struct pick_type<false, T, F> {
    typedef F type;
};

// Family dispatch of the built-in kernels (a wave-uniform branch per tile).
template <bool F64>
struct BuiltinDispatch {
    template <int FAM>
    using Ev = typename pick_type<F64, Eval64<FAM>, Eval32<FAM>>::type;
    __device__ static __forceinline__ bool run(CDevFn* fn, uint32_t fam, uint32_t seg0, uint32_t seg_log2,
                                               uint32_t wave, uint32_t lane, Partial* s_seg)
    {
        switch (fam) {
        case HARMONIC: tile_segments<Ev<HARMONIC>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case ABS_LINEAR: tile_segments<Ev<ABS_LINEAR>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case GAUSSIAN: tile_segments<Ev<GAUSSIAN>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case POLY_PRODUCT: tile_segments<Ev<POLY_PRODUCT>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        default: return false;
        }
    }
};

// ---------------------------------------------------------------- resident engine
//
// Memory ordering.  On this GPU an agent-scope acquire invalidates the L2 of the
// workgroup's XCD and a release writes it back, and the kernel hands data
// between workgroups at every chunk, so it uses neither.  Everything one
// workgroup writes for another -- records in the arena, tile partials, the
// finalize tree's sums, results in host memory -- is written through to memory
// with system-scope atomic stores, and waited for (s_waitcnt) before the word
// that announces it; partials and everything the host writes (ring entries,
// the record mirror) are read with system-scope atomic loads, which bypass the
// caches.  No line of shared data is ever dirty or stale in any cache, with one
// more fact for records: they are read through the scalar cache, and a record
// is written at a position no CU has read since the launch started (the host
// hands out fresh arena positions, and every cache is invalidated at a kernel's
// start), so those loads miss down to memory.  Polled words (tickets, the
// control words, ready and done tokens, tile counts) are relaxed atomics.

// 8-byte words written by the host, read past every cache.
__device__ __forceinline__ uint64_t host_word(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The device's copy of the control word after folding in a value read from the
// host.  Once the copy carries kCtlStop it is final (fetch_max of a word
// without the top bit cannot change it).
__device__ __forceinline__ uint64_t fold_host_ctl(uint64_t* pos, uint64_t cached, uint64_t host)
{
    if (host <= cached) return cached;
    const uint64_t old = __hip_atomic_fetch_max(&pos[1], host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return old > host ? old : host;
}

enum : uint32_t { kTake = 0, kLeave = 1 };

// Thread 0: wait (bounded) until ring entry `t` exists.  kTake: process it;
// kLeave: the launch is stopping and `t` is not below its final count.
__device__ inline uint32_t wait_ticket(const ResidentDesc* R, uint64_t t, bool leader)
{
    uint64_t* pos = R->pos;
    for (uint32_t polls = 0;; ++polls) {
        uint64_t c = __hip_atomic_load(&pos[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // leaders read the host's word at every check, the others every 64th
        // (so new entries are seen even while every leader is busy)
        if ((leader || (polls & 63u) == 63u) && (c & kCtlStop) == 0u && t >= c)
            c = fold_host_ctl(pos, c, host_word(R->host_ctl));
        if ((c & kCtlStop) != 0u) return t < (c & ~kCtlStop) ? kTake : kLeave;
        if (t < c) return kTake;
        if (polls + 1 >= R->idle_polls) {
            // nothing came for this ticket: stop the launch at the count as it stands
            const uint64_t old = __hip_atomic_fetch_or(&pos[1], kCtlStop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return t < (old & ~kCtlStop) ? kTake : kLeave;
        }
        __builtin_amdgcn_s_sleep(127);
    }
}

static_assert(sizeof(DevFn) == kWave * sizeof(uint4), "a record is one 16-byte word per lane of a wave");

// The resident kernel's body, with the family dispatch of FP32 and of FP64
// records as parameters.  Every wait is bounded: a ticket's entry (idle_polls
// polls, after which the launch stops itself) and a record another workgroup
// is copying into the arena (ready_polls; a chunk whose record does not show up
// is counted with its function's result reporting MC_ERR_HIP).  The last
// workgroup to leave stores `epoch` into host_exit.
template <class D32, class D64>
__device__ __forceinline__ void resident_body(const ResidentDesc* __restrict__ R, uint32_t epoch)
{
    __shared__ Partial s_seg[kBlockWaves << kMaxSegLog2];
    __shared__ Chunk s_chunk;
    __shared__ uint32_t s_state, s_ok, s_fin;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const bool leader = R->leader_every != 0u && blockIdx.x % R->leader_every == 0u;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t t = __hip_atomic_fetch_add(&R->pos[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t st = wait_ticket(R, t, leader);
            if (st == kTake) {
                // (the host wrote the entry before the count that shows it)
                const uint64_t* e = reinterpret_cast<const uint64_t*>(R->ring + (t & R->ring_mask));
                uint64_t w[sizeof(Chunk) / 8];
                for (uint32_t k = 0; k < (uint32_t)(sizeof(Chunk) / 8); ++k) w[k] = host_word(e + k);
                __builtin_memcpy(&s_chunk, w, sizeof(Chunk));
                // the entry has been read (its words are in registers) before the
                // host may reuse its place
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_s_waitcnt(0);
                __hip_atomic_store(&R->ack[t & R->ring_mask], t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            s_state = st;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_state) != kTake) break;
        const Chunk c = s_chunk;
        const uint32_t fi = __builtin_amdgcn_readfirstlane(c.fn);
        const uint32_t rec = __builtin_amdgcn_readfirstlane(c.rec);
        const uint32_t token = __builtin_amdgcn_readfirstlane(c.token);
        const uint32_t count = __builtin_amdgcn_readfirstlane(c.count);
        const uint32_t first = __builtin_amdgcn_readfirstlane(c.first);
        const uint32_t seg_log2 = __builtin_amdgcn_readfirstlane(c.seg_flags & 0xFFu);
        const bool upload = (__builtin_amdgcn_readfirstlane(c.seg_flags) >> 8 & kChunkUpload) != 0u;
        const uint32_t n_tiles = __builtin_amdgcn_readfirstlane(c.n_tiles);
        const uint32_t part0 = __builtin_amdgcn_readfirstlane(c.part0);
        // a chunk that fails these checks touches nothing but the bad-record count
        // (and, with a valid slot, its function's counters)
        if (!(fi < R->n_fns) || !(count >= 1u && count <= kChunkTiles)) {
            if (threadIdx.x == 0) atomicAdd(R->bad_records, 1u);
            __syncthreads();
            continue;
        }
        bool ok = rec < R->n_arena && seg_log2 <= (uint32_t)kMaxSegLog2 && first < n_tiles &&
                  count <= n_tiles - first && (uint64_t)part0 + n_tiles <= R->n_partials;
        if (ok && upload) {
            // the run's record goes to its arena position, copied by wave 0 alone
            // (one 16-byte word per lane): the release of the ready word waits for
            // that wave's stores, which a barrier would not do for other waves'
            if (wave == 0) {
                const uint64_t* src = reinterpret_cast<const uint64_t*>(R->mirror + fi) + 2 * lane;
                uint64_t* dst = reinterpret_cast<uint64_t*>(R->arena + rec) + 2 * lane;
                const uint64_t a = host_word(src), b = host_word(src + 1);
                __hip_atomic_store(dst, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(dst + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                CoherentMem::sync();
                if (lane == 0) __hip_atomic_store(&R->ready[rec], token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (threadIdx.x == 0) s_ok = rec + 1;
        } else if (ok) {
            if (threadIdx.x == 0) {
                uint32_t n = 0;
                while (__hip_atomic_load(&R->ready[rec], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != token &&
                       n < R->ready_polls) {
                    __builtin_amdgcn_s_sleep(8);
                    ++n;
                }
                s_ok = n < R->ready_polls ? rec + 1 : 0u;
            }
        } else if (threadIdx.x == 0) {
            s_ok = 0u;
        }
        __syncthreads();
        // the record's address comes from this LDS word, read after the barrier,
        // so no load of the record can be moved before the copy or the wait
        const uint32_t rec1 = __builtin_amdgcn_readfirstlane(s_ok);
        ok = rec1 != 0u;
        CDevFn* fn = scalar_view(R->arena + (ok ? rec1 - 1u : 0u));
        if (ok) {
            const uint32_t dim = fn->dim;
            ok = dim >= 1 && dim <= (uint32_t)kMaxDim;
        }
        if (ok) {
            const bool f64 = fn->precision != 0u;
            const uint32_t per_tile = (uint32_t)kBlockWaves << seg_log2;
            for (uint32_t i = 0; i < count && ok; ++i) {
                const uint32_t t = first + i;
                ok = f64 ? D64::run(fn, fn->kfam, t * per_tile, seg_log2, wave, lane, s_seg)
                         : D32::run(fn, fn->kfam, t * per_tile, seg_log2, wave, lane, s_seg);
                __syncthreads();
                if (ok && wave == 0) tile_tree<CoherentMem>(s_seg, per_tile, lane, &R->partials[part0 + t]);
                __syncthreads();
            }
        }
        // count the chunk's tiles once its partials (written by this thread)
        // are in memory; the workgroup that counts the run's last one finalizes it
        if (threadIdx.x == 0) {
            if (!ok) {
                atomicAdd(R->bad_records, 1u);
                __hip_atomic_store(&R->slot_err[fi], token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            CoherentMem::sync();
            const uint32_t before =
                __hip_atomic_fetch_add(&R->tiles_done[fi], count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_fin = before + count == n_tiles ? 1u : 0u;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_fin) != 0u && wave == 0) {
            const bool err = !ok || __hip_atomic_load(&R->slot_err[fi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == token;
            DevResult r{};
            if (!err) {
                r = finalize_function<CoherentMem>(fn, R->partials + part0, n_tiles, lane, 0);
            } else {
                r.status = -8;  // MC_ERR_HIP
            }
            if (lane == 0) {
                static_assert(sizeof(DevResult) == 6 * sizeof(uint64_t), "result words");
                uint64_t w[6];
                __builtin_memcpy(w, &r, sizeof r);
                uint64_t* dst = reinterpret_cast<uint64_t*>(R->host_results + fi);
                for (int k = 0; k < 6; ++k) __hip_atomic_store(dst + k, w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&R->tiles_done[fi], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // (the result and the counter reset are done before the done word)
                CoherentMem::sync();
                __hip_atomic_store(&R->host_done[fi], token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // acknowledgements and results above are visible before the exit word
        const uint32_t left = __hip_atomic_fetch_sub(R->running, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
        if (left == 1u) {
            const uint32_t bad = __hip_atomic_load(R->bad_records, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(R->host_exit + 1, bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(R->host_exit, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

}  // namespace zmc
