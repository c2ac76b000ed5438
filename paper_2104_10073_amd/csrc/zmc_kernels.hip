// zmc_kernels.hip -- gfx950 kernels of the multi-function direct Monte Carlo path.
//
// Per sample (paper, "Solution method": direct Monte Carlo per integrand):
//   1. counter-based uniforms: Philox4x32-10 (SC'11) in registers, coordinate j of
//      sample i reads word g = i*d + j of the function's stream;
//   2. mapping into the function's box;
//   3. the integrand (Eq. (1) harmonic, Eq. (2) |linear|, Gaussian, product polynomial);
//   4. compensated per-lane sums of f and f^2;
// then per segment a fixed 64-lane butterfly in FP64, per tile an LDS tree over
// its segments, and per function an atomic-free FP64 finalize pass giving the
// mean and standard error.  No MFMA: nothing here is a dense contraction; the
// bound is VALU issue (integer multiplies of Philox, FP32 FMAs, transcendentals).
#include <hip/hip_runtime.h>
#include <stdint.h>

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
                                             uint32_t* out)
{
    uint32_t c0, c1, c2, c3;
    {   // round 1: c2 = c3 = 0
        const uint64_t p0 = (uint64_t)kPhiloxM0 * b_lo;
        c0 = b_hi ^ k0;
        c1 = 0u;
        c2 = (uint32_t)(p0 >> 32) ^ k1;
        c3 = (uint32_t)p0;
    }
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    {   // round 2: c1 = 0
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

// ---------------------------------------------------------------- FP32 integrands

// Evaluators work incrementally so a quad's Philox words are consumed as soon
// as their block is produced: init() gives the per-sample state, add(st, j, w)
// folds coordinate j (from word w) into it, finish(st) returns g with
// f = scale1 * g (scale1 and scale2 = scale1^2 are applied in FP64 at
// finalize).  Constants are wave-uniform, loaded once per tile, and were
// derived on the host in FP64 and rounded once.

template <int FAM, int D> struct Eval32;

// Eq. (1): a cos(theta) + b sin(theta) = R cos(theta - phi).  The phase in
// revolutions is f0 + sum_j kappa_j t_j; v_fract + v_cos_f32 (which computes
// cos(2 pi x)) give the cosine: one transcendental per sample.
template <int D> struct Eval32<HARMONIC, D> {
    float c[D];
    float f0;
    __device__ __forceinline__ void load(const DevFn* fn)
    {
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = fn->fc[j];
        f0 = fn->f0;
    }
    __device__ __forceinline__ float init() const { return f0; }
    __device__ __forceinline__ void add(float& th, int j, uint32_t w) const { th = fmaf(c[j], word_to_t(w), th); }
    __device__ __forceinline__ float finish(float th) const
    {
        return __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(th));
    }
};

// Eq. (2): a |c0 + c.x|; the offset is carried as a two-float sum so the
// hyperplane is placed to FP64 accuracy.
template <int D> struct Eval32<ABS_LINEAR, D> {
    float c[D];
    float f0, f0lo;
    __device__ __forceinline__ void load(const DevFn* fn)
    {
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = fn->fc[j];
        f0 = fn->f0;
        f0lo = fn->f0lo;
    }
    __device__ __forceinline__ float init() const { return f0; }
    __device__ __forceinline__ void add(float& s, int j, uint32_t w) const { s = fmaf(c[j], word_to_t(w), s); }
    __device__ __forceinline__ float finish(float s) const { return fabsf(s + f0lo); }
};

// A exp(-|x - mu|^2 / (2 sigma^2)) = A 2^(-sum_j (c_j (t_j - m_j))^2); t - m is
// exact (both in [1, 2] for a centre inside the box), v_exp_f32 computes 2^x.
template <int D> struct Eval32<GAUSSIAN, D> {
    float c[D], m[D];
    __device__ __forceinline__ void load(const DevFn* fn)
    {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            c[j] = fn->fc[j];
            m[j] = fn->fo[j];
        }
    }
    __device__ __forceinline__ float init() const { return 0.0f; }
    __device__ __forceinline__ void add(float& q, int j, uint32_t w) const
    {
        const float y = c[j] * (word_to_t(w) - m[j]);
        q = fmaf(y, y, q);
    }
    __device__ __forceinline__ float finish(float q) const { return __builtin_amdgcn_exp2f(-q); }
};

// prod_j (1 + p_j x_j^{n_j}), x_j = lo_j + w_j u_j with u_j = t_j - (1 - 2^-24) exact.
// Each factor is a degree-MAXDEG polynomial in x_j whose only non-zero
// coefficients are the constant 1 and p_j at power n_j (the constant is 1 + p_j
// when n_j = 0); Horner's rule evaluates it without branches.
template <int D, int MAXDEG> struct Eval32Poly {
    float c[D], o[D];
    float h[D][MAXDEG];   // h[j][k]: coefficient of x^(k+1)
    float h0[D];          // constant term
    __device__ __forceinline__ void load(const DevFn* fn)
    {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            c[j] = fn->fc[j];
            o[j] = fn->fo[j];
            const int n = fn->deg[j];
            const float pj = fn->fp[j];
#pragma unroll
            for (int k = 0; k < MAXDEG; ++k) h[j][k] = (n == k + 1) ? pj : 0.0f;
            h0[j] = (n == 0) ? 1.0f + pj : 1.0f;
        }
    }
    __device__ __forceinline__ float init() const { return 1.0f; }
    __device__ __forceinline__ void add(float& g, int j, uint32_t w) const
    {
        const float x = fmaf(c[j], word_to_t(w) - kTShift, o[j]);
        float acc = h[j][MAXDEG - 1];
#pragma unroll
        for (int k = MAXDEG - 2; k >= 0; --k) acc = fmaf(acc, x, h[j][k]);
        g *= fmaf(acc, x, h0[j]);
    }
    __device__ __forceinline__ float finish(float g) const { return g; }
};

template <int D> struct Eval32<POLY_PRODUCT, D> : Eval32Poly<D, 4> {};
// Degrees 5..8 use the same evaluator with eight Horner steps (family id 4 inside the kernels).
constexpr int kPolyHighFamily = 4;
template <int D> struct Eval32<kPolyHighFamily, D> : Eval32Poly<D, 8> {};

// ---------------------------------------------------------------- FP64 integrands

// The definition in its reference operation order (explicit fma), FP64 libm.
template <int FAM, int D> struct Eval64 {
    double lo[D], w[D], v[D];
    double s0, s1, h;
    int n[D];
    __device__ __forceinline__ void load(const DevFn* fn)
    {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            lo[j] = fn->lo[j];
            w[j] = fn->w[j];
            v[j] = fn->v[j];
            n[j] = fn->deg[j];
        }
        s0 = fn->s0;
        s1 = fn->s1;
        h = fn->h;
    }
    __device__ __forceinline__ double init() const
    {
        if constexpr (FAM == ABS_LINEAR) return s1;
        else if constexpr (FAM == POLY_PRODUCT) return 1.0;
        else return 0.0;
    }
    __device__ __forceinline__ void add(double& st, int j, uint32_t wd) const
    {
        const double x = fma(w[j], word_to_u64(wd), lo[j]);
        if constexpr (FAM == HARMONIC || FAM == ABS_LINEAR) {
            st = fma(v[j], x, st);
        } else if constexpr (FAM == GAUSSIAN) {
            const double t = x - v[j];
            st = fma(t, t, st);
        } else {
            double xp = 1.0;
            const int e = n[j];
            for (int k = 0; k < e; ++k) xp *= x;
            st *= fma(v[j], xp, 1.0);
        }
    }
    __device__ __forceinline__ double finish(double st) const
    {
        if constexpr (FAM == HARMONIC) {
            double sn, cs;
            sincos(st, &sn, &cs);
            return fma(s0, cs, s1 * sn);
        } else if constexpr (FAM == ABS_LINEAR) {
            return s0 * fabs(st);
        } else if constexpr (FAM == GAUSSIAN) {
            return s0 * exp(-st * h);
        } else {
            return st;
        }
    }
};

// One quad (4 consecutive samples, quad index q): the d Philox blocks q*d .. q*d+d-1
// hold the 4d words in sample-major order; each block's words are folded into
// the states of the samples they belong to as soon as it is produced.
constexpr int kIlpBlocks = 2;

template <class Ev, int D, class T>
__device__ __forceinline__ void eval_quad(const Ev& ev, uint32_t k0, uint32_t k1, uint64_t q, T g[4])
{
    T st[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) st[s] = ev.init();
    const uint64_t b0 = q * (uint64_t)D;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const uint64_t b = b0 + (uint64_t)i;
        uint32_t w[4];
        philox_block((uint32_t)b, (uint32_t)(b >> 32), k0, k1, w);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = 4 * i + e;   // word index inside the quad: sample gi / D, coordinate gi % D
            ev.add(st[gi / D], gi % D, w[e]);
        }
        // Keep at most kIlpBlocks blocks in flight: enough independent work per wave
        // to cover latencies, few enough registers for several waves per SIMD.
        if ((i % kIlpBlocks) == kIlpBlocks - 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) g[s] = ev.finish(st[s]);
}

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

// Lane sums over the lane's 16 quads of one segment.  TAIL marks the function's
// last segment, the only one that can hold quads or samples past N.
template <int FAM, int D, bool TAIL>
__device__ __forceinline__ void segment_fp32(const Eval32<FAM, D>& ev, uint32_t k0, uint32_t k1, uint64_t quad0,
                                             uint64_t n_quads, uint64_t n_samples, double& out1, double& out2)
{
    float s1 = 0.0f, c1 = 0.0f, s2 = 0.0f, c2 = 0.0f;
#pragma unroll 1
    for (int k = 0; k < kQuadsPerLane; ++k) {
        const uint64_t q = quad0 + (uint64_t)(k * kWave);
        if (TAIL && q >= n_quads) break;
        float g[4];
        eval_quad<Eval32<FAM, D>, D, float>(ev, k0, k1, q, g);
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

template <int FAM, int D, bool TAIL>
__device__ __forceinline__ void segment_fp64(const Eval64<FAM, D>& ev, uint32_t k0, uint32_t k1, uint64_t quad0,
                                             uint64_t n_quads, uint64_t n_samples, double& out1, double& out2)
{
    double s1 = 0.0, s2 = 0.0;
#pragma unroll 1
    for (int k = 0; k < kQuadsPerLane; ++k) {
        const uint64_t q = quad0 + (uint64_t)(k * kWave);
        if (TAIL && q >= n_quads) break;
        double f[4];
        eval_quad<Eval64<FAM, D>, D, double>(ev, k0, k1, q, f);
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

// ---------------------------------------------------------------- one tile

// Wave `wave` of the workgroup evaluates segments seg0 + wave*2^L + i, i < 2^L,
// and leaves each segment's (S1, S2) in LDS slot wave*2^L + i (zero past the
// function's last segment).
template <bool F64, int FAM, int D>
__device__ __forceinline__ void tile_segments(const DevFn* __restrict__ fn, uint32_t seg0, uint32_t seg_log2,
                                           uint32_t wave, uint32_t lane, Partial* s_seg)
{
    // Everything here is wave-uniform; say so, so the function's constants are
    // fetched with scalar loads and stay in scalar registers.
    fn = (const DevFn*)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)fn)) |
                        ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uintptr_t)fn >> 32)) << 32));
    seg0 = __builtin_amdgcn_readfirstlane(seg0);
    seg_log2 = __builtin_amdgcn_readfirstlane(seg_log2);
    wave = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t per_wave = 1u << seg_log2;
    const uint32_t n_seg = fn->n_segments;
    const uint64_t n_quads = fn->n_quads;
    const uint64_t n_samples = fn->n_samples;
    const uint32_t k0 = fn->key0, k1 = fn->key1;
    const uint32_t first = seg0 + wave * per_wave;
    if constexpr (F64) {
        Eval64<FAM, D> ev;
        ev.load(fn);
        for (uint32_t i = 0; i < per_wave; ++i) {
            const uint32_t seg = first + i;
            double a = 0.0, b = 0.0;
            if (seg < n_seg) {
                const uint64_t quad0 = (uint64_t)seg * kSegQuads + lane;
                if ((uint64_t)(seg + 1) * kSegSamples <= n_samples)
                    segment_fp64<FAM, D, false>(ev, k0, k1, quad0, n_quads, n_samples, a, b);
                else
                    segment_fp64<FAM, D, true>(ev, k0, k1, quad0, n_quads, n_samples, a, b);
                a = wave_sum(a);
                b = wave_sum(b);
            }
            if (lane == 0) s_seg[wave * per_wave + i] = Partial{a, b};
        }
    } else {
        Eval32<FAM, D> ev;
        ev.load(fn);
        for (uint32_t i = 0; i < per_wave; ++i) {
            const uint32_t seg = first + i;
            double a = 0.0, b = 0.0;
            if (seg < n_seg) {
                const uint64_t quad0 = (uint64_t)seg * kSegQuads + lane;
                if ((uint64_t)(seg + 1) * kSegSamples <= n_samples)
                    segment_fp32<FAM, D, false>(ev, k0, k1, quad0, n_quads, n_samples, a, b);
                else
                    segment_fp32<FAM, D, true>(ev, k0, k1, quad0, n_quads, n_samples, a, b);
                a = wave_sum(a);
                b = wave_sum(b);
            }
            if (lane == 0) s_seg[wave * per_wave + i] = Partial{a, b};
        }
    }
}

template <bool F64, int FAM>
__device__ __forceinline__ void dispatch_dim(uint32_t dim, const DevFn* fn, uint32_t seg0, uint32_t seg_log2,
                                             uint32_t wave, uint32_t lane, Partial* s_seg)
{
    switch (dim) {
    case 1: tile_segments<F64, FAM, 1>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 2: tile_segments<F64, FAM, 2>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 3: tile_segments<F64, FAM, 3>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 4: tile_segments<F64, FAM, 4>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 5: tile_segments<F64, FAM, 5>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 6: tile_segments<F64, FAM, 6>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 7: tile_segments<F64, FAM, 7>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 8: tile_segments<F64, FAM, 8>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 9: tile_segments<F64, FAM, 9>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 10: tile_segments<F64, FAM, 10>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    case 11: tile_segments<F64, FAM, 11>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    default: tile_segments<F64, FAM, 12>(fn, seg0, seg_log2, wave, lane, s_seg); break;
    }
}

// Pairwise tree over the tile's 4 * 2^L segment sums (L <= 6, so at most 4 per lane),
// then the lane butterfly: the same tree as over the whole function.
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
    if (lane == 0) *out = Partial{a, b};
}

// ---------------------------------------------------------------- kernels

// Persistent batched kernel: every workgroup fetches tiles from the launch's
// tile list through one counter until the list is exhausted (or the host-mapped
// abort word is set), evaluates them, and writes one partial per tile.
template <bool F64>
__device__ __forceinline__ void batched_body(const LaunchDesc* __restrict__ Ld)
{
    __shared__ Partial s_seg[kBlockWaves << kMaxSegLog2];
    __shared__ uint32_t s_tile;
    const DevFn* __restrict__ fns = Ld->fns;
    const Tile* __restrict__ tiles = F64 ? Ld->tiles64 : Ld->tiles32;
    const uint32_t n_tiles = F64 ? Ld->n_tiles64 : Ld->n_tiles32;
    uint32_t* counters = Ld->counters;
    Partial* partials = Ld->partials;
    const volatile uint32_t* abort_flag = Ld->abort_flag;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t iter = 0;; ++iter) {
        if (threadIdx.x == 0) {
            uint32_t ti = atomicAdd(&counters[F64 ? 1 : 0], 1u);
            if (abort_flag != nullptr && (iter & 7u) == 0u && *abort_flag != 0u) {
                atomicOr(&counters[2], 1u);
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
        const DevFn* fn = fns + fi;
        const uint32_t fam = __builtin_amdgcn_readfirstlane(fn->kfam);
        const uint32_t dim = __builtin_amdgcn_readfirstlane(fn->dim);
        switch (fam) {
        case HARMONIC: dispatch_dim<F64, HARMONIC>(dim, fn, seg0, seg_log2, wave, lane, s_seg); break;
        case ABS_LINEAR: dispatch_dim<F64, ABS_LINEAR>(dim, fn, seg0, seg_log2, wave, lane, s_seg); break;
        case GAUSSIAN: dispatch_dim<F64, GAUSSIAN>(dim, fn, seg0, seg_log2, wave, lane, s_seg); break;
        case POLY_PRODUCT: dispatch_dim<F64, POLY_PRODUCT>(dim, fn, seg0, seg_log2, wave, lane, s_seg); break;
        default:
            if constexpr (F64) dispatch_dim<F64, POLY_PRODUCT>(dim, fn, seg0, seg_log2, wave, lane, s_seg);
            else dispatch_dim<F64, kPolyHighFamily>(dim, fn, seg0, seg_log2, wave, lane, s_seg);
            break;
        }
        __syncthreads();
        if (wave == 0) tile_tree(s_seg, (uint32_t)kBlockWaves << seg_log2, lane, &partials[t.out]);
    }
}

extern "C" __global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void zmc_batched_fp32(const LaunchDesc* __restrict__ Ld)
{
    batched_body<false>(Ld);
}

extern "C" __global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void zmc_batched_fp64(const LaunchDesc* __restrict__ Ld)
{
    batched_body<true>(Ld);
}

// Per-function second pass, one wave per function: the tile partials are summed
// by repeated 64-wide butterflies over aligned chunks (compacted in place), which
// is the pairwise tree over tile index; then mean and standard error in FP64.
extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_finalize(const LaunchDesc* __restrict__ Ld)
{
    const DevFn* __restrict__ fns = Ld->fns;
    const Fin* __restrict__ fins = Ld->fins;
    Partial* partials = Ld->partials;
    DevResult* results = Ld->results;
    const uint32_t n_fins = Ld->n_fins;
    const bool aborted = __builtin_amdgcn_readfirstlane(((volatile uint32_t*)Ld->counters)[2]) != 0u;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t gw = blockIdx.x * kBlockWaves + threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * kBlockWaves;
    for (uint32_t f = gw; f < n_fins; f += nw) {
        const Fin fin = fins[f];
        const DevFn* fn = fns + fin.fn;
        Partial* P = partials + fin.part0;
        uint32_t n = fin.n_tiles;
        while (n > 1) {
            const uint32_t chunks = (n + kWave - 1) / kWave;
            for (uint32_t c = 0; c < chunks; ++c) {
                const uint32_t i = c * kWave + lane;
                double a = 0.0, b = 0.0;
                if (i < n) {
                    a = P[i].s1;
                    b = P[i].s2;
                }
                a = wave_sum(a);
                b = wave_sum(b);
                if (lane == 0) P[c] = Partial{a, b};
                __threadfence_block();
            }
            n = chunks;
        }
        if (lane == 0) {
            const double g1 = P[0].s1, g2 = P[0].s2;
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
            r.status = aborted ? -10 : 0;
            r.precision = fn->precision;
            results[fin.res] = r;
        }
    }
}

// ---------------------------------------------------------------- plain FP64 path

// One thread per quad over a grid sized to the function's N, block sums in LDS,
// one partial per block; a second single-block kernel reduces the partials.
template <int FAM, int D>
__global__ __launch_bounds__(256) void plain_fp64_kernel(const DevFn* __restrict__ fn, Partial* __restrict__ out)
{
    __shared__ double s1[256], s2[256];
    Eval64<FAM, D> ev;
    ev.load(fn);
    const uint64_t q = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t n_samples = fn->n_samples;
    double a = 0.0, b = 0.0;
    if (q < fn->n_quads) {
        double f[4];
        eval_quad<Eval64<FAM, D>, D, double>(ev, fn->key0, fn->key1, q, f);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (4 * q + (uint64_t)s < n_samples) {
                a += f[s];
                b += f[s] * f[s];
            }
        }
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = Partial{s1[0], s2[0]};
}

extern "C" __global__ __launch_bounds__(256) void zmc_plain_reduce(const DevFn* __restrict__ fn,
                                                                   const Partial* __restrict__ parts,
                                                                   uint32_t n_parts, DevResult* __restrict__ res)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (uint32_t i = threadIdx.x; i < n_parts; i += 256) {
        a += parts[i].s1;
        b += parts[i].s2;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double S1 = s1[0], S2 = s2[0];
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
        r.status = 0;
        r.precision = 1;
        *res = r;
    }
}

// Host-side table of the plain kernels, indexed [family][dim - 1].
typedef void (*PlainKernel)(const DevFn*, Partial*);

#define ZMC_PLAIN_ROW(F)                                                                              \
    {plain_fp64_kernel<F, 1>, plain_fp64_kernel<F, 2>, plain_fp64_kernel<F, 3>, plain_fp64_kernel<F, 4>, \
     plain_fp64_kernel<F, 5>, plain_fp64_kernel<F, 6>, plain_fp64_kernel<F, 7>, plain_fp64_kernel<F, 8>, \
     plain_fp64_kernel<F, 9>, plain_fp64_kernel<F, 10>, plain_fp64_kernel<F, 11>, plain_fp64_kernel<F, 12>}

const PlainKernel kPlainKernels[kNumFamilies][kMaxDim] = {
    ZMC_PLAIN_ROW(HARMONIC), ZMC_PLAIN_ROW(ABS_LINEAR), ZMC_PLAIN_ROW(GAUSSIAN), ZMC_PLAIN_ROW(POLY_PRODUCT)};

const void* plain_kernel_ptr(uint32_t family, uint32_t dim)
{
    return (const void*)kPlainKernels[family][dim - 1];
}

const void* batched_kernel_ptr(bool fp64)
{
    return fp64 ? (const void*)zmc_batched_fp64 : (const void*)zmc_batched_fp32;
}

const void* finalize_kernel_ptr() { return (const void*)zmc_finalize; }
const void* plain_reduce_kernel_ptr() { return (const void*)zmc_plain_reduce; }

}  // namespace zmc
