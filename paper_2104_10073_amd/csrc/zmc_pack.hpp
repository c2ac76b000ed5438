// zmc_pack.hpp -- packing of one function-table entry (include/zmc.h) into the
// device record the kernels read, shared by the host runtime (mc_submit) and
// the grid kernel that builds records on the device (mc_submit_grid).
//
// FP64 fields: box corner lo, width w = hi - lo, per-dimension vector v, the
// two scalars, degrees, volume (the direct Monte Carlo estimate is V times the
// sample mean).  FP32 fields: each family folded into local coordinates in
// t = u + (1 - 2^-24) in [1, 2), computed in FP64 and rounded once:
//   harmonic (Eq. (1))  a cos(k.x) + b sin(k.x) = R cos(2 pi (phi0 + sum kappa_j t_j)),
//                       R = hypot(a, b), kappa_j = k_j w_j / 2 pi;
//   |linear| (Eq. (2))  c0 + c.x = off + sum gamma_j t_j, off kept as two floats;
//   Gaussian            exp(-|x - mu|^2 / 2 s^2) = 2^(-sum (c_j (t_j - m_j))^2);
//   polynomial          x_j = fma(w_j, u_j, lo_j) in FP32;
//   run-time families   the point in the box, parameters rounded to float.
#pragma once

#include <math.h>
#include <stdint.h>

#include "zmc.h"
#include "zmc_device.hpp"

namespace zmc {

constexpr double kPackTwoPi = 6.283185307179586476925286766559;
constexpr double kPackLog2e = 1.4426950408889634073599246810019;
constexpr double kPackPi = 3.141592653589793238462643383280;
constexpr double kPackPi2 = 1.570796326794896619231321691640;
constexpr double kPackPi4 = 0.785398163397448309615660845820;

// Records are packed by the host (tables) and by the device (parameter grids),
// and a function must get the same record bits either way.  Division, square
// root, floor and conversions are correctly rounded on both, and no product is
// fused into a sum (-ffp-contract=off), but libm's hypot and atan2 are not the
// same functions on the host and the device, so the packing computes them from
// correctly rounded operations only: the same bits everywhere, within a few
// units in the last place of the exact values.

// sqrt(a^2 + b^2), scaled by the larger magnitude so no square overflows.
__host__ __device__ inline double pack_hypot(double a, double b)
{
    a = fabs(a);
    b = fabs(b);
    const double m = a > b ? a : b, n = a > b ? b : a;
    if (!(m > 0.0) || !(m <= 1.7976931348623157e308)) return m + n;  // zero, infinity or NaN
    const double r = n / m;
    return m * sqrt(1.0 + r * r);
}

// atan(z) for |z| <= tan(pi/8): one halving, atan z = 2 atan(z / (1 + sqrt(1 + z^2))),
// brings the argument below 0.2, then the series sum_k (-1)^k h^(2k+1) / (2k + 1)
// to k = 13 (truncation below 1e-20 relative).
__host__ __device__ inline double pack_atan_small(double z)
{
    const double h = z / (1.0 + sqrt(1.0 + z * z));
    const double h2 = h * h;
    double s = 0.0;
    for (int k = 13; k >= 0; --k) s = s * h2 + ((k & 1) ? -1.0 : 1.0) / (double)(2 * k + 1);
    return 2.0 * (h * s);
}

// The angle of (x, y) in (-pi, pi] (0 at the origin).
__host__ __device__ inline double pack_atan2(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    if (!(ax > 0.0) && !(ay > 0.0)) return 0.0;
    const bool swap = ay > ax;
    const double t = swap ? ax / ay : ay / ax;  // in [0, 1]
    double r = t > 0.41421356237309503 ? kPackPi4 + pack_atan_small((t - 1.0) / (t + 1.0)) : pack_atan_small(t);
    if (swap) r = kPackPi2 - r;
    if (x < 0.0) r = kPackPi - r;
    return y < 0.0 ? -r : r;
}

__host__ __device__ inline float pack_frac_to_float(double x)
{
    double r = x - floor(x);
    float f = (float)r;
    if (f >= 1.0f) f = 0.0f;
    return f;
}

// The factor the FP32 path takes out of every sample of a built-in family
// (f = scale * g; S1 and S2 are scaled by it and its square in FP64 at
// finalize): the amplitude for Eq. (1), |linear| and Gaussian forms, 1 for the
// product polynomial and run-time families.
__host__ __device__ inline double fp32_scale(const mc_function& f)
{
    if (f.family >= kUserFamily0) return 1.0;
    switch (f.family) {
    case MC_FAMILY_HARMONIC: return pack_hypot(f.params[0], f.params[1]);
    case MC_FAMILY_ABS_LINEAR:
    case MC_FAMILY_GAUSSIAN: return f.params[0];
    default: return 1.0;
    }
}

// `f` must have passed validation; `precision` is MC_PREC_FP32_EVAL or MC_PREC_FP64.
__host__ __device__ inline void pack_function(const mc_function& f, int precision, DevFn* d)
{
    {
        uint32_t* w = reinterpret_cast<uint32_t*>(d);
        for (size_t i = 0; i < sizeof(DevFn) / sizeof(uint32_t); ++i) w[i] = 0u;
    }
    const uint32_t D = f.dim;
    d->family = f.family;
    d->kfam = f.family;
    d->dim = D;
    d->key0 = (uint32_t)(f.seed & 0xFFFFFFFFull);
    d->key1 = (uint32_t)(f.seed >> 32);
    d->n_samples = f.n_samples;
    d->n_quads = (f.n_samples + 3) / 4;
    d->n_segments = (uint32_t)((d->n_quads + kSegQuads - 1) / kSegQuads);
    d->precision = (uint32_t)precision;
    double vol = 1.0;
    for (uint32_t j = 0; j < D; ++j) {
        d->lo[j] = f.lo[j];
        d->w[j] = f.hi[j] - f.lo[j];
        d->v[j] = f.params[MC_PARAM_V0 + j];
        vol *= d->w[j];
    }
    d->volume = vol;
    d->s0 = f.params[0];
    d->s1 = f.params[1];
    if (f.family == MC_FAMILY_GAUSSIAN) d->h = 0.5 / (f.params[1] * f.params[1]);
    if (f.family == MC_FAMILY_POLY_PRODUCT)
        for (uint32_t j = 0; j < D; ++j) d->deg[j] = (int32_t)f.params[MC_PARAM_W0 + j];
    d->scale1 = 1.0;
    d->scale2 = 1.0;
    if (f.family >= kUserFamily0) {
        // run-time family: the point in the box and the raw parameters (both precisions)
        for (int k = 0; k < kUserParams; ++k) {
            d->up[k] = f.params[k];
            d->up32[k] = (float)f.params[k];
        }
        for (uint32_t j = 0; j < D; ++j) {
            d->fc[j] = (float)d->w[j];
            d->fo[j] = (float)f.lo[j];
        }
        return;
    }
    if (precision == MC_PREC_FP64) return;

    // FP32 evaluation: coefficients in t_j = u_j + C, C = 1 - 2^-24.
    const double C = 1.0 - 0x1p-24;
    switch (f.family) {
    case MC_FAMILY_HARMONIC: {
        const double a = f.params[0], b = f.params[1];
        const double R = fp32_scale(f);
        const double phi = (R > 0.0) ? pack_atan2(b, a) : 0.0;
        double off = -phi / kPackTwoPi;
        for (uint32_t j = 0; j < D; ++j) {
            const double k = f.params[MC_PARAM_V0 + j];
            d->fc[j] = (float)(k * d->w[j] / kPackTwoPi);
            off += k * f.lo[j] / kPackTwoPi - C * (double)d->fc[j];
        }
        d->f0 = pack_frac_to_float(off);
        d->scale1 = R;
        d->scale2 = R * R;
        break;
    }
    case MC_FAMILY_ABS_LINEAR: {
        double off = f.params[1];
        for (uint32_t j = 0; j < D; ++j) {
            const double c = f.params[MC_PARAM_V0 + j];
            d->fc[j] = (float)(c * d->w[j]);
            off += c * f.lo[j] - C * (double)d->fc[j];
        }
        d->f0 = (float)off;
        d->f0lo = (float)(off - (double)d->f0);
        d->scale1 = fp32_scale(f);
        d->scale2 = d->scale1 * d->scale1;
        break;
    }
    case MC_FAMILY_GAUSSIAN: {
        const double sigma = f.params[1];
        const double hh = kPackLog2e / (2.0 * sigma * sigma);  // log2(e) / (2 s^2)
        const double sq = sqrt(hh);
        for (uint32_t j = 0; j < D; ++j) {
            d->fc[j] = (float)(d->w[j] * sq);
            d->fo[j] = (float)(C + (f.params[MC_PARAM_V0 + j] - f.lo[j]) / d->w[j]);
        }
        d->scale1 = fp32_scale(f);
        d->scale2 = d->scale1 * d->scale1;
        break;
    }
    default: {  // POLY_PRODUCT
        for (uint32_t j = 0; j < D; ++j) {
            d->fc[j] = (float)d->w[j];
            d->fo[j] = (float)f.lo[j];
            d->fp[j] = (float)f.params[MC_PARAM_V0 + j];
        }
        break;
    }
    }
}

// A parameter grid as the device builds it: base function, axes, precision,
// number of functions.
struct GridSpec {
    mc_function base;
    mc_grid_axis axes[MC_MAX_GRID_AXES];
    uint32_t n_axes;
    int32_t precision;
    uint64_t n;
};

// Function i of a parameter grid (axis 0 varies fastest; seed = base seed + i).
__host__ __device__ inline void grid_function(const mc_function& base, const mc_grid_axis* axes, uint32_t n_axes,
                                              uint64_t i, mc_function* out)
{
    *out = base;
    uint64_t rest = i;
    for (uint32_t a = 0; a < n_axes; ++a) {
        const uint64_t k = rest % axes[a].count;
        rest /= axes[a].count;
        out->params[axes[a].param] = axes[a].start + (double)k * axes[a].step;
    }
    out->seed = base.seed + i;
}

}  // namespace zmc
