// zmc_kernels.hip -- the launch's other gfx950 kernels: staging of the work
// list, the finalize pass, publication of results, the grid packer, and the
// plain one-launch-per-function FP64 path.  The persistent batched kernels are
// in zmc_batched.hip; the device code they share is in zmc_device_code.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zmc_device_code.hpp"
#include "zmc_pack.hpp"

namespace zmc {

// First kernel of a launch: copy the staged descriptor, counters and finalize
// records from pinned host memory into the slot's device block (their byte
// count is the descriptor's first field, bounded by `cap`), copy the function
// records that runs flag from the host mirror of the function table
// (`mirror`, fine-grained, `n_fns` records) into the device table `fns`, and
// expand the staged tile runs into the device tile list (bounded by
// `tile_cap`).
extern "C" __global__ __launch_bounds__(256) void zmc_stage(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                            uint64_t cap, uint32_t tile_cap,
                                                            const DevFn* __restrict__ mirror,
                                                            DevFn* __restrict__ fns, uint32_t n_fns)
{
    __shared__ uint64_t s_bytes;
    __shared__ uint32_t s_runs, s_runs_off;
    __shared__ Tile* s_tiles;
    if (threadIdx.x == 0) {
        const LaunchDesc* hd = reinterpret_cast<const LaunchDesc*>(src);
        s_bytes = hd->stage_bytes;
        s_runs = hd->n_runs;
        s_runs_off = hd->runs_off;
        s_tiles = const_cast<Tile*>(hd->tiles);
    }
    __syncthreads();
    const uint64_t bytes = s_bytes < cap ? s_bytes : cap;
    const uint64_t n = bytes / sizeof(uint4);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
    const TileRun* runs = reinterpret_cast<const TileRun*>(reinterpret_cast<const uint8_t*>(src) + s_runs_off);
    Tile* tiles = s_tiles;
    for (uint32_t r = blockIdx.x; r < s_runs; r += gridDim.x) {
        const TileRun run = runs[r];
        if ((run.flags & kRunUploadRecord) != 0u && run.fn < n_fns) {
            // the function's record, packed on the host since its last use, goes up
            // with the launch that first needs it (the batched kernels run after
            // this kernel in the same stream)
            const uint4* rs = reinterpret_cast<const uint4*>(mirror + run.fn);
            uint4* rd = reinterpret_cast<uint4*>(fns + run.fn);
            for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(DevFn) / sizeof(uint4)); i += blockDim.x)
                rd[i] = rs[i];
        }
        if (run.dst > tile_cap || run.count > tile_cap - run.dst || run.seg_log2 > (uint32_t)kMaxSegLog2) continue;
        const uint32_t per_tile = (uint32_t)kBlockWaves << run.seg_log2;  // segments
        for (uint32_t i = threadIdx.x; i < run.count; i += blockDim.x) {
            const uint32_t t = run.first + i;
            tiles[run.dst + i] = Tile{run.fn, t * per_tile, run.seg_log2, run.part0 + t};
        }
    }
}

// Per-function second pass, one wave per function: the tile partials are summed
// by repeated 64-wide butterflies over aligned chunks (compacted in place), which
// is the pairwise tree over tile index; then mean and standard error in FP64.
extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_finalize(const LaunchDesc* __restrict__ Ld)
{
    const DevFn* fns = Ld->fns;
    const Fin* fins = Ld->fins;
    Partial* partials = Ld->partials;
    DevResult* results = Ld->results;
    const uint32_t n_fins = Ld->n_fins;
    const uint32_t n_fns = Ld->n_fns;
    const uint64_t n_partials = Ld->n_partials;
    uint32_t* counters = Ld->counters;
    const bool aborted =
        __hip_atomic_load(&counters[kCounterAborted], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t gw = blockIdx.x * kBlockWaves + threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * kBlockWaves;
    for (uint32_t f = gw; f < n_fins; f += nw) {
        const Fin fin = fins[f];
        if (!(fin.fn < n_fns && fin.n_tiles >= 1 && (uint64_t)fin.part0 + fin.n_tiles <= n_partials &&
              fin.res < n_fins)) {
            if (lane == 0) atomicAdd(&counters[kCounterBadRecords], 1u);
            continue;
        }
        CDevFn* fn = scalar_view(fns + fin.fn);
        const DevResult r = finalize_function(fn, partials + fin.part0, fin.n_tiles, lane, aborted ? -10 : 0);
        if (lane == 0) results[fin.res] = r;
    }
}

// Last kernel of a launch: copy the results and counters into pinned host
// memory, then publish the launch's sequence number (system scope, after every
// thread's copies are complete), which the host polls.
extern "C" __global__ __launch_bounds__(1024) void zmc_publish(const LaunchDesc* __restrict__ Ld)
{
    // 16-byte words: both areas are 16-byte aligned (256-aligned blocks, 48-byte results)
    static_assert(sizeof(DevResult) % sizeof(uint4) == 0, "result size");
    const uint64_t words = (uint64_t)Ld->n_fins * (sizeof(DevResult) / sizeof(uint4));
    const uint4* src = reinterpret_cast<const uint4*>(Ld->results);
    uint4* dst = reinterpret_cast<uint4*>(Ld->host_results);
    for (uint64_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x < (uint32_t)kNumCounters) Ld->host_counters[threadIdx.x] = Ld->counters[threadIdx.x];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(Ld->host_done, Ld->seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Records of a parameter grid, one thread per function (the paper's functional
// mode: one integrand form over a large parameter space), written straight into
// the request's function slots.
extern "C" __global__ __launch_bounds__(256) void zmc_pack_grid(GridSpec spec, DevFn* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= spec.n) return;
    mc_function f;
    grid_function(spec.base, spec.axes, spec.n_axes, i, &f);
    pack_function(f, spec.precision, &out[i]);
}

// Records of a validated function table already in device memory, one thread
// per function (the same packing code the host runs for tables).
extern "C" __global__ __launch_bounds__(256) void zmc_pack_table(const mc_function* __restrict__ fns, uint32_t n,
                                                                 int32_t precision, DevFn* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const mc_function f = fns[i];
    pack_function(f, precision, &out[i]);
}

// The points of samples [first, first + count) of one function, row-major
// (count x dim), from the batched kernels' generator and FP64 mapping: block
// q*d + j of sample i = 4q + s gives coordinate j from its word s.
extern "C" __global__ __launch_bounds__(256) void zmc_sample_points(const DevFn* __restrict__ fn_in, uint64_t first,
                                                                    uint64_t count, double* __restrict__ out)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    CDevFn* fn = scalar_view(fn_in);
    const uint64_t i = first + t;
    const uint64_t q = i >> 2;
    const uint32_t s = (uint32_t)(i & 3u);
    const uint32_t d = fn->dim;
    for (uint32_t j = 0; j < d && j < (uint32_t)kMaxDim; ++j) {
        const uint64_t b = q * d + j;
        uint32_t w[4];
        philox_block((uint32_t)b, (uint32_t)(b >> 32), fn->key0, fn->key1, w);
        out[t * d + j] = fma(fn->w[j], word_to_u64(w[s]), fn->lo[j]);
    }
}

// ---------------------------------------------------------------- plain FP64 path

// One thread per quad over a grid sized to the function's N, block sums in LDS,
// one partial per block; a second single-block kernel reduces the partials.
template <int FAM>
__device__ __forceinline__ void plain_quad(CDevFn* fn, uint64_t q, double f[4])
{
    const Eval64<FAM> ev{fn};
    ev.quad(fn->dim, fn->key0, fn->key1, q * (uint64_t)fn->dim, f);
}

extern "C" __global__ __launch_bounds__(256) void zmc_plain_fp64(const DevFn* __restrict__ fn_in,
                                                                 Partial* __restrict__ out)
{
    __shared__ double s1[256], s2[256];
    CDevFn* fn = scalar_view(fn_in);
    const uint64_t q = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t n_samples = fn->n_samples;
    double a = 0.0, b = 0.0;
    if (q < fn->n_quads) {
        double f[4];
        switch (fn->family) {
        case HARMONIC: plain_quad<HARMONIC>(fn, q, f); break;
        case ABS_LINEAR: plain_quad<ABS_LINEAR>(fn, q, f); break;
        case GAUSSIAN: plain_quad<GAUSSIAN>(fn, q, f); break;
        default: plain_quad<POLY_PRODUCT>(fn, q, f); break;
        }
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

extern "C" __global__ __launch_bounds__(256) void zmc_plain_reduce(const DevFn* __restrict__ fn_in,
                                                                   const Partial* __restrict__ parts,
                                                                   uint32_t n_parts, DevResult* __restrict__ res)
{
    CDevFn* fn = scalar_view(fn_in);
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

const void* plain_kernel_ptr() { return (const void*)zmc_plain_fp64; }
const void* stage_kernel_ptr() { return (const void*)zmc_stage; }
const void* publish_kernel_ptr() { return (const void*)zmc_publish; }
const void* pack_grid_kernel_ptr() { return (const void*)zmc_pack_grid; }
const void* pack_table_kernel_ptr() { return (const void*)zmc_pack_table; }
const void* sample_points_kernel_ptr() { return (const void*)zmc_sample_points; }
const void* finalize_kernel_ptr() { return (const void*)zmc_finalize; }
const void* plain_reduce_kernel_ptr() { return (const void*)zmc_plain_reduce; }

}  // namespace zmc
