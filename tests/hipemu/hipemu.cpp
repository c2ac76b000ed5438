// hipemu.cpp -- CPU emulation of the HIP runtime for the library's host code.
//
// TEST INFRASTRUCTURE ONLY.  The host runtime (zmc_host.hip) is compiled as
// ordinary C++ against include/hip/hip_runtime.h of this directory and linked
// with this file, so its admission, scheduling, launch building, completion,
// error and failure paths run on a machine without a GPU -- under
// AddressSanitizer and UndefinedBehaviorSanitizer in the tests.
//
// * "Device" memory is ordinary host memory.  Fresh allocations are filled
//   with 0xFF bytes (NaN doubles), so a result that reads memory no kernel
//   wrote is visibly wrong.
// * Streams execute in order and synchronously: a kernel runs when it is
//   launched (or, while a stream is capturing, when the graph is replayed).
// * Every kernel is replaced by a host routine with the kernel's effect on the
//   buffers the host reads back, following the kernels' contracts: the stage
//   kernel copies the staged launch and expands tile runs, the persistent
//   kernels write one partial per tile, finalize sums a function's partials
//   and compacts them in place, publish copies results and counters to the
//   host block and stores the done word.  Sample values are not Monte Carlo
//   estimates: every segment (batched path) or block (plain path) of n
//   samples of a function contributes n + t to the sum and 3 n + t^2 to the
//   sum of squares, with a tag t in [0, 4), a multiple of 2^-10 drawn from the
//   function's key and the unit index.  Every sum is exact in any order, the
//   spread is never zero, and a test knows each result in advance
//   (expected_batched / expected_plain below).  A tile of the FP32 kernel of a
//   function whose seed has bit 63 set contributes a constant instead (zero
//   spread), which the library's FP32 check sends to FP64.
// * The resident kernel runs in worker threads that start at its launch and
//   follow the kernel's protocol on the same words: tickets, the host's control
//   word with the stop bit, acknowledgements, the record copy into the arena
//   and its ready word, per-slot tile counts, the finalize by whichever worker
//   counts a run's last tile, done words, the exit word of the last worker to
//   leave, and the bounded waits (shortened to milliseconds).  A stream whose
//   resident launch is running finishes it before anything else enqueued on it.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "hipemu.hpp"
#include "zmc.h"
#include "zmc_device.hpp"
#include "zmc_pack.hpp"

using namespace zmc;

namespace {

std::mutex g_mu;
std::set<const void*> g_host_blocks;  // pinned blocks, to check frees

void* fresh(size_t n)
{
    const size_t sz = std::max<size_t>(256, (n + 255) & ~(size_t)255);
    void* p = std::aligned_alloc(256, sz);
    if (p) std::memset(p, 0xFF, sz);
    return p;
}

// ------------------------------------------------------------------ kernels

typedef void (*EmuFn)(void** args, dim3 grid);

struct EmuKernel {
    EmuFn fn;
    std::vector<size_t> arg_sizes;
};

double unit_tag(uint32_t key0, uint64_t unit)
{
    uint32_t h = key0 ^ (uint32_t)(unit * 0x9E3779B9ull) ^ (uint32_t)(unit >> 32) * 0x85EBCA6Bu;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (double)(h >> 20) / 1024.0;
}

bool constant_in_fp32(const DevFn& fn) { return (fn.key1 & 0x80000000u) != 0u; }

void k_stage(void** a, dim3)
{
    const uint8_t* src = *(const uint8_t**)a[0];
    uint8_t* dst = *(uint8_t**)a[1];
    const uint64_t cap = *(const uint64_t*)a[2];
    const uint32_t tile_cap = *(const uint32_t*)a[3];
    const DevFn* mirror = *(const DevFn**)a[4];
    DevFn* fns = *(DevFn**)a[5];
    const uint32_t n_fns = *(const uint32_t*)a[6];
    const LaunchDesc* hd = (const LaunchDesc*)src;
    const uint64_t bytes = std::min<uint64_t>(hd->stage_bytes, cap) / 16 * 16;
    Tile* tiles = const_cast<Tile*>(hd->tiles);
    const uint32_t n_runs = hd->n_runs;
    const TileRun* runs = (const TileRun*)(src + hd->runs_off);
    std::memmove(dst, src, bytes);
    for (uint32_t r = 0; r < n_runs; ++r) {
        const TileRun run = runs[r];
        if ((run.flags & kRunUploadRecord) != 0u && run.fn < n_fns) std::memcpy(fns + run.fn, mirror + run.fn, sizeof(DevFn));
        if (run.dst > tile_cap || run.count > tile_cap - run.dst || run.seg_log2 > (uint32_t)kMaxSegLog2) continue;
        const uint32_t per_tile = (uint32_t)kBlockWaves << run.seg_log2;
        for (uint32_t i = 0; i < run.count; ++i) {
            const uint32_t t = run.first + i;
            tiles[run.dst + i] = Tile{run.fn, t * per_tile, run.seg_log2, run.part0 + t};
        }
    }
}

void batched(const LaunchDesc* Ld, uint32_t kidx)
{
    const uint32_t n_tiles = Ld->tile_count[kidx];
    if (n_tiles == 0) return;
    uint32_t* counters = Ld->counters;
    if (*Ld->abort_word != 0u) {  // the real kernels stop at a tile fetch
        counters[kCounterAborted] |= 1u;
        return;
    }
    const Tile* tiles = Ld->tiles + Ld->tile_begin[kidx];
    for (uint32_t ti = 0; ti < n_tiles; ++ti) {
        counters[kCounterTiles + kidx]++;
        const Tile t = tiles[ti];
        bool ok = t.fn < Ld->n_fns && t.seg_log2 <= (uint32_t)kMaxSegLog2 && t.out < Ld->n_partials;
        const DevFn& fn = Ld->fns[ok ? t.fn : 0u];
        ok = ok && fn.dim >= 1 && fn.dim <= (uint32_t)kMaxDim && fn.kfam < (uint32_t)kNumFamilies;
        if (!ok) {
            counters[kCounterBadRecords]++;
            continue;
        }
        const uint32_t per_tile = (uint32_t)kBlockWaves << t.seg_log2;
        double s1 = 0.0, s2 = 0.0;
        for (uint32_t s = t.seg0; s < t.seg0 + per_tile && s < fn.n_segments; ++s) {
            const uint64_t first = (uint64_t)s * kSegSamples;
            const double n = (double)std::min<uint64_t>(kSegSamples, fn.n_samples - first);
            if (kidx == (uint32_t)kKernelBuiltin32 && constant_in_fp32(fn)) {
                s1 += n;
                s2 += n;
            } else {
                const double tag = unit_tag(fn.key0, s);
                s1 += n + tag;
                s2 += 3.0 * n + tag * tag;
            }
        }
        Ld->partials[t.out] = Partial{s1, s2};
    }
}

void k_batched32(void** a, dim3) { batched(*(const LaunchDesc**)a[0], kKernelBuiltin32); }
void k_batched64(void** a, dim3) { batched(*(const LaunchDesc**)a[0], kKernelBuiltin64); }

DevResult result_from(const DevFn& fn, double S1, double S2, int32_t status, uint32_t precision)
{
    const double dn = (double)fn.n_samples;
    double var = (S2 - S1 * S1 / dn) / (dn - 1.0);
    if (!(var > 0.0)) var = 0.0;
    DevResult r;
    r.mean = fn.volume * (S1 / dn);
    r.std_error = fn.volume * std::sqrt(var / dn);
    r.sum_f = S1;
    r.sum_f2 = S2;
    r.n = fn.n_samples;
    r.status = status;
    r.precision = precision;
    return r;
}

void k_finalize(void** a, dim3)
{
    const LaunchDesc* Ld = *(const LaunchDesc**)a[0];
    uint32_t* counters = Ld->counters;
    const bool aborted = counters[kCounterAborted] != 0u;
    for (uint32_t f = 0; f < Ld->n_fins; ++f) {
        const Fin fin = Ld->fins[f];
        if (!(fin.fn < Ld->n_fns && fin.n_tiles >= 1 && (uint64_t)fin.part0 + fin.n_tiles <= Ld->n_partials &&
              fin.res < Ld->n_fins)) {
            counters[kCounterBadRecords]++;
            continue;
        }
        const DevFn& fn = Ld->fns[fin.fn];
        Partial* P = Ld->partials + fin.part0;
        double g1 = 0.0, g2 = 0.0;
        for (uint32_t i = 0; i < fin.n_tiles; ++i) {
            g1 += P[i].s1;
            g2 += P[i].s2;
        }
        // the real pass compacts the partials in place: only P[0] keeps a meaning
        P[0] = Partial{g1, g2};
        for (uint32_t i = 1; i < fin.n_tiles; ++i) P[i] = Partial{NAN, NAN};
        Ld->results[fin.res] = result_from(fn, fn.scale1 * g1, fn.scale2 * g2, aborted ? -10 : 0, fn.precision);
    }
}

void k_publish(void** a, dim3)
{
    const LaunchDesc* Ld = *(const LaunchDesc**)a[0];
    std::memcpy(Ld->host_results, Ld->results, (size_t)Ld->n_fins * sizeof(DevResult));
    std::memcpy(Ld->host_counters, Ld->counters, kNumCounters * sizeof(uint32_t));
    __atomic_store_n(Ld->host_done, Ld->seq, __ATOMIC_RELEASE);
}

void k_pack_grid(void** a, dim3)
{
    const GridSpec spec = *(const GridSpec*)a[0];
    DevFn* out = *(DevFn**)a[1];
    for (uint64_t i = 0; i < spec.n; ++i) {
        mc_function f;
        grid_function(spec.base, spec.axes, spec.n_axes, i, &f);
        pack_function(f, spec.precision, &out[i]);
    }
}

void k_pack_table(void** a, dim3)
{
    const mc_function* fns = *(const mc_function**)a[0];
    const uint32_t n = *(const uint32_t*)a[1];
    const int32_t precision = *(const int32_t*)a[2];
    DevFn* out = *(DevFn**)a[3];
    for (uint32_t i = 0; i < n; ++i) pack_function(fns[i], precision, &out[i]);
}

void k_sample_points(void** a, dim3)
{
    const DevFn* fn = *(const DevFn**)a[0];
    const uint64_t count = *(const uint64_t*)a[2];
    double* out = *(double**)a[3];
    std::memset(out, 0, (size_t)count * fn->dim * sizeof(double));
}

void k_plain(void** a, dim3 grid)
{
    const DevFn* fn = *(const DevFn**)a[0];
    Partial* out = *(Partial**)a[1];
    for (uint32_t b = 0; b < grid.x; ++b) {
        const uint64_t first = (uint64_t)b * 1024u;
        const double n = first < fn->n_samples ? (double)std::min<uint64_t>(1024u, fn->n_samples - first) : 0.0;
        const double tag = unit_tag(fn->key0, b);
        out[b] = Partial{n + tag, 3.0 * n + tag * tag};
    }
}

void k_plain_reduce(void** a, dim3)
{
    const DevFn* fn = *(const DevFn**)a[0];
    const Partial* parts = *(const Partial**)a[1];
    const uint32_t n_parts = *(const uint32_t*)a[2];
    DevResult* res = *(DevResult**)a[3];
    double S1 = 0.0, S2 = 0.0;
    for (uint32_t i = 0; i < n_parts; ++i) {
        S1 += parts[i].s1;
        S2 += parts[i].s2;
    }
    *res = result_from(*fn, S1, S2, 0, 1u);
}

// One tile's partial, as the batched emulation computes it.
Partial tile_partial(const DevFn& fn, uint32_t seg0, uint32_t per_tile, bool fp32_kernel)
{
    double s1 = 0.0, s2 = 0.0;
    for (uint32_t s = seg0; s < seg0 + per_tile && s < fn.n_segments; ++s) {
        const uint64_t first = (uint64_t)s * kSegSamples;
        const double n = (double)std::min<uint64_t>(kSegSamples, fn.n_samples - first);
        if (fp32_kernel && constant_in_fp32(fn)) {
            s1 += n;
            s2 += n;
        } else {
            const double tag = unit_tag(fn.key0, s);
            s1 += n + tag;
            s2 += 3.0 * n + tag * tag;
        }
    }
    return Partial{s1, s2};
}

void short_sleep()
{
    struct timespec ts{0, 2000};
    nanosleep(&ts, nullptr);
}

uint64_t fetch_max_u64(uint64_t* p, uint64_t v)
{
    uint64_t old = __atomic_load_n(p, __ATOMIC_ACQUIRE);
    while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
    }
    return old;
}

// The resident kernel's loop, for one worker (a workgroup of the real launch).
void resident_worker(const ResidentDesc* R, uint32_t epoch, bool leader, uint32_t share)
{
    uint64_t* pos = R->pos;
    // the real waits poll every few microseconds; the emulation's polls are
    // slower, so the bounds are scaled down to keep them in milliseconds
    const uint32_t idle_polls = std::max<uint32_t>(R->idle_polls / 100, 16);
    const uint32_t ready_polls = std::max<uint32_t>(R->ready_polls / 1000, 16);
    for (;;) {
        const uint64_t t = __atomic_fetch_add(&pos[0], 1ull, __ATOMIC_RELAXED);
        bool take = false;
        for (uint32_t polls = 0;; ++polls) {
            uint64_t c = __atomic_load_n(&pos[1], __ATOMIC_ACQUIRE);
            if ((leader || (polls & 63u) == 63u) && (c & kCtlStop) == 0u && t >= c) {
                const uint64_t h = __atomic_load_n(R->host_ctl, __ATOMIC_ACQUIRE);
                if (h > c) {
                    const uint64_t old = fetch_max_u64(&pos[1], h);
                    c = old > h ? old : h;
                }
            }
            if ((c & kCtlStop) != 0u) {
                take = t < (c & ~kCtlStop);
                break;
            }
            if (t < c) {
                take = true;
                break;
            }
            if (polls + 1 >= idle_polls) {
                const uint64_t old = __atomic_fetch_or(&pos[1], kCtlStop, __ATOMIC_ACQ_REL);
                take = t < (old & ~kCtlStop);
                break;
            }
            short_sleep();
        }
        if (!take) break;
        const Chunk c = R->ring[t & R->ring_mask];
        __atomic_store_n(&R->ack[t & R->ring_mask], t + 1, __ATOMIC_RELEASE);
        const uint32_t fi = c.fn, rec = c.rec, token = c.token, count = c.count, first = c.first;
        const uint32_t seg_log2 = c.seg_flags & 0xFFu;
        const bool upload = ((c.seg_flags >> 8) & kChunkUpload) != 0u;
        if (!(fi < R->n_fns) || !(count >= 1u && count <= kChunkTiles)) {
            __atomic_fetch_add(R->bad_records, 1u, __ATOMIC_RELAXED);
            continue;
        }
        bool ok = rec < R->n_arena && seg_log2 <= (uint32_t)kMaxSegLog2 && first < c.n_tiles &&
                  count <= c.n_tiles - first && (uint64_t)c.part0 + c.n_tiles <= R->n_partials;
        if (ok && upload) {
            std::memcpy(R->arena + rec, R->mirror + fi, sizeof(DevFn));
            __atomic_store_n(&R->ready[rec], token, __ATOMIC_RELEASE);
        } else if (ok) {
            uint32_t n = 0;
            while (__atomic_load_n(&R->ready[rec], __ATOMIC_ACQUIRE) != token && n < ready_polls) {
                short_sleep();
                ++n;
            }
            ok = n < ready_polls;
        }
        const DevFn& fn = R->arena[ok ? rec : 0u];
        ok = ok && fn.dim >= 1 && fn.dim <= (uint32_t)kMaxDim && fn.kfam < (uint32_t)kNumFamilies;
        if (ok) {
            const uint32_t per_tile = (uint32_t)kBlockWaves << seg_log2;
            for (uint32_t i = 0; i < count; ++i) {
                const uint32_t tt = first + i;
                R->partials[c.part0 + tt] = tile_partial(fn, tt * per_tile, per_tile, fn.precision == 0u);
            }
        } else {
            __atomic_fetch_add(R->bad_records, 1u, __ATOMIC_RELAXED);
            __atomic_store_n(&R->slot_err[fi], token, __ATOMIC_RELAXED);
        }
        const uint32_t before = __atomic_fetch_add(&R->tiles_done[fi], count, __ATOMIC_ACQ_REL);
        if (before + count != c.n_tiles) continue;
        DevResult r{};
        const bool err = !ok || __atomic_load_n(&R->slot_err[fi], __ATOMIC_RELAXED) == token;
        if (!err) {
            Partial* P = R->partials + c.part0;
            double g1 = 0.0, g2 = 0.0;
            for (uint32_t i = 0; i < c.n_tiles; ++i) {
                g1 += P[i].s1;
                g2 += P[i].s2;
            }
            P[0] = Partial{g1, g2};
            for (uint32_t i = 1; i < c.n_tiles; ++i) P[i] = Partial{NAN, NAN};
            r = result_from(fn, fn.scale1 * g1, fn.scale2 * g2, 0, fn.precision);
        } else {
            r.status = -8;
        }
        R->host_results[fi] = r;
        __atomic_store_n(&R->tiles_done[fi], 0u, __ATOMIC_RELAXED);
        __atomic_store_n(&R->host_done[fi], token, __ATOMIC_RELEASE);
    }
    if (__atomic_sub_fetch(R->running, share, __ATOMIC_ACQ_REL) == 0u) {
        __atomic_store_n(R->host_exit + 1, __atomic_load_n(R->bad_records, __ATOMIC_RELAXED), __ATOMIC_RELAXED);
        __atomic_store_n(R->host_exit, epoch, __ATOMIC_RELEASE);
    }
}

void k_resident(void**, dim3) {}  // (started asynchronously by hipLaunchKernel)

const EmuKernel g_stage{k_stage, {8, 8, 8, 4, 8, 8, 4}};
const EmuKernel g_batched32{k_batched32, {8}};
const EmuKernel g_batched64{k_batched64, {8}};
const EmuKernel g_finalize{k_finalize, {8}};
const EmuKernel g_publish{k_publish, {8}};
const EmuKernel g_pack_grid{k_pack_grid, {sizeof(GridSpec), 8}};
const EmuKernel g_pack_table{k_pack_table, {8, 4, 4, 8}};
const EmuKernel g_sample_points{k_sample_points, {8, 8, 8, 8}};
const EmuKernel g_plain{k_plain, {8, 8}};
const EmuKernel g_plain_reduce{k_plain_reduce, {8, 8, 4, 8}};
const EmuKernel g_resident{k_resident, {8, 4}};

const EmuKernel* kernel_of(const void* p)
{
    for (const EmuKernel* k : {&g_stage, &g_batched32, &g_batched64, &g_finalize, &g_publish, &g_pack_grid,
                               &g_pack_table, &g_sample_points, &g_plain, &g_plain_reduce, &g_resident})
        if (p == (const void*)k) return k;
    return nullptr;
}

struct Launch {
    const EmuKernel* kernel;
    dim3 grid;
    std::vector<std::vector<uint8_t>> args;
};

void run(const Launch& l)
{
    std::vector<void*> ptrs;
    for (const auto& v : l.args) ptrs.push_back(const_cast<uint8_t*>(v.data()));
    l.kernel->fn(ptrs.data(), l.grid);
}

uint64_t g_launches = 0;
uint64_t g_api_calls = 0;  // calls into the emulated runtime

}  // namespace

struct ihipStream_t {
    bool capturing = false;
    std::vector<Launch> captured;
    std::vector<std::thread> workers;  // a running resident launch
    std::atomic<int> live{0};
};

namespace {

// In-order streams: whatever is enqueued after a resident launch waits for it.
void drain(hipStream_t s)
{
    if (!s) return;
    for (auto& w : s->workers) w.join();
    s->workers.clear();
}

}  // namespace
struct ihipEvent_t {
    int dummy = 0;
};
struct ihipGraph {
    std::vector<Launch> launches;
};
struct hipGraphExec {
    std::vector<Launch> launches;
};

// ------------------------------------------------------------------ the library's kernel table

namespace zmc {
const void* plain_kernel_ptr() { return &g_plain; }
const void* batched_kernel_ptr(bool fp64) { return fp64 ? &g_batched64 : &g_batched32; }
const void* finalize_kernel_ptr() { return &g_finalize; }
const void* stage_kernel_ptr() { return &g_stage; }
const void* publish_kernel_ptr() { return &g_publish; }
const void* pack_grid_kernel_ptr() { return &g_pack_grid; }
const void* pack_table_kernel_ptr() { return &g_pack_table; }
const void* sample_points_kernel_ptr() { return &g_sample_points; }
const void* plain_reduce_kernel_ptr() { return &g_plain_reduce; }
const void* resident_kernel_ptr() { return &g_resident; }
extern const char* const kRtcHeaderDevice;
extern const char* const kRtcHeaderCode;
const char* const kRtcHeaderDevice = "";
const char* const kRtcHeaderCode = "";
}  // namespace zmc

// ------------------------------------------------------------------ expected results

namespace hipemu {

mc_result expected_batched(const mc_function& f, bool fp64)
{
    DevFn d;
    pack_function(f, fp64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &d);
    double S1 = 0.0, S2 = 0.0;
    for (uint32_t s = 0; s < d.n_segments; ++s) {
        const double n = (double)std::min<uint64_t>(kSegSamples, d.n_samples - (uint64_t)s * kSegSamples);
        const double tag = unit_tag(d.key0, s);
        S1 += n + tag;
        S2 += 3.0 * n + tag * tag;
    }
    const DevResult r = result_from(d, d.scale1 * S1, d.scale2 * S2, 0, fp64 ? 1u : 0u);
    mc_result out;
    std::memcpy(&out, &r, sizeof out);
    return out;
}

mc_result expected_plain(const mc_function& f)
{
    DevFn d;
    pack_function(f, MC_PREC_FP64, &d);
    const uint32_t blocks = (uint32_t)((d.n_quads + 255) / 256);
    double S1 = 0.0, S2 = 0.0;
    for (uint32_t b = 0; b < blocks; ++b) {
        const uint64_t first = (uint64_t)b * 1024u;
        const double n = (double)std::min<uint64_t>(1024u, d.n_samples - first);
        const double tag = unit_tag(d.key0, b);
        S1 += n + tag;
        S2 += 3.0 * n + tag * tag;
    }
    const DevResult r = result_from(d, S1, S2, 0, 1u);
    mc_result out;
    std::memcpy(&out, &r, sizeof out);
    return out;
}

uint64_t kernel_launches() { return g_launches; }

uint64_t api_calls() { return g_api_calls; }

}  // namespace hipemu

// ------------------------------------------------------------------ runtime API

hipError_t hipGetDeviceCount(int* count)
{
    ++g_api_calls;
    *count = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int device) {
    ++g_api_calls; return device == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int)
{
    ++g_api_calls;
    std::memset(prop, 0, sizeof *prop);
    std::strcpy(prop->name, "emulated");
    std::strcpy(prop->gcnArchName, "gfx950:sramecc+:xnack-");
    prop->multiProcessorCount = 8;
    return hipSuccess;
}
hipError_t hipGetLastError() {
    ++g_api_calls; return hipSuccess; }
const char* hipGetErrorString(hipError_t e)
{
    switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorNotReady: return "hipErrorNotReady";
    default: return "hipError (emulated)";
    }
}

hipError_t hipMalloc(void** ptr, size_t bytes)
{
    ++g_api_calls;
    *ptr = fresh(bytes);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* ptr)
{
    ++g_api_calls;
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned)
{
    ++g_api_calls;
    *ptr = fresh(bytes);
    if (!*ptr) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lock(g_mu);
    g_host_blocks.insert(*ptr);
    return hipSuccess;
}
hipError_t hipHostFree(void* ptr)
{
    ++g_api_calls;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (ptr && g_host_blocks.erase(ptr) == 0) std::abort();  // not from hipHostMalloc
    }
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned)
{
    ++g_api_calls;
    *dev = host;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** dev, const void* symbol)
{
    ++g_api_calls;
    *dev = const_cast<void*>(symbol);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t stream)
{
    ++g_api_calls;
    if (stream && stream->capturing) return hipErrorNotSupported;  // the library captures kernels only
    drain(stream);
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t stream)
{
    ++g_api_calls;
    if (stream && stream->capturing) return hipErrorNotSupported;
    drain(stream);
    std::memset(dst, value, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned)
{
    ++g_api_calls;
    *stream = new ihipStream_t();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t stream)
{
    ++g_api_calls;
    drain(stream);
    delete stream;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t stream)
{
    ++g_api_calls;
    drain(stream);
    return hipSuccess;
}
hipError_t hipStreamQuery(hipStream_t stream)
{
    ++g_api_calls;
    return stream && stream->live.load() > 0 ? hipErrorNotReady : hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) {
    ++g_api_calls; return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t* event)
{
    ++g_api_calls;
    *event = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* event, unsigned) {
    ++g_api_calls; return hipEventCreate(event); }
hipError_t hipEventDestroy(hipEvent_t event)
{
    ++g_api_calls;
    delete event;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t stream)
{
    ++g_api_calls;
    if (stream && stream->capturing) return hipErrorNotSupported;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t) {
    ++g_api_calls; return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) {
    ++g_api_calls; return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t)
{
    ++g_api_calls;
    *ms = 0.001f;
    return hipSuccess;
}

hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* blocks, const void*, int, size_t)
{
    ++g_api_calls;
    *blocks = 8;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* kernel, dim3 grid, dim3, void** args, size_t, hipStream_t stream)
{
    ++g_api_calls;
    const EmuKernel* k = kernel_of(kernel);
    if (!k) return hipErrorInvalidValue;
    Launch l{k, grid, {}};
    for (size_t i = 0; i < k->arg_sizes.size(); ++i) {
        const uint8_t* p = (const uint8_t*)args[i];
        l.args.emplace_back(p, p + k->arg_sizes[i]);
    }
    if (stream && stream->capturing) {
        stream->captured.push_back(std::move(l));
        return hipSuccess;
    }
    ++g_launches;
    drain(stream);
    if (k == &g_resident) {
        if (!stream) return hipErrorInvalidValue;  // (the library gives it a stream of its own)
        const ResidentDesc* R = *(const ResidentDesc**)args[0];
        const uint32_t epoch = *(const uint32_t*)args[1];
        const uint32_t n = std::min<uint32_t>(grid.x, 4);
        stream->live.store((int)n);
        for (uint32_t w = 0; w < n; ++w) {
            const uint32_t share = grid.x / n + (w < grid.x % n ? 1u : 0u);
            stream->workers.emplace_back([R, epoch, w, share, stream] {
                resident_worker(R, epoch, w % 2 == 0, share);
                stream->live.fetch_sub(1);
            });
        }
        return hipSuccess;
    }
    run(l);
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode)
{
    ++g_api_calls;
    if (!stream || stream->capturing) return hipErrorInvalidValue;
    stream->capturing = true;
    stream->captured.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t* graph)
{
    ++g_api_calls;
    if (!stream || !stream->capturing) return hipErrorInvalidValue;
    stream->capturing = false;
    *graph = new ihipGraph{std::move(stream->captured)};
    stream->captured.clear();
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t*, char*, size_t)
{
    ++g_api_calls;
    *exec = new hipGraphExec{graph->launches};
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t)
{
    ++g_api_calls;
    for (const Launch& l : exec->launches) {
        ++g_launches;
        run(l);
    }
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph)
{
    ++g_api_calls;
    delete graph;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    ++g_api_calls;
    delete exec;
    return hipSuccess;
}

hipError_t hipModuleLoadData(hipModule_t*, const void*) {
    ++g_api_calls; return hipErrorNotSupported; }
hipError_t hipModuleGetFunction(hipFunction_t*, hipModule_t, const char*) {
    ++g_api_calls; return hipErrorNotSupported; }
hipError_t hipModuleUnload(hipModule_t) {
    ++g_api_calls; return hipSuccess; }
hipError_t hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(int*, hipFunction_t, int, size_t)
{
    ++g_api_calls;
    return hipErrorNotSupported;
}
hipError_t hipModuleLaunchKernel(hipFunction_t, unsigned, unsigned, unsigned, unsigned, unsigned, unsigned, unsigned,
                                 hipStream_t, void**, void**)
{
    ++g_api_calls;
    return hipErrorNotSupported;
}

hiprtcResult hiprtcCreateProgram(hiprtcProgram* prog, const char*, const char*, int, const char* const*,
                                 const char* const*)
{
    ++g_api_calls;
    *prog = nullptr;
    return HIPRTC_SUCCESS;
}
hiprtcResult hiprtcCompileProgram(hiprtcProgram, int, const char* const*) {
    ++g_api_calls; return HIPRTC_ERROR_COMPILATION; }
hiprtcResult hiprtcGetProgramLogSize(hiprtcProgram, size_t* size)
{
    ++g_api_calls;
    *size = 0;
    return HIPRTC_SUCCESS;
}
hiprtcResult hiprtcGetProgramLog(hiprtcProgram, char*) {
    ++g_api_calls; return HIPRTC_SUCCESS; }
hiprtcResult hiprtcGetCodeSize(hiprtcProgram, size_t* size)
{
    ++g_api_calls;
    *size = 0;
    return HIPRTC_ERROR_COMPILATION;
}
hiprtcResult hiprtcGetCode(hiprtcProgram, char*) {
    ++g_api_calls; return HIPRTC_ERROR_COMPILATION; }
hiprtcResult hiprtcDestroyProgram(hiprtcProgram* prog)
{
    ++g_api_calls;
    *prog = nullptr;
    return HIPRTC_SUCCESS;
}
const char* hiprtcGetErrorString(hiprtcResult) { return "run-time compilation is not available in the emulation"; }
