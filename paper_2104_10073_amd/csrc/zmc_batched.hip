// zmc_batched.hip -- the persistent batched kernels for the four built-in
// families, FP32 and FP64 evaluation (the hot path: Philox samples, box mapping,
// integrand, compensated sums, segment and tile reductions).  The device code is
// in zmc_device_code.hpp; this file only instantiates it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "zmc_device_code.hpp"

namespace zmc {

// Family dispatch of the built-in kernels (a wave-uniform branch per tile).
template <bool F64>
struct BuiltinDispatch {
    template <int FAM>
    using Ev = typename std::conditional<F64, Eval64<FAM>, Eval32<FAM>>::type;
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

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp32(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<false>>(Ld, kKernelBuiltin32);
}

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp64(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<true>>(Ld, kKernelBuiltin64);
}

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

namespace {

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
__device__ uint32_t wait_ticket(const ResidentDesc* R, uint64_t t, bool leader)
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

}  // namespace

static_assert(sizeof(DevFn) == kWave * sizeof(uint4), "a record is one 16-byte word per lane of a wave");

// The resident kernel.  Every wait is bounded: a ticket's entry (idle_polls
// polls, after which the launch stops itself) and a record another workgroup
// is copying into the arena (ready_polls; a chunk whose record does not show up
// is counted with its function's result reporting MC_ERR_HIP).  The last
// workgroup to leave stores `epoch` into host_exit.
extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_resident(const ResidentDesc* __restrict__ R, uint32_t epoch)
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
                ok = f64 ? BuiltinDispatch<true>::run(fn, fn->kfam, t * per_tile, seg_log2, wave, lane, s_seg)
                         : BuiltinDispatch<false>::run(fn, fn->kfam, t * per_tile, seg_log2, wave, lane, s_seg);
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

const void* batched_kernel_ptr(bool fp64) { return fp64 ? (const void*)zmc_batched_fp64 : (const void*)zmc_batched_fp32; }
const void* resident_kernel_ptr() { return (const void*)zmc_resident; }

}  // namespace zmc
